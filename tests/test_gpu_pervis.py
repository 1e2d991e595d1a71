"""Per-visibility (per-baseline) kernels on the matrix-core path against the FP64
oracle (oracle.grid_per_baseline / degrid_per_baseline, pinned in
tests/test_oracle_pins.py), and supports beyond 16 with the shared kernel.

Bound: the BF16x3 bound of tests/test_gpu_mfma.py (per-channel relative L2 3e-5);
the per-baseline tables enter as FP32 values, split hi + lo like the shared
table."""
import numpy as np
import pytest

import oracle as O
from synth import make_baseline_kernels
from tests.gpu_helpers import rel_l2, small_case, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
BF16X3_RTOL = 3e-5


@pytest.fixture(scope="module")
def rts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_5575_amd as rts
    rts._lib.load()
    return rts


def _case(W, OS, N, conj, seed=0, channels=(0, 17, 31)):
    wl, freq, du = small_case(seed=seed, n_ant=40, channels=channels, N=N, W=W, OS=OS, weights="uniform",
                              flag_frac=0.1, offgrid_frac=0.02)
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS, conjugate=conj)
    return wl, freq, du, geom


@pytest.mark.parametrize("W,OS,N,tile,conj", [(24, 8, 256, 0, False), (24, 8, 256, 32, True), (7, 8, 256, 0, False),
                                              (16, 4, 192, 48, False), (24, 16, 128, 64, True)])
def test_per_baseline_grid_and_degrid(rts, W, OS, N, tile, conj):
    wl, freq, du, geom = _case(W, OS, N, conj)
    B = wl.uvw_m.shape[0]
    tab = make_baseline_kernels(B, W, OS, seed=W + OS)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, conjugate=conj, tile=tile,
                        precision="bf16x3")
    plan.set_baseline_kernels(torch.from_numpy(tab).cuda())
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid_per_baseline(geom, wl.vis, wl.weights, tab)
    rng = np.random.default_rng(W)
    Gin = (rng.standard_normal((len(freq), N, N)) + 1j * rng.standard_normal((len(freq), N, N))).astype(np.complex64)
    M = plan.degrid(torch.from_numpy(Gin).cuda()).cpu().numpy()
    Mref = O.degrid_per_baseline(geom, Gin.astype(np.complex128), tab)
    assert np.all(M[~geom.valid] == 0)
    ge = [rel_l2(G[c], Gref[c]) for c in range(len(freq))]
    me = [rel_l2(M[c], Mref[c]) for c in range(len(freq))]
    print(f"per-baseline W={W} OS={OS} N={N} conj={conj}: grid {['%.2e' % e for e in ge]} "
          f"degrid {['%.2e' % e for e in me]}")
    assert max(ge) <= BF16X3_RTOL and max(me) <= BF16X3_RTOL


def test_per_baseline_kernels_can_be_replaced_and_removed(rts):
    """New tables replace the old ones in place; None restores the shared kernel."""
    W, OS, N = 24, 8, 256
    wl, freq, du, geom = _case(W, OS, N, False, seed=1, channels=(3, 29))
    B = wl.uvw_m.shape[0]
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, precision="bf16x3")
    for seed in (1, 2):
        tab = make_baseline_kernels(B, W, OS, seed=seed)
        plan.set_baseline_kernels(torch.from_numpy(tab).cuda())
        G = plan.grid(vis, w).cpu().numpy()
        Gref = O.grid_per_baseline(geom, wl.vis, wl.weights, tab)
        assert max(rel_l2(G[c], Gref[c]) for c in range(2)) <= BF16X3_RTOL
    plan.set_baseline_kernels(None)
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid(geom, wl.vis, wl.weights)
    assert max(rel_l2(G[c], Gref[c]) for c in range(2)) <= BF16X3_RTOL


def test_shared_table_given_per_baseline_matches_shared_path(rts):
    """Every baseline given the plan's own table: the per-baseline path agrees with
    the shared-kernel path within the BF16x3 bound (the split inputs differ: FP32
    table values against FP64 kernel values)."""
    W, OS, N = 7, 8, 256
    wl, freq, du, geom = _case(W, OS, N, False, seed=2)
    B = wl.uvw_m.shape[0]
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, precision="bf16x3")
    G0 = plan.grid(vis, w).cpu().numpy()
    tab = np.ascontiguousarray(np.broadcast_to(plan.table(), (B, OS, W))).astype(np.float32)
    plan.set_baseline_kernels(torch.from_numpy(tab).cuda())
    G1 = plan.grid(vis, w).cpu().numpy()
    for c in range(G0.shape[0]):
        assert rel_l2(G1[c], G0[c]) <= 2 * BF16X3_RTOL


def test_fp32_plan_refuses_per_baseline_kernels(rts):
    wl, freq, du, geom = _case(7, 8, 256, False, seed=3, channels=(0,))
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 256, du)
    tab = torch.ones((wl.uvw_m.shape[0], 8, 7), dtype=torch.float32, device="cuda")
    with pytest.raises(rts.RtsError):
        plan.set_baseline_kernels(tab)


@pytest.mark.parametrize("W,OS,N,tile", [(24, 8, 256, 0), (24, 32, 128, 64), (20, 8, 192, 48)])
def test_shared_kernel_supports_beyond_16(rts, W, OS, N, tile):
    """Supports 17-24 with the shared Kaiser-Bessel kernel (padded LDS tables)."""
    wl, freq, du, geom = _case(W, OS, N, False, seed=4)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, tile=tile, precision="bf16x3")
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid(geom, wl.vis, wl.weights)
    rng = np.random.default_rng(OS)
    Gin = (rng.standard_normal((len(freq), N, N)) + 1j * rng.standard_normal((len(freq), N, N))).astype(np.complex64)
    M = plan.degrid(torch.from_numpy(Gin).cuda()).cpu().numpy()
    Mref = O.degrid(geom, Gin.astype(np.complex128))
    for c in range(len(freq)):
        assert rel_l2(G[c], Gref[c]) <= BF16X3_RTOL
        assert rel_l2(M[c], Mref[c]) <= BF16X3_RTOL
