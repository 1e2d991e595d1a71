"""BF16x3 matrix-core gridding against the FP64 oracle, error stated per channel.

Bound: every operand is split into two BF16 parts (16 significant bits; the
representation error is at most 2^-17 of the value) and the product keeps three
of the four cross terms, so each product is within about 3 * 2^-17 = 2.3e-5 of
exact, and sums of products of random sign average this down.  The test requires
a per-channel relative L2 error below 3e-5 and prints the measured values."""
import numpy as np
import pytest

import oracle as O
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


@pytest.mark.parametrize("W,OS,N,conj", [(7, 8, 256, False), (16, 16, 256, False), (16, 16, 512, True),
                                         (8, 4, 128, False)])
def test_bf16x3_grid_error_per_channel(rts, W, OS, N, conj):
    wl, freq, du = small_case(n_ant=48, channels=(0, 11, 31), N=N, W=W, OS=OS, weights="uniform",
                              flag_frac=0.1, offgrid_frac=0.02)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, conjugate=conj, precision="bf16x3")
    assert plan.info["tile"] == 16
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid(O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS, conjugate=conj), wl.vis, wl.weights)
    errs = [rel_l2(G[c], Gref[c]) for c in range(len(freq))]
    print(f"BF16x3 W={W} OS={OS} N={N} conj={conj}: per-channel rel L2 {['%.2e' % e for e in errs]}")
    assert max(errs) <= BF16X3_RTOL
    # an FP32 plan of the same inputs is far more accurate: the split is what limits it
    plan32 = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, conjugate=conj)
    G32 = plan32.grid(vis, w).cpu().numpy()
    assert max(rel_l2(G32[c], Gref[c]) for c in range(len(freq))) < min(errs)


def test_bf16x3_plan_degrid_uses_fp32(rts):
    wl, freq, du = small_case(n_ant=32, channels=(5,), N=256, W=16, OS=16)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 256, du, support=16, oversample=16, precision="bf16x3")
    rng = np.random.default_rng(0)
    Gin = (rng.standard_normal((1, 256, 256)) + 1j * rng.standard_normal((1, 256, 256))).astype(np.complex64)
    M = plan.degrid(torch.from_numpy(Gin).cuda()).cpu().numpy()
    Mref = O.degrid(O.Geometry(wl.uvw_m, freq, wl.weights, 256, du, 16, 16), Gin.astype(np.complex128))
    assert rel_l2(M, Mref) <= 1e-5
