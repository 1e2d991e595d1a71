"""The fused residual step (rts_grid_degrid) of matrix-core plans against the
FP64 oracle: M = degrid(G_in); r = V - M on the valid samples; G_out = grid(w r);
chi2 = sum w |r|^2 (oracle.grid_degrid; with per-baseline kernels, the same
composition of oracle.degrid_per_baseline and oracle.grid_per_baseline).

Bounds: gridding and degridding each meet relative L2 tol per channel (3e-5
for BF16x3, 1e-5 for FP32 operands).  The residual carries the model's error
into the gridding pass: |dr| <= |dM|, so G_out meets (1 + |M| / |r|) tol, and
chi2 = |r|_w^2 meets 2 |dr|_w / |r|_w + tol^2, both used with a margin of 2."""
import numpy as np
import pytest

import oracle as O
from synth import make_baseline_kernels
from tests.gpu_helpers import RTOL_L2, rel_l2, small_case, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = {"bf16x3": 3e-5, "fp32_mfma": RTOL_L2}


@pytest.fixture(scope="module")
def rts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_5575_amd as rts
    rts._lib.load()
    return rts


def reference(geom, vis, w, Gin, tab=None):
    """The fused step composed from the oracle's gridding and degridding."""
    if tab is None:
        return O.grid_degrid(geom, vis, w, Gin)
    M = O.degrid_per_baseline(geom, Gin, tab)
    r = np.where(geom.valid, np.asarray(vis, np.complex128) - M, 0.0)
    G = O.grid_per_baseline(geom, r, w, tab)
    chi2 = float(np.sum(np.where(geom.valid, np.asarray(w, np.float64) * np.abs(r) ** 2, 0.0)))
    return M, G, chi2, r


def check(M, G, chi2, ref, valid, tol, label):
    Mo, Go, chi2o, ro = ref
    assert np.all(M[~valid] == 0)
    C = Go.shape[0]
    me = [rel_l2(M[c], Mo[c]) for c in range(C)]
    ge = [rel_l2(G[c], Go[c]) for c in range(C)]
    amp = [1.0 + np.linalg.norm(Mo[c]) / max(np.linalg.norm(ro[c]), 1e-300) for c in range(C)]
    ce = abs(chi2 - chi2o) / chi2o
    print(f"{label}: model {['%.1e' % e for e in me]} grid {['%.1e' % e for e in ge]} chi2 {ce:.1e}")
    assert max(me) <= tol
    assert all(ge[c] <= 2 * amp[c] * tol for c in range(C))
    assert ce <= 2 * (2 * max(amp) * tol + tol * tol)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32_mfma"])
@pytest.mark.parametrize("W,OS,N,tile,per_baseline", [
    (7, 8, 256, 0, False), (24, 8, 256, 32, False), (16, 4, 192, 48, False), (12, 16, 128, 16, False),
    (24, 8, 256, 0, True), (20, 8, 192, 48, True),
])
def test_mfma_fused_step_matches_oracle(rts, prec, W, OS, N, tile, per_baseline):
    wl, freq, du = small_case(seed=W, n_ant=40, channels=(0, 17, 31), N=N, W=W, OS=OS, weights="uniform",
                              flag_frac=0.1, offgrid_frac=0.02)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, tile=tile, precision=prec)
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS)
    rng = np.random.default_rng(W + N)
    Gin = (0.1 * (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N)))).astype(np.complex64)
    tab = None
    if per_baseline:
        tab = make_baseline_kernels(wl.uvw_m.shape[0], W, OS, seed=W + 1)
        plan.set_baseline_kernels(torch.from_numpy(tab).cuda())
    m, g, c2 = plan.grid_degrid(vis, w, torch.from_numpy(Gin).cuda())
    ref = reference(geom, wl.vis, wl.weights, Gin.astype(np.complex128), tab)
    check(m.cpu().numpy(), g.cpu().numpy(), c2.item(), ref, geom.valid, TOL[prec],
          f"{prec} W={W} OS={OS} N={N} tile={tile} pb={per_baseline}")


@pytest.mark.parametrize("prec", ["bf16x3", "fp32_mfma"])
def test_mfma_fused_step_agrees_with_separate_calls(rts, prec):
    """The fused step equals degrid, then grid of the residual, through the same
    plan, to the rounding of the order of FP32 atomic additions."""
    W, OS, N = 24, 8, 256
    wl, freq, du = small_case(seed=5, n_ant=40, channels=(2, 30), N=N, W=W, OS=OS, weights="uniform",
                              flag_frac=0.2)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, precision=prec)
    rng = np.random.default_rng(1)
    gin = torch.from_numpy((0.1 * (rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))))
                           .astype(np.complex64)).cuda()
    m, g, c2 = plan.grid_degrid(vis, w, gin)
    m2 = plan.degrid(gin)
    r = (vis - m2).masked_fill_(~plan.valid_mask(), 0)
    g2 = plan.grid(r, w)
    for c in range(2):
        assert rel_l2(m[c].cpu().numpy(), m2[c].cpu().numpy()) <= 1e-6
    for c in range(2):
        assert rel_l2(g[c].cpu().numpy(), g2[c].cpu().numpy()) <= 1e-6
    c2ref = float((w.double() * (r.abs().double() ** 2)).sum())
    assert abs(c2.item() - c2ref) <= 1e-6 * c2ref


def test_mfma_fused_step_needs_model_out(rts):
    wl, freq, du = small_case(seed=6, n_ant=40, channels=(0,), N=256, W=24, OS=8)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 256, du, support=24, oversample=8, precision="bf16x3")
    gin = torch.zeros((1, 256, 256), dtype=torch.complex64, device="cuda")
    with pytest.raises(rts.RtsError):
        plan.grid_degrid(vis, w, gin, model_out=False)
    m, g, c2 = plan.grid_degrid(vis, w, gin)           # the library still works afterwards
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, 256, du, 24, 8)
    assert rel_l2(g[0].cpu().numpy(), O.grid(geom, wl.vis, wl.weights)[0]) <= TOL["bf16x3"]
    assert torch.count_nonzero(m) == 0


@pytest.mark.parametrize("prec,per_baseline", [("fp32_mfma", False), ("bf16x3", True)])
def test_mfma_cadence_graph_replays_new_data(rts, prec, per_baseline):
    """A cadence graph of a matrix-core plan (W=24): replays on new samples and
    flags, with eager work between them, each against the oracle."""
    W, OS, N = 24, 8, 256

    def cadence(seed):
        return small_case(seed=seed, n_ant=40, channels=(0, 13, 31), N=N, W=W, OS=OS, weights="uniform",
                          flag_frac=0.1)

    wl0, freq, du = cadence(0)
    uvw, vis, w = to_dev(torch, wl0)
    rng = np.random.default_rng(0)
    gin_np = (0.1 * (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N)))).astype(np.complex64)
    gin = torch.from_numpy(gin_np).cuda()
    model = torch.empty_like(vis)
    gout = torch.empty((3, N, N), dtype=torch.complex64, device="cuda")
    chi2 = torch.empty((), dtype=torch.float64, device="cuda")
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, precision=prec)
    tab = None
    if per_baseline:
        tab = make_baseline_kernels(wl0.uvw_m.shape[0], W, OS, seed=3)
        plan.set_baseline_kernels(torch.from_numpy(tab).cuda())
    graph = plan.cadence_graph(uvw, vis, w, gin, model, gout, chi2)
    for seed in (1, 2, 0):
        wl, _, _ = cadence(seed)
        wl.uvw_m = wl0.uvw_m
        u2, v2, w2 = to_dev(torch, wl)
        uvw.copy_(u2); vis.copy_(v2); w.copy_(w2)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert plan.info["n_dropped"] == 0
        geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS)
        ref = reference(geom, wl.vis, wl.weights, gin_np.astype(np.complex128), tab)
        check(model.cpu().numpy(), gout.cpu().numpy(), chi2.item(), ref, geom.valid, TOL[prec],
              f"graph {prec} pb={per_baseline} seed={seed}")
    graph.close()


def test_mfma_cadence_graph_needs_model_out(rts):
    wl, freq, du = small_case(seed=7, n_ant=40, channels=(0,), N=256, W=24, OS=8)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 256, du, support=24, oversample=8, precision="fp32_mfma")
    gin = torch.zeros((1, 256, 256), dtype=torch.complex64, device="cuda")
    gout = torch.empty_like(gin)
    with pytest.raises(rts.RtsError):
        plan.cadence_graph(uvw, vis, w, gin, None, gout, None)


def test_graph_lifetime_guards(rts):
    """While a cadence graph of a plan is alive, adding or removing per-baseline
    tables and destroying the plan are refused; replacing the tables is allowed
    and the next replay uses them."""
    W, OS, N = 24, 8, 256
    wl, freq, du = small_case(seed=8, n_ant=40, channels=(0, 9), N=N, W=W, OS=OS, weights="uniform")
    uvw, vis, w = to_dev(torch, wl)
    B = wl.uvw_m.shape[0]
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, precision="bf16x3")
    tab1 = make_baseline_kernels(B, W, OS, seed=1)
    tab2 = make_baseline_kernels(B, W, OS, seed=2)
    plan.set_baseline_kernels(torch.from_numpy(tab1).cuda())
    gin = torch.zeros((2, N, N), dtype=torch.complex64, device="cuda")
    model = torch.empty_like(vis)
    gout = torch.empty_like(gin)
    graph = plan.cadence_graph(uvw, vis, w, gin, model, gout, None)
    with pytest.raises(rts.RtsError):
        plan.set_baseline_kernels(None)
    with pytest.raises(rts.RtsError):
        plan.close()
    plan.set_baseline_kernels(torch.from_numpy(tab2).cuda())     # same address: allowed
    graph.launch()
    torch.cuda.synchronize()
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS)
    Gref = O.grid_per_baseline(geom, wl.vis, wl.weights, tab2)
    g = gout.cpu().numpy()
    for c in range(2):
        assert rel_l2(g[c], Gref[c]) <= TOL["bf16x3"]
    graph.close()
    plan.set_baseline_kernels(None)                               # no live graph: allowed
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fused_step_refuses_a_model_that_aliases_an_input(rts, prec):
    """model_out may not share memory with vis, weights or the grids (the model is
    written while they are still read); the refusal leaves the outputs alone."""
    wl, freq, du = small_case(seed=9, n_ant=40, channels=(0, 1), N=256)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 256, du, precision=prec)
    gin = torch.zeros((2, 256, 256), dtype=torch.complex64, device="cuda")
    vis0 = vis.clone()
    with pytest.raises(rts.RtsError):
        plan.grid_degrid(vis, w, gin, model_out=vis)
    assert torch.equal(vis, vis0)
    gview = gin.view(-1)[:vis.numel()].view(vis.shape)
    with pytest.raises(rts.RtsError):
        plan.grid_degrid(vis, w, gin, model_out=gview)
    m, g, c2 = plan.grid_degrid(vis, w, gin)              # distinct buffers: accepted
    assert torch.count_nonzero(m) == 0


def test_mfma_maximum_sizes(rts):
    """The largest grid and support of the matrix-core path (N = 8192, W = 24,
    OS = 16, 16,384 tiles of 64 cells on one channel): gridding and the fused step
    against the oracle."""
    N, W, OS = 8192, 24, 16
    wl, freq, du = small_case(seed=11, n_ant=40, channels=(17,), N=N, W=W, OS=OS, weights="uniform",
                              flag_frac=0.1)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, precision="bf16x3")
    assert plan.info["tile"] == 64
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS)
    G = plan.grid(vis, w).cpu().numpy()
    assert rel_l2(G[0], O.grid(geom, wl.vis, wl.weights)[0]) <= TOL["bf16x3"]
    del G
    rng = np.random.default_rng(3)
    Gin = (0.1 * (rng.standard_normal((1, N, N)) + 1j * rng.standard_normal((1, N, N)))).astype(np.complex64)
    m, g, c2 = plan.grid_degrid(vis, w, torch.from_numpy(Gin).cuda())
    ref = O.grid_degrid(geom, wl.vis, wl.weights, Gin.astype(np.complex128))
    check(m.cpu().numpy(), g.cpu().numpy(), c2.item(), ref, geom.valid, TOL["bf16x3"], "max sizes bf16x3")


@pytest.mark.parametrize("T", [1, 3, 5, 9, 16])
@pytest.mark.parametrize("prec", ["bf16x3", "fp32_mfma"])
def test_mfma_fused_step_ragged_time_axis(rts, T, prec):
    """Track lengths below, between and above the per-segment sample limit, with
    20% of the samples flagged, through the matrix-core fused step (W = 16)."""
    from synth import mwa
    from tests.gpu_helpers import fit_cell
    W, OS, N = 16, 8, 256
    cfg = mwa.Config("t%d" % T, 30, T, 3, 140e6, 10e6, N, W, OS, n_sources=2)
    wl = mwa.make_workload(cfg, seed=T)
    freq = wl.freq_hz
    du = fit_cell(wl.uvw_m, freq, N, W)
    rng = np.random.default_rng(T)
    wl.weights = rng.uniform(0.5, 1.5, wl.weights.shape).astype(np.float32)
    wl.weights[rng.random(wl.weights.shape) < 0.2] = 0
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, tile=32, precision=prec)
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS)
    Gin = (0.1 * (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N)))).astype(np.complex64)
    m, g, c2 = plan.grid_degrid(vis, w, torch.from_numpy(Gin).cuda())
    ref = O.grid_degrid(geom, wl.vis, wl.weights, Gin.astype(np.complex128))
    check(m.cpu().numpy(), g.cpu().numpy(), c2.item(), ref, geom.valid, TOL[prec], f"ragged T={T} {prec}")


@pytest.mark.parametrize("prec", ["bf16x3", "fp32_mfma"])
def test_mfma_fused_step_everything_flagged(rts, prec):
    """No valid sample: zero model, zero grid, chi2 exactly 0."""
    wl, freq, du = small_case(seed=12, n_ant=20, channels=(0, 5), N=128, W=24, OS=8)
    wl.weights[:] = 0
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 128, du, support=24, oversample=8, precision=prec)
    assert plan.info["n_valid"] == 0
    gin = torch.ones((2, 128, 128), dtype=torch.complex64, device="cuda")
    m, g, c2 = plan.grid_degrid(vis, w, gin)
    assert torch.all(m == 0) and torch.all(g == 0) and c2.item() == 0.0
