"""The batched configuration's kernel path against the FP64 oracle, through the C ABI.

The batched workload (768 channels of 40 kHz, four time steps, per-channel flag
fractions U(0, 30%), 1024 x 1024 grids, W = 7, OS = 8) is reduced here to a few
channels spread over the band and a smaller array, keeping every property that
selects its code path: four-sample tracks (one segment each, vector loads of the
whole track), 64-cell tiles, uneven per-channel counts and 16-byte aligned device
buffers.  Also here: long tracks (the plan's per-track fallback beyond 64 samples),
shuffled baseline order, and repeatability.

Bar: FP32 results within relative L2 1e-5 of the oracle per channel (Eq. (1) and
its adjoint); integer results and the per-sample model exactly reproducible.
"""
import numpy as np
import pytest

import oracle as O
from tests.gpu_helpers import RTOL_L2, fit_cell, rel_l2, small_case, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CHANNELS = (0, 383, 767)      # band edges and centre of the 768-channel band


@pytest.fixture(scope="module")
def rts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_5575_amd as rts
    rts._lib.load()
    return rts


def batched_case(seed=0, n_ant=64, N=1024):
    wl, freq, du = small_case("batched", seed=seed, n_ant=n_ant, channels=CHANNELS, N=N)
    assert wl.n_time == 4
    return wl, freq, du


def gin_for(shape, seed):
    rng = np.random.default_rng(seed)
    return (0.1 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))).astype(np.complex64)


def check_all(geom, vis, weights, G, M, fused, gin):
    Gref = O.grid(geom, vis, weights)
    Mref = O.degrid(geom, gin.astype(np.complex128))
    Mo, Go, chi2o, _ = O.grid_degrid(geom, vis, weights, gin.astype(np.complex128))
    Mf, Gf, chi2 = (x.cpu().numpy() for x in fused)
    assert np.all(M[~geom.valid] == 0) and np.all(Mf[~geom.valid] == 0)
    for c in range(G.shape[0]):
        assert rel_l2(G[c], Gref[c]) <= RTOL_L2, f"grid channel {c}"
        assert rel_l2(M[c], Mref[c]) <= RTOL_L2, f"degrid channel {c}"
        assert rel_l2(Gf[c], Go[c]) <= RTOL_L2, f"fused grid channel {c}"
        assert rel_l2(Mf[c], Mo[c]) <= RTOL_L2, f"fused model channel {c}"
    assert abs(float(chi2) - chi2o) <= RTOL_L2 * abs(chi2o)


@pytest.mark.parametrize("schedule", ["tiles", "persistent"])
def test_batched_path_matches_oracle(rts, schedule):
    """Four-sample tracks on 64-cell tiles with per-channel flag fractions:
    grid, degrid and the fused step against the oracle, both launch schedules."""
    wl, freq, du = batched_case()
    N = 1024
    flagged = (wl.weights == 0).mean(axis=(1, 2))
    assert flagged.max() - flagged.min() > 0.02          # uneven per-channel counts
    uvw, vis, w = to_dev(torch, wl)
    for t in (uvw, vis, w):
        assert t.data_ptr() % 16 == 0
    plan = rts.GridPlan(uvw, freq, w, N, du, schedule=schedule)
    info = plan.info
    assert info["tile"] == 64 and info["seg_max"] == 4
    assert info["n_segments"] == len(freq) * wl.n_base    # every track is one segment
    gin_np = gin_for((len(freq), N, N), 1)
    gin = torch.from_numpy(gin_np).cuda()
    G = plan.grid(vis, w).cpu().numpy()
    M = plan.degrid(gin).cpu().numpy()
    fused = plan.grid_degrid(vis, w, gin)
    torch.cuda.synchronize()
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du)
    assert info["n_valid"] == int(geom.valid.sum())
    check_all(geom, wl.vis, wl.weights, G, M, fused, gin_np)


def test_batched_cadence_graph_with_new_flags(rts):
    """The captured cadence step (re-plan + fused pass) replayed over new
    visibilities and new per-channel flag fractions on the same array."""
    wl0, freq, du = batched_case(seed=0)
    N = 1024
    uvw, vis, w = to_dev(torch, wl0)
    gin_np = gin_for((len(freq), N, N), 2)
    gin = torch.from_numpy(gin_np).cuda()
    model = torch.empty_like(vis)
    gout = torch.empty((len(freq), N, N), dtype=torch.complex64, device="cuda")
    chi2 = torch.empty((), dtype=torch.float64, device="cuda")
    plan = rts.GridPlan(uvw, freq, w, N, du)
    graph = plan.cadence_graph(uvw, vis, w, gin, model, gout, chi2)
    for seed in (3, 4, 0):
        wl, _, _ = batched_case(seed=seed)
        wl.uvw_m = wl0.uvw_m
        _, v2, w2 = to_dev(torch, wl)
        vis.copy_(v2)
        w.copy_(w2)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert plan.info["n_dropped"] == 0
        geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du)
        Mo, Go, chi2o, _ = O.grid_degrid(geom, wl.vis, wl.weights, gin_np.astype(np.complex128))
        g, m = gout.cpu().numpy(), model.cpu().numpy()
        for c in range(len(freq)):
            assert rel_l2(g[c], Go[c]) <= RTOL_L2, (seed, c)
            assert rel_l2(m[c], Mo[c]) <= RTOL_L2, (seed, c)
        assert abs(chi2.item() - chi2o) <= RTOL_L2 * chi2o
    graph.close()


def test_long_tracks_use_per_track_plan_path(rts):
    """Tracks of 80 samples (beyond the 64 lanes of the plan's lane path) are
    segmented and sorted by the per-track plan kernels; results match the oracle."""
    from synth import mwa
    cfg = mwa.Config("t80", 24, 80, 2, 140e6, 15e6, 256, 7, 8, n_sources=1, cadence_s=400.0)
    wl = mwa.make_workload(cfg, seed=2)
    freq = wl.freq_hz
    N = 256
    du = fit_cell(wl.uvw_m, freq, N, 7)
    rng = np.random.default_rng(9)
    wl.weights = rng.uniform(0.5, 1.5, wl.weights.shape).astype(np.float32)
    wl.weights[rng.random(wl.weights.shape) < 0.15] = 0
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, tile=32)
    info = plan.info
    assert info["n_segments"] > len(freq) * wl.n_base      # tracks longer than a segment
    gin_np = gin_for((len(freq), N, N), 5)
    gin = torch.from_numpy(gin_np).cuda()
    G = plan.grid(vis, w).cpu().numpy()
    M = plan.degrid(gin).cpu().numpy()
    fused = plan.grid_degrid(vis, w, gin)
    torch.cuda.synchronize()
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du)
    check_all(geom, wl.vis, wl.weights, G, M, fused, gin_np)


def test_shuffled_baseline_order(rts):
    """Section 5: a scatter must not depend on the order in which visibilities
    arrive.  Permuting the baselines (uvw rows with their visibilities and weights)
    permutes the model the same way, bit for bit (each sample's model is one
    fixed-order sum), and leaves the grid unchanged to rounding: the tile sums are
    taken in FP64 and rounded once to FP32, so two orders differ by at most one
    FP32 ulp per cell."""
    wl, freq, du = batched_case(seed=1)
    N = 1024
    perm = np.random.default_rng(7).permutation(wl.n_base)
    uvw, vis, w = to_dev(torch, wl)
    up = torch.from_numpy(np.ascontiguousarray(wl.uvw_m[perm])).cuda()
    vp = torch.from_numpy(np.ascontiguousarray(wl.vis[:, perm])).cuda()
    wp = torch.from_numpy(np.ascontiguousarray(wl.weights[:, perm])).cuda()
    gin = torch.from_numpy(gin_for((len(freq), N, N), 3)).cuda()
    p1 = rts.GridPlan(uvw, freq, w, N, du)
    p2 = rts.GridPlan(up, freq, wp, N, du)
    M1, G1, c1 = (x.cpu().numpy() for x in p1.grid_degrid(vis, w, gin))
    M2, G2, c2 = (x.cpu().numpy() for x in p2.grid_degrid(vp, wp, gin))
    assert np.array_equal(M1[:, perm], M2)
    ulp = np.spacing(np.maximum(np.abs(G1.view(np.float32)), np.abs(G2.view(np.float32))))
    assert np.all(np.abs(G1.view(np.float32) - G2.view(np.float32)) <= ulp)
    assert abs(float(c1) - float(c2)) <= 1e-12 * abs(float(c1))


def test_repeated_calls(rts):
    """Two identical calls: the snapped coordinates, the valid mask, the plan's
    counts and every model value are identical bit for bit; grid cells differ by
    at most one FP32 ulp (FP64 tile sums whose order of addition may differ,
    rounded once)."""
    wl, freq, du = batched_case(seed=2)
    N = 1024
    uvw, vis, w = to_dev(torch, wl)
    gin = torch.from_numpy(gin_for((len(freq), N, N), 4)).cuda()
    c1 = rts.compute_coords(uvw, freq, w, N, du).cpu().numpy()
    c2 = rts.compute_coords(uvw, freq, w, N, du).cpu().numpy()
    assert np.array_equal(c1, c2)
    plan = rts.GridPlan(uvw, freq, w, N, du)
    i1 = plan.info
    plan.update(uvw, w)
    assert plan.info == i1
    assert torch.equal(plan.valid_mask(), plan.valid_mask())
    a = [x.cpu().numpy() for x in plan.grid_degrid(vis, w, gin)]
    b = [x.cpu().numpy() for x in plan.grid_degrid(vis, w, gin)]
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(plan.degrid(gin).cpu().numpy(), plan.degrid(gin).cpu().numpy())
    ga, gb = a[1].view(np.float32), b[1].view(np.float32)
    assert np.all(np.abs(ga - gb) <= np.spacing(np.maximum(np.abs(ga), np.abs(gb))))
