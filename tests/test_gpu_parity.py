"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar: integer outputs (snapped coordinates, validity) bit-exact; FP32 grids, models
and chi-squared within relative L2 1e-5 of the oracle, per channel.
"""
import numpy as np
import pytest

import oracle as O
from tests.gpu_helpers import RTOL_L2, fit_cell, rel_l2, small_case, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_5575_amd as rts
    rts._lib.load()
    return rts


def run_all(rts, wl, freq, du, N, W, OS, tile=0, conjugate=False, seed=0, schedule="auto"):
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, tile=tile, conjugate=conjugate,
                        schedule=schedule)
    G = plan.grid(vis, w)
    rng = np.random.default_rng(seed)
    Gin_np = (0.1 * (rng.standard_normal(G.shape) + 1j * rng.standard_normal(G.shape))).astype(np.complex64)
    Gin = torch.from_numpy(Gin_np).cuda()
    M = plan.degrid(Gin) if not conjugate else None
    fused = plan.grid_degrid(vis, w, Gin) if not conjugate else None
    torch.cuda.synchronize()
    return plan, G.cpu().numpy(), Gin_np, (M.cpu().numpy() if M is not None else None), fused


def check_against_oracle(wl, freq, du, N, W, OS, G, Gin, M, fused, conjugate=False):
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS, conjugate=conjugate)
    Gref = O.grid(geom, wl.vis, wl.weights)
    for c in range(len(freq)):
        assert rel_l2(G[c], Gref[c]) <= RTOL_L2, f"grid channel {c}"
    if conjugate:
        return
    Mref = O.degrid(geom, Gin.astype(np.complex128))
    assert np.all(M[~geom.valid] == 0)
    for c in range(len(freq)):
        assert rel_l2(M[c], Mref[c]) <= RTOL_L2, f"degrid channel {c}"
    Mf, Gf, chi2 = fused
    Mo, Go, chi2o, _ = O.grid_degrid(geom, wl.vis, wl.weights, Gin.astype(np.complex128))
    Mf, Gf = Mf.cpu().numpy(), Gf.cpu().numpy()
    for c in range(len(freq)):
        assert rel_l2(Mf[c], Mo[c]) <= RTOL_L2, f"fused model channel {c}"
        assert rel_l2(Gf[c], Go[c]) <= RTOL_L2, f"fused grid channel {c}"
    assert abs(chi2.item() - chi2o) <= RTOL_L2 * abs(chi2o)


def test_library_is_native_hip(rts):
    import os
    assert os.path.exists(rts.library_path())
    maps = open("/proc/self/maps").read()
    assert "librtsgrid.so" in maps


def test_coords_bit_exact(rts):
    for (W, OS, N) in [(7, 8, 256), (8, 8, 512), (16, 16, 512), (5, 3, 128)]:
        wl, freq, du = small_case(n_ant=48, channels=(0, 7, 31), N=N, W=W, OS=OS, flag_frac=0.1,
                                  offgrid_frac=0.05)
        uvw, vis, w = to_dev(torch, wl)
        out = rts.compute_coords(uvw, freq, w, N, du, W, OS).cpu().numpy()
        xs, ys, fin = O.snapped(wl.uvw_m, freq, N, du, OS)
        valid = O.coords(wl.uvw_m, freq, wl.weights, N, du, W, OS)[4]
        assert np.array_equal(out[..., 0], np.where(fin, xs, 0))
        assert np.array_equal(out[..., 1], np.where(fin, ys, 0))
        assert np.array_equal(out[..., 2].astype(bool), valid)


def test_kernel_table_matches_oracle(rts):
    for W, OS in [(7, 8), (8, 8), (16, 16), (4, 64)]:
        wl, freq, du = small_case(n_ant=8, channels=(0,), N=128, W=W, OS=OS)
        uvw, vis, w = to_dev(torch, wl)
        plan = rts.GridPlan(uvw, freq, w, 128, du, support=W, oversample=OS)
        tab = plan.table()
        ref = O.table(W, OS, O.default_beta(W))
        assert np.all(np.abs(tab - ref) <= 1.2e-7 * np.maximum(np.abs(ref), 1e-30) + 1e-45)


def test_plan_counts(rts):
    wl, freq, du = small_case(n_ant=40, channels=(0, 31), N=256, flag_frac=0.2, offgrid_frac=0.1)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 256, du, tile=32)
    info = plan.info
    valid = O.coords(wl.uvw_m, freq, wl.weights, 256, du, 7, 8)[4]
    assert info["n_samples"] == valid.size
    assert info["n_valid"] == int(valid.sum())
    assert info["n_flagged"] == int((wl.weights == 0).sum())
    assert info["n_offgrid"] == valid.size - int(valid.sum()) - int((wl.weights == 0).sum())
    assert info["n_segments"] >= wl.vis.shape[0] * wl.vis.shape[1]
    assert info["n_listings"] >= info["n_segments"]


@pytest.mark.parametrize("W,OS,N,tile", [(7, 8, 256, 0), (7, 8, 256, 16), (7, 8, 512, 32), (8, 8, 256, 32),
                                         (5, 4, 128, 16), (12, 8, 256, 32), (16, 16, 256, 64)])
def test_grid_degrid_fused_parity(rts, W, OS, N, tile):
    wl, freq, du = small_case(n_ant=40, channels=(0, 13, 31), N=N, W=W, OS=OS, weights="uniform",
                              flag_frac=0.15, offgrid_frac=0.03)
    plan, G, Gin, M, fused = run_all(rts, wl, freq, du, N, W, OS, tile=tile)
    check_against_oracle(wl, freq, du, N, W, OS, G, Gin, M, fused)


@pytest.mark.parametrize("W,OS,N,tile,channels", [(7, 8, 256, 0, (0, 13, 31)), (7, 8, 512, 32, (0, 13, 31)),
                                                  (12, 8, 256, 16, (3, 9)), (16, 16, 256, 64, (5,)),
                                                  (7, 8, 64, 32, (2,))])
def test_persistent_schedule_parity(rts, W, OS, N, tile, channels):
    """The persistent longest-first launch gives the oracle's results, also with
    fewer tiles than queues (N=64, tile 32: four tiles, eight queues)."""
    wl, freq, du = small_case(n_ant=40, channels=channels, N=N, W=W, OS=OS, weights="uniform",
                              flag_frac=0.15, offgrid_frac=0.03)
    plan, G, Gin, M, fused = run_all(rts, wl, freq, du, N, W, OS, tile=tile, schedule="persistent")
    check_against_oracle(wl, freq, du, N, W, OS, G, Gin, M, fused)


def test_persistent_schedule_after_update(rts):
    """rts_plan_update rebuilds the longest-first order with the work list."""
    wl, freq, du = small_case(n_ant=40, channels=(0, 13, 31), N=256, weights="uniform", flag_frac=0.1)
    wl2, _, _ = small_case(seed=5, n_ant=40, channels=(0, 13, 31), N=256, weights="uniform", flag_frac=0.1)
    uvw, vis, w = to_dev(torch, wl)
    uvw2, vis2, w2 = to_dev(torch, wl2)
    plan = rts.GridPlan(uvw, freq, w, 256, du, schedule="persistent")
    ref = rts.GridPlan(uvw2, freq, w2, 256, du, schedule="tiles")
    for _ in range(2):
        plan.update(uvw2, w2)
        G = plan.grid(vis2, w2).cpu().numpy()
        Gt = ref.grid(vis2, w2).cpu().numpy()
        assert rel_l2(G, Gt) <= 1e-6
    geom = O.Geometry(wl2.uvw_m, freq, wl2.weights, 256, du)
    Gref = O.grid(geom, wl2.vis, wl2.weights)
    for c in range(3):
        assert rel_l2(G[c], Gref[c]) <= RTOL_L2


@pytest.mark.parametrize("T", [1, 3, 12])
def test_ragged_time_axis(rts, T):
    """Track lengths below, between and above the per-segment sample limit."""
    from synth import mwa
    cfg = mwa.Config("t%d" % T, 30, T, 3, 140e6, 10e6, 256, 7, 8, n_sources=2)
    wl = mwa.make_workload(cfg, seed=T)
    freq = wl.freq_hz
    du = fit_cell(wl.uvw_m, freq, 256, 7)
    rng = np.random.default_rng(T)
    wl.weights = rng.uniform(0.5, 1.5, wl.weights.shape).astype(np.float32)
    wl.weights[rng.random(wl.weights.shape) < 0.2] = 0
    plan, G, Gin, M, fused = run_all(rts, wl, freq, du, 256, 7, 8, tile=32)
    check_against_oracle(wl, freq, du, 256, 7, 8, G, Gin, M, fused)


def test_conjugate_grid_parity_and_hermitian(rts):
    wl, freq, du = small_case(n_ant=40, channels=(0, 31), N=256)
    plan, G, Gin, M, fused = run_all(rts, wl, freq, du, 256, 7, 8, conjugate=True)
    check_against_oracle(wl, freq, du, 256, 7, 8, G, Gin, M, fused, conjugate=True)
    idx = (256 - np.arange(256)) % 256
    for c in range(2):
        mirror = G[c][idx][:, idx]
        assert rel_l2(mirror, np.conj(G[c])) <= 1e-6


@pytest.mark.parametrize("W,OS,N,tile", [(8, 8, 256, 0), (16, 16, 256, 0), (12, 8, 256, 16)])
def test_conjugate_grid_even_and_wide_supports(rts, W, OS, N, tile):
    """Conjugate gridding with even and wide supports (64-cell and 16-cell tiles):
    oracle parity and Hermitian symmetry about the grid centre."""
    wl, freq, du = small_case(n_ant=40, channels=(0, 31), N=N, W=W, OS=OS, weights="uniform", flag_frac=0.1)
    plan, G, Gin, M, fused = run_all(rts, wl, freq, du, N, W, OS, tile=tile, conjugate=True)
    check_against_oracle(wl, freq, du, N, W, OS, G, Gin, M, fused, conjugate=True)
    idx = (N - np.arange(N)) % N
    for c in range(2):
        assert rel_l2(G[c][idx][:, idx], np.conj(G[c])) <= 1e-6


def test_everything_flagged_gives_zeros(rts):
    wl, freq, du = small_case(n_ant=20, channels=(0, 5), N=128)
    wl.weights[:] = 0
    plan, G, Gin, M, fused = run_all(rts, wl, freq, du, 128, 7, 8)
    assert plan.info["n_valid"] == 0
    assert np.all(G == 0) and np.all(M == 0)
    Mf, Gf, chi2 = fused
    assert torch.all(Gf == 0) and torch.all(Mf == 0) and chi2.item() == 0.0


def test_literal_half_lambda_cell_drops_offgrid(rts):
    from synth import make_workload
    wl = make_workload("tiny_literal", seed=0)
    plan, G, Gin, M, fused = run_all(rts, wl, wl.freq_hz, wl.cell_lambda, 256, 7, 8)
    geom = O.Geometry(wl.uvw_m, wl.freq_hz, wl.weights, 256, wl.cell_lambda)
    assert plan.info["n_valid"] == int(geom.valid.sum())
    check_against_oracle(wl, wl.freq_hz, wl.cell_lambda, 256, 7, 8, G, Gin, M, fused)


def test_tiny_config(rts):
    from synth import make_workload
    wl = make_workload("tiny", seed=0)
    plan, G, Gin, M, fused = run_all(rts, wl, wl.freq_hz, wl.cell_lambda, 256, 7, 8)
    check_against_oracle(wl, wl.freq_hz, wl.cell_lambda, 256, 7, 8, G, Gin, M, fused)


def test_repeat_calls_are_stable(rts):
    """Two identical calls agree to rounding (the LDS accumulation order may vary)."""
    wl, freq, du = small_case(n_ant=40, channels=(0, 31), N=256)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 256, du)
    a = plan.grid(vis, w).cpu().numpy()
    b = plan.grid(vis, w).cpu().numpy()
    assert rel_l2(a, b) <= 1e-6


def test_plan_update_matches_fresh_plan(rts):
    """Re-planning in place for a new cadence gives the fresh plan's results."""
    wl, freq, du = small_case(n_ant=40, channels=(0, 13, 31), N=256, weights="uniform", flag_frac=0.1)
    wl2, _, _ = small_case(seed=5, n_ant=40, channels=(0, 13, 31), N=256, weights="uniform", flag_frac=0.1)
    uvw, vis, w = to_dev(torch, wl)
    uvw2, vis2, w2 = to_dev(torch, wl2)
    plan = rts.GridPlan(uvw, freq, w, 256, du)
    plan.update(uvw2, w2)
    G = plan.grid(vis2, w2).cpu().numpy()
    info = plan.info
    assert info["n_dropped"] == 0
    geom = O.Geometry(wl2.uvw_m, freq, wl2.weights, 256, du)
    Gref = O.grid(geom, wl2.vis, wl2.weights)
    for c in range(3):
        assert rel_l2(G[c], Gref[c]) <= RTOL_L2
    assert info["n_valid"] == int(geom.valid.sum())


def test_plan_update_overflow_is_reported_not_fatal(rts):
    """A cadence that needs more work-list entries than the plan holds drops the
    excess, reports it, and stays in bounds."""
    wl, freq, du = small_case(n_ant=60, channels=(0, 31), N=256)
    uvw, vis, w = to_dev(torch, wl)
    w0 = torch.zeros_like(w)
    # every sample flagged: one listing per track; 16-cell tiles later double that
    plan = rts.GridPlan(uvw, freq, w0, 256, du, tile=16)
    cap_listings = plan.info["n_listings"]
    plan.update(uvw, w)
    G = plan.grid(vis, w)
    torch.cuda.synchronize()
    info = plan.info
    assert info["n_listings"] > cap_listings
    assert info["n_dropped"] > 0
    assert torch.isfinite(torch.view_as_real(G)).all()


@pytest.mark.parametrize("cadence_s,T", [(4000.0, 8), (20000.0, 16)])
def test_fast_moving_tracks_split_into_segments(rts, cadence_s, T):
    """Tracks that cross several cells per step are cut into many segments (the
    plan's multi-segment path); results still match the oracle."""
    from synth import mwa
    cfg = mwa.Config("fast", 36, T, 2, 140e6, 15e6, 256, 7, 8, n_sources=1, cadence_s=cadence_s)
    wl = mwa.make_workload(cfg, seed=3)
    freq = wl.freq_hz
    du = fit_cell(wl.uvw_m, freq, 256, 7)
    rng = np.random.default_rng(1)
    wl.weights = rng.uniform(0.5, 1.5, wl.weights.shape).astype(np.float32)
    wl.weights[rng.random(wl.weights.shape) < 0.1] = 0
    plan, G, Gin, M, fused = run_all(rts, wl, freq, du, 256, 7, 8, tile=32)
    info = plan.info
    assert info["n_segments"] > 2 * wl.vis.shape[0] * wl.vis.shape[1]   # most tracks split
    check_against_oracle(wl, freq, du, 256, 7, 8, G, Gin, M, fused)


def test_maximum_sizes(rts):
    """The largest grid, support and oversampling the library accepts (N = 8192,
    W = 16, OS = 64) on one channel: grid, degrid and the fused step against the
    oracle."""
    N, W, OS = 8192, 16, 64
    wl, freq, du = small_case(n_ant=40, channels=(17,), N=N, W=W, OS=OS, weights="uniform", flag_frac=0.1)
    plan, G, Gin, M, fused = run_all(rts, wl, freq, du, N, W, OS)
    assert plan.info["tile"] == 64
    check_against_oracle(wl, freq, du, N, W, OS, G, Gin, M, fused)
