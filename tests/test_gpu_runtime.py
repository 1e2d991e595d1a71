"""Cadence graph (captured re-plan + fused pass replayed per cadence) and the
tile autotuner, through the C ABI."""
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


def cadence(seed, flag_frac=0.1):
    return small_case(seed=seed, n_ant=40, channels=(0, 13, 31), N=256, weights="uniform", flag_frac=flag_frac)


def test_cadence_graph_replays_new_data(rts):
    wl0, freq, du = cadence(0)
    uvw, vis, w = to_dev(torch, wl0)
    rng = np.random.default_rng(0)
    gin_np = (0.1 * (rng.standard_normal((3, 256, 256)) + 1j * rng.standard_normal((3, 256, 256)))).astype(np.complex64)
    gin = torch.from_numpy(gin_np).cuda()
    model = torch.empty_like(vis)
    gout = torch.empty((3, 256, 256), dtype=torch.complex64, device="cuda")
    chi2 = torch.empty((), dtype=torch.float64, device="cuda")
    plan = rts.GridPlan(uvw, freq, w, 256, du)
    graph = plan.cadence_graph(uvw, vis, w, gin, model, gout, chi2)
    for seed in (1, 2, 0, 3):
        wl, _, _ = cadence(seed)
        wl.uvw_m = wl0.uvw_m                        # same array geometry, new samples and flags
        u2, v2, w2 = to_dev(torch, wl)
        uvw.copy_(u2); vis.copy_(v2); w.copy_(w2)   # eager work between replays
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert plan.info["n_dropped"] == 0
        geom = O.Geometry(wl.uvw_m, freq, wl.weights, 256, du)
        Mo, Go, chi2o, _ = O.grid_degrid(geom, wl.vis, wl.weights, gin_np.astype(np.complex128))
        g, m = gout.cpu().numpy(), model.cpu().numpy()
        for c in range(3):
            assert rel_l2(g[c], Go[c]) <= RTOL_L2, (seed, c)
            assert rel_l2(m[c], Mo[c]) <= RTOL_L2, (seed, c)
        assert abs(chi2.item() - chi2o) <= RTOL_L2 * chi2o
    graph.close()


def test_cadence_graph_matches_eager_bitwise_inputs(rts):
    """Replaying the graph on unchanged inputs reproduces the eager outputs."""
    wl, freq, du = cadence(4)
    uvw, vis, w = to_dev(torch, wl)
    gin = torch.zeros((3, 256, 256), dtype=torch.complex64, device="cuda")
    plan = rts.GridPlan(uvw, freq, w, 256, du)
    m_e, g_e, c_e = plan.grid_degrid(vis, w, gin)
    model = torch.empty_like(vis)
    gout = torch.empty_like(g_e)
    chi2 = torch.empty((), dtype=torch.float64, device="cuda")
    graph = plan.cadence_graph(uvw, vis, w, gin, model, gout, chi2)
    for _ in range(3):
        graph.launch()
        torch.cuda.synchronize()
        assert rel_l2(gout.cpu().numpy(), g_e.cpu().numpy()) <= 1e-6
        assert torch.equal(model, m_e)              # degridding has a fixed order
        assert abs(chi2.item() - c_e.item()) <= 1e-9 * c_e.item()


def test_autotune_picks_a_legal_tile(rts):
    wl, freq, du = cadence(5)
    uvw, vis, w = to_dev(torch, wl)
    gin = torch.zeros((3, 256, 256), dtype=torch.complex64, device="cuda")
    best, times = rts.autotune_tile(uvw, freq, w, vis, gin, 256, du)
    assert best in (16, 32, 64) and best in times
    assert set(times) == {16, 32, 64}
    assert times[best] == min(times.values())
    best2, _ = rts.autotune_tile(uvw, freq, w, vis, gin, 256, du, measure=False)   # cached
    assert best2 == best
    plan = rts.GridPlan(uvw, freq, w, 256, du, tile=best)
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid(O.Geometry(wl.uvw_m, freq, wl.weights, 256, du), wl.vis, wl.weights)
    for c in range(3):
        assert rel_l2(G[c], Gref[c]) <= RTOL_L2
