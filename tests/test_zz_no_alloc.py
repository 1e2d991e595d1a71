"""rts_grid_degrid_noalloc (plan + fused residual step with the library's static
workspace, for callers that cannot allocate device memory) against the existing
entry points rts_grid_plan + rts_grid_degrid, through the C ABI: two calls in a
row on one device, the second with a smaller input, each to the FP32 bar
(relative L2 1e-5 per channel against the existing path and the FP64 oracle),
the model identical to the existing path's bit for bit where both sum in the
same order.  Also: a problem too large for the static workspace is refused with
RTS_E_INVALID and a message."""
import ctypes

import numpy as np
import pytest

import oracle as O
from tests.gpu_helpers import RTOL_L2, rel_l2, small_case, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_5575_amd as rts
    rts._lib.load()
    return rts


def _case(name, n_ant, channels, N, seed):
    wl, freq, du = small_case(name, seed=seed, n_ant=n_ant, channels=channels, N=N, weights="uniform",
                              flag_frac=0.1)
    rng = np.random.default_rng(seed + 50)
    gin = (0.1 * (rng.standard_normal((len(freq), N, N)) + 1j * rng.standard_normal((len(freq), N, N)))
           ).astype(np.complex64)
    return wl, freq, du, gin


def _run_both(rts, wl, freq, du, gin_np, N):
    uvw, vis, w = to_dev(torch, wl)
    gin = torch.from_numpy(gin_np).cuda()
    plan = rts.GridPlan(uvw, freq, w, N, du)
    M1, G1, c1 = plan.grid_degrid(vis, w, gin)
    model = torch.empty_like(vis)
    chi2 = torch.empty((), dtype=torch.float64, device="cuda")
    M2, G2, c2 = rts.grid_degrid_noalloc(uvw, freq, w, vis, gin, N, du, model_out=model, chi2_out=chi2)
    torch.cuda.synchronize()
    plan.close()
    return [x.cpu().numpy() for x in (M1, G1, c1)], [x.cpu().numpy() for x in (M2, G2, c2)]


def test_noalloc_matches_plan_path_twice(rts):
    runs = [("batched", 48, (0, 400, 767), 512, 3), ("single_cadence", 24, (5, 20), 256, 4)]
    for name, n_ant, chans, N, seed in runs:           # second call: fewer samples, channels, cells
        wl, freq, du, gin = _case(name, n_ant, chans, N, seed)
        (M1, G1, c1), (M2, G2, c2) = _run_both(rts, wl, freq, du, gin, N)
        geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du)
        Mo, Go, chi2o, _ = O.grid_degrid(geom, wl.vis, wl.weights, gin.astype(np.complex128))
        for c in range(len(freq)):
            assert rel_l2(G2[c], G1[c]) <= RTOL_L2, (name, c)
            assert rel_l2(M2[c], M1[c]) <= RTOL_L2, (name, c)
            assert rel_l2(G2[c], Go[c]) <= RTOL_L2, (name, c)
            assert rel_l2(M2[c], Mo[c]) <= RTOL_L2, (name, c)
        # each sample's model is one sum in a fixed order in both paths
        assert np.array_equal(M1, M2), name
        assert np.all(M2[~geom.valid] == 0)
        assert abs(float(c2) - float(c1)) <= 1e-9 * abs(float(c1)), name
        assert abs(float(c2) - chi2o) <= RTOL_L2 * chi2o, name


def test_noalloc_refuses_oversized_problem(rts):
    lib = rts._lib.load()
    C, B, T, N = 64, 130816, 8, 1024            # 67M samples: beyond the static workspace
    p = rts.make_params(N, 1.0, 7, 8, C, B, T)
    fr = (ctypes.c_double * C)(*([150e6] * C))
    dummy = torch.empty(16, dtype=torch.float64, device="cuda")
    ptr = ctypes.c_void_p(dummy.data_ptr())
    st = lib.rts_grid_degrid_noalloc(ctypes.byref(p), ptr, ctypes.cast(fr, ctypes.c_void_p), ptr, ptr, ptr, None,
                                     ctypes.c_void_p(dummy.data_ptr() + 2 ** 40), None, None)
    assert st == rts._lib.RTS_E_INVALID
    assert b"workspace" in lib.rts_last_error()
