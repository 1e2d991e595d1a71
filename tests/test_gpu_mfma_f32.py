"""FP32 operands on the matrix cores (precision "fp32_mfma"): gridding and
degridding against the FP64 oracle at the FP32 tolerance of the vector path
(relative L2 <= 1e-5 per channel), for shared and per-baseline kernels, supports
up to 24, every tile edge and conjugate copies."""
import numpy as np
import pytest

import oracle as O
from synth import make_baseline_kernels
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


@pytest.mark.parametrize("W,OS,N,tile,conj,per_baseline", [
    (7, 8, 256, 0, False, False), (16, 16, 256, 0, True, False), (24, 8, 256, 32, False, False),
    (8, 4, 192, 48, False, False), (12, 16, 128, 16, False, False),
    (24, 8, 256, 0, True, True), (7, 8, 256, 0, False, True), (16, 4, 192, 48, False, True),
])
def test_fp32_mfma_matches_oracle(rts, W, OS, N, tile, conj, per_baseline):
    wl, freq, du = small_case(n_ant=40, channels=(0, 17, 31), N=N, W=W, OS=OS, weights="uniform",
                              flag_frac=0.1, offgrid_frac=0.02)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, conjugate=conj, tile=tile,
                        precision="fp32_mfma")
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS, conjugate=conj)
    rng = np.random.default_rng(W + N)
    Gin = (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))).astype(np.complex64)
    if per_baseline:
        tab = make_baseline_kernels(wl.uvw_m.shape[0], W, OS, seed=W)
        plan.set_baseline_kernels(torch.from_numpy(tab).cuda())
        Gref = O.grid_per_baseline(geom, wl.vis, wl.weights, tab)
        Mref = O.degrid_per_baseline(geom, Gin.astype(np.complex128), tab)
    else:
        Gref = O.grid(geom, wl.vis, wl.weights)
        Mref = O.degrid(geom, Gin.astype(np.complex128))
    G = plan.grid(vis, w).cpu().numpy()
    M = plan.degrid(torch.from_numpy(Gin).cuda()).cpu().numpy()
    assert np.all(M[~geom.valid] == 0)
    ge = [rel_l2(G[c], Gref[c]) for c in range(3)]
    me = [rel_l2(M[c], Mref[c]) for c in range(3)]
    print(f"fp32_mfma W={W} OS={OS} N={N} tile={tile} conj={conj} pb={per_baseline}: "
          f"grid {['%.1e' % e for e in ge]} degrid {['%.1e' % e for e in me]}")
    assert max(ge) <= RTOL_L2 and max(me) <= RTOL_L2


def test_fp32_mfma_fused_step_with_an_empty_model(rts):
    """The fused step of an fp32_mfma plan with G_in = 0 grids the visibilities."""
    wl, freq, du = small_case(n_ant=40, channels=(3, 29), N=256, W=7, OS=8, weights="uniform")
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 256, du, precision="fp32_mfma")
    gin = torch.zeros((2, 256, 256), dtype=torch.complex64, device="cuda")
    m, g, chi2 = plan.grid_degrid(vis, w, gin)
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, 256, du)
    Gref = O.grid(geom, wl.vis, wl.weights)
    for c in range(2):
        assert rel_l2(g.cpu().numpy()[c], Gref[c]) <= RTOL_L2
