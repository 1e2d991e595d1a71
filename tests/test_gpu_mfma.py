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
    assert plan.info["tile"] % 16 == 0
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid(O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS, conjugate=conj), wl.vis, wl.weights)
    errs = [rel_l2(G[c], Gref[c]) for c in range(len(freq))]
    print(f"BF16x3 W={W} OS={OS} N={N} conj={conj}: per-channel rel L2 {['%.2e' % e for e in errs]}")
    assert max(errs) <= BF16X3_RTOL
    # an FP32 plan of the same inputs is far more accurate: the split is what limits it
    plan32 = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, conjugate=conj)
    G32 = plan32.grid(vis, w).cpu().numpy()
    assert max(rel_l2(G32[c], Gref[c]) for c in range(len(freq))) < min(errs)


@pytest.mark.parametrize("W,OS,N,conj", [(7, 8, 256, False), (16, 16, 256, False), (8, 4, 128, False),
                                         (5, 8, 64, False), (7, 8, 256, True), (16, 16, 256, True)])
def test_bf16x3_degrid_error_per_channel(rts, W, OS, N, conj):
    """Degridding as H = Av G_tile on the matrix cores, per-region partial values
    summed into the model: error per channel against the FP64 oracle (with the
    conjugate copies listed, degridding reads the +uv samples only)."""
    wl, freq, du = small_case(n_ant=48, channels=(0, 11, 31), N=N, W=W, OS=OS, flag_frac=0.1, offgrid_frac=0.02)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, conjugate=conj, precision="bf16x3")
    rng = np.random.default_rng(W)
    Gin = (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))).astype(np.complex64)
    M = plan.degrid(torch.from_numpy(Gin).cuda()).cpu().numpy()
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS, conjugate=conj)
    Mref = O.degrid(geom, Gin.astype(np.complex128))
    assert np.all(M[~geom.valid] == 0)
    errs = [rel_l2(M[c], Mref[c]) for c in range(len(freq))]
    print(f"BF16x3 degrid W={W} OS={OS} N={N} conj={conj}: per-channel rel L2 {['%.2e' % e for e in errs]}")
    assert max(errs) <= BF16X3_RTOL


@pytest.mark.parametrize("tile", [16, 32, 48, 64])
def test_bf16x3_every_tile_edge(rts, tile):
    """Tiles of one, two and three subtiles per edge: a wave covers one subtile
    (tile 16, 48) or a pair of them (tile 32, 64); grid and degrid both."""
    N, W, OS = 192, 7, 8
    wl, freq, du = small_case(n_ant=40, channels=(0, 20), N=N, W=W, OS=OS, flag_frac=0.1, offgrid_frac=0.02)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, tile=tile, precision="bf16x3")
    assert plan.info["tile"] == tile
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS)
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid(geom, wl.vis, wl.weights)
    rng = np.random.default_rng(tile)
    Gin = (rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))).astype(np.complex64)
    M = plan.degrid(torch.from_numpy(Gin).cuda()).cpu().numpy()
    Mref = O.degrid(geom, Gin.astype(np.complex128))
    for c in range(2):
        assert rel_l2(G[c], Gref[c]) <= BF16X3_RTOL
        assert rel_l2(M[c], Mref[c]) <= BF16X3_RTOL


@pytest.mark.parametrize("tile", [48, 64])
def test_bf16x3_widest_tables(rts, tile):
    """The largest support and oversampling (W=16, OS=64): the zero-padded kernel
    tables in LDS are at their largest."""
    N, W, OS = 192, 16, 64
    wl, freq, du = small_case(n_ant=40, channels=(5, 25), N=N, W=W, OS=OS, flag_frac=0.1, offgrid_frac=0.02)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, tile=tile, precision="bf16x3")
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS)
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid(geom, wl.vis, wl.weights)
    rng = np.random.default_rng(tile + 1)
    Gin = (rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))).astype(np.complex64)
    M = plan.degrid(torch.from_numpy(Gin).cuda()).cpu().numpy()
    Mref = O.degrid(geom, Gin.astype(np.complex128))
    for c in range(2):
        assert rel_l2(G[c], Gref[c]) <= BF16X3_RTOL
        assert rel_l2(M[c], Mref[c]) <= BF16X3_RTOL


def test_bf16x3_degrid_is_adjoint_of_bf16x3_grid(rts):
    """<grid(V), G> = <V, degrid(G)> (unit weights) within the BF16x3 error."""
    N = 256
    wl, freq, du = small_case(n_ant=40, channels=(3, 17), N=N, W=7, OS=8)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, precision="bf16x3")
    rng = np.random.default_rng(1)
    Gin = (rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))).astype(np.complex64)
    G = plan.grid(vis, w).cpu().numpy().astype(np.complex128)
    M = plan.degrid(torch.from_numpy(Gin).cuda()).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(G.ravel(), Gin.astype(np.complex128).ravel())
    rhs = np.vdot(wl.vis.astype(np.complex128).ravel(), M.ravel())
    assert abs(lhs - rhs) <= 1e-4 * max(abs(lhs), 1.0)


def test_bf16x3_in_key_order_with_many_tiles(rts):
    """More (channel, tile) pairs than 64 per CU: the kernels walk the tiles in
    key order instead of longest first (the small cases above take the
    longest-first order); both grid and degrid against the oracle."""
    N, W, OS = 2048, 7, 8
    wl, freq, du = small_case(n_ant=40, channels=(2, 30), N=N, W=W, OS=OS, flag_frac=0.1)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, tile=16, precision="bf16x3")
    assert 2 * (N // 16) ** 2 > 64 * torch.cuda.get_device_properties(0).multi_processor_count
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS)
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid(geom, wl.vis, wl.weights)
    rng = np.random.default_rng(5)
    Gin = (rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))).astype(np.complex64)
    M = plan.degrid(torch.from_numpy(Gin).cuda()).cpu().numpy()
    Mref = O.degrid(geom, Gin.astype(np.complex128))
    for c in range(2):
        assert rel_l2(G[c], Gref[c]) <= BF16X3_RTOL
        assert rel_l2(M[c], Mref[c]) <= BF16X3_RTOL
