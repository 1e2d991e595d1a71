"""Autograd through the HIP kernels: gradients against the FP64 oracle's
analytic gradients and against central finite differences of the oracle's
chi-squared on random grid cells."""
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


def setup(rts, seed=0, N=256, n_ant=40, channels=(0, 17, 31)):
    wl, freq, du = small_case(seed=seed, n_ant=n_ant, channels=channels, N=N, weights="uniform", flag_frac=0.1,
                              offgrid_frac=0.02)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du)
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du)
    return wl, freq, du, uvw, vis, w, plan, geom


def test_valid_mask_matches_oracle(rts):
    wl, freq, du, uvw, vis, w, plan, geom = setup(rts)
    assert np.array_equal(plan.valid_mask().cpu().numpy(), geom.valid)


def test_degrid_backward_is_grid(rts):
    wl, freq, du, uvw, vis, w, plan, geom = setup(rts, seed=1)
    rng = np.random.default_rng(1)
    G0 = (rng.standard_normal((3, 256, 256)) + 1j * rng.standard_normal((3, 256, 256))).astype(np.complex64)
    y = (rng.standard_normal(wl.vis.shape) + 1j * rng.standard_normal(wl.vis.shape)).astype(np.complex64)
    G = torch.from_numpy(G0).cuda().requires_grad_(True)
    yt = torch.from_numpy(y).cuda()
    M = rts.degrid(G, plan)
    loss = (torch.conj(yt) * M).real.sum()
    loss.backward()
    ref = O.grid(geom, np.where(geom.valid, y, 0), np.ones_like(wl.weights))
    for c in range(3):
        assert rel_l2(G.grad[c].cpu().numpy(), ref[c]) <= RTOL_L2


def test_grid_backward_matches_oracle_vjp(rts):
    wl, freq, du, uvw, vis, w, plan, geom = setup(rts, seed=2)
    rng = np.random.default_rng(2)
    Gt = (rng.standard_normal((3, 256, 256)) + 1j * rng.standard_normal((3, 256, 256))).astype(np.complex64)
    V = vis.clone().requires_grad_(True)
    wt = w.clone().requires_grad_(True)
    G = rts.grid(V, wt, plan)
    loss = (G - torch.from_numpy(Gt).cuda()).abs().pow(2).sum()
    loss.backward()
    Gref = O.grid(geom, wl.vis, wl.weights)
    gV, gw = O.grid_vjp(geom, wl.vis, wl.weights, 2.0 * (Gref - Gt))
    for c in range(3):
        assert rel_l2(V.grad[c].cpu().numpy(), gV[c]) <= RTOL_L2
        assert rel_l2(wt.grad[c].cpu().numpy(), gw[c]) <= RTOL_L2


def test_chi2_gradients_match_oracle(rts):
    wl, freq, du, uvw, vis, w, plan, geom = setup(rts, seed=3)
    rng = np.random.default_rng(3)
    G0 = (0.1 * (rng.standard_normal((3, 256, 256)) + 1j * rng.standard_normal((3, 256, 256)))).astype(np.complex64)
    G = torch.from_numpy(G0).cuda().requires_grad_(True)
    V = vis.clone().requires_grad_(True)
    wt = w.clone().requires_grad_(True)
    loss = rts.chi2(V, wt, G, plan)
    loss.backward()
    chi2, gG, gw, gV = O.chi2_gradients(geom, wl.vis, wl.weights, G0.astype(np.complex128))
    assert abs(loss.item() - chi2) <= RTOL_L2 * chi2
    for c in range(3):
        assert rel_l2(G.grad[c].cpu().numpy(), gG[c]) <= RTOL_L2
        assert rel_l2(wt.grad[c].cpu().numpy(), gw[c]) <= RTOL_L2
        assert rel_l2(V.grad[c].cpu().numpy(), gV[c]) <= RTOL_L2


def test_chi2_grad_against_oracle_finite_differences_on_64_cells(rts):
    """Central differences of the FP64 oracle's chi-squared (exact for a quadratic)
    at 64 random grid cells under the footprint, Re and Im separately."""
    wl, freq, du, uvw, vis, w, plan, geom = setup(rts, seed=4, N=128, n_ant=20, channels=(9,))
    rng = np.random.default_rng(4)
    G0 = (0.1 * (rng.standard_normal((1, 128, 128)) + 1j * rng.standard_normal((1, 128, 128)))).astype(np.complex64)
    G = torch.from_numpy(G0).cuda().requires_grad_(True)
    loss = rts.chi2(vis, w, G, plan)
    loss.backward()
    grad = G.grad.cpu().numpy()
    cover = np.argwhere(np.abs(O.grid(geom, np.ones_like(wl.vis), np.ones_like(wl.weights))) > 0)
    cells = cover[rng.choice(len(cover), 64, replace=False)]
    G64 = G0.astype(np.complex128)
    h = 1e-3 * np.sqrt(np.mean(np.abs(G64) ** 2))
    scale = np.max(np.abs(grad))
    for (c, yy, xx) in cells:
        for unit in (1.0, 1j):
            Gp = G64.copy(); Gp[c, yy, xx] += h * unit
            Gm = G64.copy(); Gm[c, yy, xx] -= h * unit
            fd = (O.grid_degrid(geom, wl.vis, wl.weights, Gp)[2] - O.grid_degrid(geom, wl.vis, wl.weights, Gm)[2]) / (2 * h)
            got = grad[c, yy, xx].real if unit == 1.0 else grad[c, yy, xx].imag
            assert abs(got - fd) <= 1e-5 * scale + 1e-5 * abs(fd)


def test_adjoint_identity_on_gpu(rts):
    """<grid_w(x), y> = <x, w * degrid(y)> with both sides from the HIP kernels."""
    wl, freq, du, uvw, vis, w, plan, geom = setup(rts, seed=5)
    rng = np.random.default_rng(5)
    x = torch.from_numpy((rng.standard_normal(wl.vis.shape) + 1j * rng.standard_normal(wl.vis.shape)).astype(np.complex64)).cuda()
    y = torch.from_numpy((rng.standard_normal((3, 256, 256)) + 1j * rng.standard_normal((3, 256, 256))).astype(np.complex64)).cuda()
    lhs = torch.vdot(plan.grid(x, w).flatten().to(torch.complex128), y.flatten().to(torch.complex128))
    rhs = torch.vdot(x.flatten().to(torch.complex128), (w * plan.degrid(y)).flatten().to(torch.complex128))
    scale = plan.grid(x, w).abs().pow(2).sum().sqrt().item() * y.abs().pow(2).sum().sqrt().item()
    assert abs((lhs - rhs).item()) <= 1e-6 * scale


@pytest.mark.parametrize("prec,W,OS,tol", [("fp32_mfma", 24, 8, RTOL_L2), ("bf16x3", 16, 16, 3e-5)])
def test_chi2_gradients_through_matrix_core_plans(rts, prec, W, OS, tol):
    """The chi-squared and its gradients with a matrix-core plan (its own fused
    step: degridding, then the residual gridding) against the oracle.  dL/dG is a
    gridding of the residual, so it carries the model's error as in the fused-step
    bound (factor 1 + |M| / |r|, about 2 here)."""
    N = 256
    wl, freq, du = small_case(seed=6, n_ant=40, channels=(0, 17, 31), N=N, W=W, OS=OS, weights="uniform",
                              flag_frac=0.1, offgrid_frac=0.02)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, precision=prec)
    geom = O.Geometry(wl.uvw_m, freq, wl.weights, N, du, W, OS)
    rng = np.random.default_rng(6)
    G0 = (0.1 * (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N)))).astype(np.complex64)
    G = torch.from_numpy(G0).cuda().requires_grad_(True)
    V = vis.clone().requires_grad_(True)
    wt = w.clone().requires_grad_(True)
    loss = rts.chi2(V, wt, G, plan)
    loss.backward()
    chi2, gG, gw, gV = O.chi2_gradients(geom, wl.vis, wl.weights, G0.astype(np.complex128))
    assert abs(loss.item() - chi2) <= 4 * tol * chi2
    for c in range(3):
        assert rel_l2(G.grad[c].cpu().numpy(), gG[c]) <= 4 * tol
        assert rel_l2(wt.grad[c].cpu().numpy(), gw[c]) <= 4 * tol
        assert rel_l2(V.grad[c].cpu().numpy(), gV[c]) <= 4 * tol


def test_backward_entry_points_through_the_abi(rts):
    """rts_grid_backward and rts_chi2_backward called directly, with an upstream
    chi-squared gradient other than 1, against the oracle's analytic gradients."""
    wl, freq, du, uvw, vis, w, plan, geom = setup(rts, seed=7)
    rng = np.random.default_rng(7)
    gGt = (rng.standard_normal((3, 256, 256)) + 1j * rng.standard_normal((3, 256, 256))).astype(np.complex64)
    gV, gw = plan.grid_backward(vis, w, torch.from_numpy(gGt).cuda())
    rV, rw = O.grid_vjp(geom, wl.vis, wl.weights, gGt.astype(np.complex128))
    for c in range(3):
        assert rel_l2(gV[c].cpu().numpy(), rV[c]) <= RTOL_L2
        assert rel_l2(gw[c].cpu().numpy(), rw[c]) <= RTOL_L2
    G0 = (0.1 * (rng.standard_normal((3, 256, 256)) + 1j * rng.standard_normal((3, 256, 256)))).astype(np.complex64)
    model, gres, chi2 = plan.grid_degrid(vis, w, torch.from_numpy(G0).cuda())
    g = torch.tensor(0.37, dtype=torch.float64, device="cuda")
    bV, bw, bG = plan.chi2_backward(vis, w, model, gres, g)
    chi2o, oG, ow, oV = O.chi2_gradients(geom, wl.vis, wl.weights, G0.astype(np.complex128))
    for c in range(3):
        assert rel_l2(bG[c].cpu().numpy(), 0.37 * oG[c]) <= RTOL_L2
        assert rel_l2(bw[c].cpu().numpy(), 0.37 * ow[c]) <= RTOL_L2
        assert rel_l2(bV[c].cpu().numpy(), 0.37 * oV[c]) <= RTOL_L2
    assert torch.all(bV.cpu()[~torch.from_numpy(geom.valid)] == 0)


def test_conjugate_plans_are_rejected(rts):
    """Gridding with conjugate copies adds conj(w V) at -uv, which is not
    complex-linear in V: the autograd functions and the backward entry points
    refuse such plans instead of returning a wrong adjoint."""
    wl, freq, du = small_case(seed=8, n_ant=30, channels=(0, 9), N=128)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, 128, du, conjugate=True)
    G = torch.zeros((2, 128, 128), dtype=torch.complex64, device="cuda")
    for f in (lambda: rts.grid(vis, w, plan), lambda: rts.degrid(G, plan), lambda: rts.chi2(vis, w, G, plan)):
        with pytest.raises(ValueError):
            f()
    with pytest.raises(rts.RtsError) as ei:
        plan.grid_backward(vis, w, G)
    assert ei.value.status == 4                      # RTS_E_UNSUPPORTED
    g = torch.ones((), dtype=torch.float64, device="cuda")
    with pytest.raises(rts.RtsError) as ei:
        plan.chi2_backward(vis, w, vis.clone(), G, g)
    assert ei.value.status == 4
