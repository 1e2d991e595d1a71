"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None re-types the oracle's own formulas: kernel
values come from mpmath's Bessel function, the gather check uses the closed-form
kernel with no phase table, the DFT check uses a brute-force Fourier sum, and the
adjoint / Hermitian / permutation checks are identities.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O
from synth import make_workload

mp.mp.dps = 40


def kb_mp(t, W, beta):
    """Closed-form Kaiser-Bessel value in 40-digit arithmetic (zero at and beyond W/2)."""
    t = mp.mpf(t)
    if abs(t) >= mp.mpf(W) / 2:
        return mp.mpf(0)
    a = 2 * t / W
    return mp.besseli(0, beta * mp.sqrt(1 - a * a)) / mp.besseli(0, beta)


def place(N, du, f, xs, ys, OS):
    """uvw (metres) whose snapped coordinate is exactly (xs, ys)."""
    s = f / (O.C_LIGHT * du)
    x = (xs + 0.25) / OS
    y = (ys + 0.25) / OS
    return (x - N / 2) / s, (y - N / 2) / s


# ------------------------------------------------------------------------ kernel
@pytest.mark.parametrize("W", [4, 7, 8, 16])
def test_kernel_values_against_bessel(W):
    beta = O.default_beta(W)
    ts = np.linspace(-W / 2 - 0.3, W / 2 + 0.3, 57)
    ref = np.array([float(kb_mp(t, W, mp.mpf(beta))) for t in ts])
    got = O.kb(ts, W, beta)
    assert np.max(np.abs(got - ref)) <= 1e-14
    assert O.kb(0.0, W, beta) == pytest.approx(1.0, abs=1e-15)
    assert O.kb(W / 2, W, beta) == 0.0 and O.kb(-W / 2, W, beta) == 0.0


def test_kernel_reference_numbers_w7():
    # values quoted for W=7, beta=16.38
    k = O.kb(np.array([0.5, 1.0, 2.0, 3.0]), 7, 16.38)
    assert k == pytest.approx([0.849791, 0.516253, 0.0585953, 4.98781e-4], rel=2e-6)


@pytest.mark.parametrize("W,OS", [(7, 8), (8, 8), (16, 16), (5, 4), (7, 1)])
def test_table_phases_cover_half_cell(W, OS):
    r, t = O.phase_range(W, OS)
    assert len(r) == OS and len(t) == W
    # every tap sits within W/2 of the snapped position, and the phase set spans one cell
    d = t[None, :] - r[:, None] / OS
    assert np.all(np.abs(d) <= W / 2)
    assert r[-1] - r[0] == OS - 1


# ------------------------------------------------------------------- coordinates
def test_snapped_within_half_phase_of_exact():
    rng = np.random.default_rng(5)
    N, du, OS = 256, 10.0, 8
    uvw = rng.uniform(-1500, 1500, (40, 3, 3))
    f = np.array([140e6, 170e6])
    xs, ys, fin = O.snapped(uvw, f, N, du, OS)
    assert fin.all()
    for c in range(2):
        for b in range(0, 40, 7):
            for t in range(3):
                s = mp.mpf(f[c]) / (mp.mpf(O.C_LIGHT) * mp.mpf(du))
                x = mp.mpf(uvw[b, t, 0]) * s + N / 2
                y = mp.mpf(uvw[b, t, 1]) * s + N / 2
                assert abs(mp.mpf(int(xs[c, b, t])) / OS - x) <= mp.mpf(1) / (2 * OS) + mp.mpf("1e-12")
                assert abs(mp.mpf(int(ys[c, b, t])) / OS - y) <= mp.mpf(1) / (2 * OS) + mp.mpf("1e-12")


def test_origin_maps_to_grid_centre():
    N, OS = 64, 8
    xs, ys, _ = O.snapped(np.zeros((1, 1, 3)), np.array([150e6]), N, 3.0, OS)
    assert xs[0, 0, 0] == N // 2 * OS and ys[0, 0, 0] == N // 2 * OS
    cx, rx = O.cell_phase(xs, 7, OS)
    assert cx[0, 0, 0] == N // 2 and rx[0, 0, 0] == 0


@pytest.mark.parametrize("W,OS", [(7, 8), (8, 8), (16, 16)])
def test_offgrid_rule_brute_force(W, OS):
    rng = np.random.default_rng(11)
    N, du, f = 32, 40.0, np.array([150e6])
    uvw = rng.uniform(-900, 900, (300, 1, 3))
    w = np.ones((1, 300, 1), np.float32)
    w[0, ::13] = 0
    cx, cy, rx, ry, valid = O.coords(uvw, f, w, N, du, W, OS)
    xs, ys, _ = O.snapped(uvw, f, N, du, OS)
    for b in range(300):
        # taps = every pixel within W/2 of the snapped position, counted with the
        # closed-form support rule; valid iff none falls off the grid and w != 0
        xq, yq = xs[0, b, 0] / OS, ys[0, b, 0] / OS
        r, t = O.phase_range(W, OS)
        px = cx[0, b, 0] + t
        py = cy[0, b, 0] + t
        assert np.all(np.abs(px - xq) <= W / 2) and np.all(np.abs(py - yq) <= W / 2)
        on = px.min() >= 0 and px.max() < N and py.min() >= 0 and py.max() < N
        assert valid[0, b, 0] == (on and w[0, b, 0] != 0)


# ------------------------------------------------------------- P1 unit visibility
@pytest.mark.parametrize("W,OS", [(7, 8), (8, 8), (6, 4), (16, 16)])
def test_unit_visibility_reproduces_kernel(W, OS):
    N, du, f = 64, 25.0, 150e6
    beta = O.default_beta(W)
    r_all, t_all = O.phase_range(W, OS)
    cx0, cy0 = 30, 33
    for ry in r_all:
        for rx in r_all[:: max(1, OS // 4)] if ry != r_all[0] else r_all:
            xs, ys = cx0 * OS + rx, cy0 * OS + ry
            u, v = place(N, du, f, xs, ys, OS)
            uvw = np.array([[[u, v, 0.0]]])
            g = O.Geometry(uvw, [f], np.ones((1, 1, 1)), N, du, W, OS)
            G = O.grid(g, np.ones((1, 1, 1), np.complex64), np.ones((1, 1, 1)))
            exp = np.zeros((N, N))
            ky = [float(kb_mp(t - mp.mpf(int(ry)) / OS, W, mp.mpf(beta))) for t in t_all]
            kx = [float(kb_mp(t - mp.mpf(int(rx)) / OS, W, mp.mpf(beta))) for t in t_all]
            for a, ty in enumerate(t_all):
                for b, tx in enumerate(t_all):
                    exp[cy0 + ty, cx0 + tx] = ky[a] * kx[b]
            assert np.max(np.abs(G[0] - exp)) <= 1e-14  # np.i0 is accurate to ~1e-15 relative
            assert np.all(G[0].imag == 0)


# --------------------------------------------------------------- P2 grid sum
@pytest.mark.parametrize("W,OS", [(7, 8), (16, 16)])
def test_grid_sum_equals_weighted_kernel_sums(W, OS):
    beta = O.default_beta(W)
    wl = make_workload("tiny", seed=3)
    g = O.Geometry(wl.uvw_m, wl.freq_hz, wl.weights, 256, wl.cell_lambda, W, OS)
    w = np.random.default_rng(1).uniform(0.5, 1.5, wl.weights.shape)
    G = O.grid(g, wl.vis, w)
    r_all, t_all = O.phase_range(W, OS)
    S = {int(r): mp.fsum(kb_mp(t - mp.mpf(int(r)) / OS, W, mp.mpf(beta)) for t in t_all) for r in r_all}
    cx, cy, rx, ry, valid = g.copies[0]
    tot = 0j
    for idx in zip(*np.nonzero(valid)):
        tot += w[idx] * complex(wl.vis[idx]) * float(S[int(rx[idx])] * S[int(ry[idx])])
    assert abs(G.sum() - tot) <= 1e-13 * np.sum(np.abs(w * wl.vis))
    # the phase sums approximate the kernel's integral, W sinh(beta)/(beta I0(beta))
    khat0 = mp.mpf(W) * mp.sinh(beta) / (beta * mp.besseli(0, beta))
    dev = max(abs(S[r] - khat0) for r in S) / khat0
    assert dev < (1.5e-6 if W == 7 else 1e-12)


# ----------------------------------------------------------- P3 Hermitian symmetry
@pytest.mark.parametrize("W,OS", [(7, 8), (8, 8)])
def test_conjugate_gridding_is_hermitian(W, OS):
    wl = make_workload("tiny", seed=4)
    N = 256
    g = O.Geometry(wl.uvw_m, wl.freq_hz, wl.weights, N, wl.cell_lambda, W, OS, conjugate=True)
    G = O.grid(g, wl.vis, wl.weights)[0]
    idx = (N - np.arange(N)) % N
    mirror = G[idx][:, idx]
    assert np.max(np.abs(mirror - np.conj(G))) <= 1e-14 * np.max(np.abs(G))
    img = O.image(G[None], W, g.beta)[0]
    assert np.max(np.abs(img.imag)) <= 1e-12 * np.max(np.abs(img.real))


# ------------------------------------------------------------ P4 direct DFT
def alias_bound(W, beta, nu_max, M=4000):
    nus = np.linspace(-nu_max, nu_max, 41)
    worst = 0.0
    for nu in nus:
        m = np.concatenate([np.arange(-M, 0), np.arange(1, M + 1)])
        s = np.sum(np.abs(O.kb_hat(nu + m, W, beta))) / O.kb_hat(np.array([nu]), W, beta)[0]
        worst = max(worst, s)
    # tail beyond M decays like 1/m^2 with |khat| <= W / (pi W |m|) * 1/(pi W |m|) ... bounded generously
    return worst + 4.0 / (math.pi ** 2 * W * M) / O.kb_hat(np.array([nu_max]), W, beta)[0]


@pytest.mark.parametrize("N,W,OS", [(256, 7, 8), (64, 7, 8), (96, 16, 16)])
def test_grid_fft_matches_direct_dft(N, W, OS):
    wl = make_workload("tiny", seed=2)
    margin = math.ceil(W / 2) + 1
    umax = np.max(np.abs(wl.uvw_m[:, :, :2])) * wl.freq_hz.max() / O.C_LIGHT
    du = umax / (N // 2 - margin)
    g = O.Geometry(wl.uvw_m, wl.freq_hz, wl.weights, N, du, W, OS)
    assert g.valid.all()
    G = O.grid(g, wl.vis, wl.weights)
    img = O.image(G, W, g.beta)[0]
    xs, ys, _ = O.snapped(wl.uvw_m, wl.freq_hz, N, du, OS)
    a = (wl.weights * wl.vis.astype(np.complex128))[0].ravel()
    q = np.arange(N // 4, 3 * N // 4 + 1)
    region = [(qy, qx) for qy in q[::3] for qx in q[::3]]
    ref = O.direct_dft(xs[0].ravel(), ys[0].ravel(), a, N, OS, region)
    got = np.array([img[qy, qx] for qy, qx in region])
    eps1 = alias_bound(W, g.beta, 0.25)
    bound = ((1 + eps1) ** 2 - 1) * np.sum(np.abs(a))
    assert np.max(np.abs(got - ref)) <= bound + 1e-9 * np.sum(np.abs(a))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= (1e-5 if W == 7 else 1e-12)


# ------------------------------------------------------------- P5 adjoint identity
@pytest.mark.parametrize("conj", [False, True])
@pytest.mark.parametrize("W,OS", [(7, 8), (8, 8)])
def test_adjoint_identity(W, OS, conj):
    rng = np.random.default_rng(7)
    wl = make_workload("tiny", seed=6)
    N = 256
    w = rng.uniform(0.5, 1.5, wl.weights.shape)
    w[0, ::9] = 0
    g = O.Geometry(wl.uvw_m, wl.freq_hz, w, N, wl.cell_lambda, W, OS, conjugate=conj)
    x = rng.standard_normal(w.shape) + 1j * rng.standard_normal(w.shape)
    y = rng.standard_normal((1, N, N)) + 1j * rng.standard_normal((1, N, N))
    lhs = np.vdot(O.grid(g, x, w), y)
    rhs = np.vdot(x, O.grid_adjoint(g, y, w))
    scale = np.linalg.norm(O.grid(g, x, w)) * np.linalg.norm(y)
    if conj:
        assert abs(lhs.real - rhs.real) <= 1e-13 * scale
    else:
        assert abs(lhs - rhs) <= 1e-13 * scale
        # without conjugates the adjoint is exactly w * degrid
        assert np.allclose(O.grid_adjoint(g, y, w), w * O.degrid(g, y), rtol=0, atol=1e-14 * np.abs(y).max())


# ------------------------------------------------- P6 scatter == gather == C oracle
@pytest.mark.parametrize("W,OS,conj", [(7, 8, False), (8, 8, True), (16, 16, False), (7, 1, False)])
def test_scatter_equals_naive_gather(W, OS, conj):
    wl = make_workload("tiny", seed=9, n_ant=14)
    N = 64 if W < 16 else 96
    margin = math.ceil(W / 2) + 1
    umax = np.max(np.abs(wl.uvw_m[:, :, :2])) * wl.freq_hz.max() / O.C_LIGHT
    du = umax / (N // 2 - margin)
    w = np.random.default_rng(3).uniform(0.5, 1.5, wl.weights.shape)
    g = O.Geometry(wl.uvw_m, wl.freq_hz, w, N, du, W, OS, conjugate=conj)
    G = O.grid(g, wl.vis, w)
    Gg = O.gather_grid(wl.uvw_m, wl.freq_hz, wl.vis, w, N, du, W, OS, conjugate=conj)
    assert np.max(np.abs(G - Gg)) <= 1e-12 * np.max(np.abs(G))


def test_c_oracle_matches_numpy_oracle(cpu_oracle):
    wl = make_workload("single_cadence", seed=1, channels=[0, 17], n_ant=40)
    freq = wl.freq_hz[wl.channels]
    N, du = 512, None
    margin = 5
    umax = np.max(np.abs(wl.uvw_m[:, :, :2])) * freq.max() / O.C_LIGHT
    du = umax / (N // 2 - margin)
    rng = np.random.default_rng(0)
    w = rng.uniform(0.5, 1.5, wl.weights.shape).astype(np.float32)
    w[:, ::7] = 0
    for W, OS in [(7, 8), (8, 4)]:
        g = O.Geometry(wl.uvw_m, freq, w, N, du, W, OS)
        G = O.grid(g, wl.vis, w)
        Gc = cpu_oracle.grid(wl.uvw_m, freq, wl.vis, w, N, du, W, OS)
        assert np.max(np.abs(G - Gc)) <= 1e-12 * np.max(np.abs(G))
        Gin = (rng.standard_normal(G.shape) + 1j * rng.standard_normal(G.shape)).astype(np.complex64)
        M = O.degrid(g, Gin.astype(np.complex128))
        Mc = cpu_oracle.degrid(wl.uvw_m, freq, w, Gin, N, du, W, OS)
        assert np.max(np.abs(M - Mc)) <= 1e-12 * np.max(np.abs(M))
        Mo, Go, chi2, _ = O.grid_degrid(g, wl.vis, w, Gin.astype(np.complex128))
        Mc2, Gc2, chi2c = cpu_oracle.grid_degrid(wl.uvw_m, freq, wl.vis, w, Gin, N, du, W, OS)
        assert np.max(np.abs(Mo - Mc2)) <= 1e-12 * np.max(np.abs(Mo))
        assert np.max(np.abs(Go - Gc2)) <= 1e-12 * np.max(np.abs(Go))
        assert chi2 == pytest.approx(chi2c.sum(), rel=1e-12)


# --------------------------------------------------------------- P7 invariances
def test_permutation_and_channel_split_invariance():
    wl = make_workload("single_cadence", seed=2, channels=[3, 9], n_ant=24)
    freq = wl.freq_hz[wl.channels]
    N = 128
    umax = np.max(np.abs(wl.uvw_m[:, :, :2])) * freq.max() / O.C_LIGHT
    du = umax / (N // 2 - 5)
    g = O.Geometry(wl.uvw_m, freq, wl.weights, N, du)
    G = O.grid(g, wl.vis, wl.weights)
    perm = np.random.default_rng(0).permutation(wl.n_base)
    gp = O.Geometry(wl.uvw_m[perm], freq, wl.weights[:, perm], N, du)
    Gp = O.grid(gp, wl.vis[:, perm], wl.weights[:, perm])
    assert np.max(np.abs(G - Gp)) <= 1e-13 * np.max(np.abs(G))
    for k in range(2):
        gk = O.Geometry(wl.uvw_m, freq[k:k + 1], wl.weights[k:k + 1], N, du)
        assert np.max(np.abs(O.grid(gk, wl.vis[k:k + 1], wl.weights[k:k + 1])[0] - G[k])) == 0.0


def test_flagged_and_offgrid_samples_contribute_nothing():
    wl = make_workload("tiny_literal", seed=0)
    g = O.Geometry(wl.uvw_m, wl.freq_hz, wl.weights, 256, wl.cell_lambda)
    n_valid = int(g.valid.sum())
    assert 0 < n_valid < 0.05 * g.valid.size        # the literal 0.5-lambda cell drops most
    G = O.grid(g, wl.vis, wl.weights)
    keep = np.where(g.valid, wl.vis, 0)
    G2 = O.grid(g, keep, wl.weights)
    assert np.array_equal(G, G2)
    M = O.degrid(g, G)
    assert np.all(M[~g.valid] == 0)


# ------------------------------------------------------------------ P8 gradients
def test_chi2_gradients_match_finite_differences():
    rng = np.random.default_rng(12)
    wl = make_workload("tiny", seed=12)
    N = 256
    w = rng.uniform(0.5, 1.5, wl.weights.shape)
    g = O.Geometry(wl.uvw_m, wl.freq_hz, w, N, wl.cell_lambda)
    G0 = 0.1 * (rng.standard_normal((1, N, N)) + 1j * rng.standard_normal((1, N, N)))
    chi2, gG, gw, gV = O.chi2_gradients(g, wl.vis, w, G0)

    def L(G=G0, ww=w, V=wl.vis):
        return O.grid_degrid(O.Geometry(wl.uvw_m, wl.freq_hz, ww, N, wl.cell_lambda), V, ww, G)[2]

    cover = np.argwhere(np.abs(O.grid(g, np.ones_like(wl.vis), np.ones_like(w))[0]) > 0)
    cells = cover[rng.choice(len(cover), 64, replace=False)]
    h = 1e-3 * np.sqrt(np.mean(np.abs(G0) ** 2))
    for (yy, xx) in cells:
        for unit in (1.0, 1j):
            Gp = G0.copy(); Gp[0, yy, xx] += h * unit
            Gm = G0.copy(); Gm[0, yy, xx] -= h * unit
            fd = (L(G=Gp) - L(G=Gm)) / (2 * h)
            an = gG[0, yy, xx].real if unit == 1.0 else gG[0, yy, xx].imag
            assert fd == pytest.approx(an, rel=1e-6, abs=1e-8 * max(1.0, chi2))
    for b in rng.choice(w.shape[1], 10, replace=False):
        wp = w.copy(); wp[0, b, 0] += 1e-3
        wm = w.copy(); wm[0, b, 0] -= 1e-3
        fd = (L(ww=wp) - L(ww=wm)) / 2e-3
        assert fd == pytest.approx(gw[0, b, 0], rel=1e-6, abs=1e-9)


def test_grid_vjp_matches_finite_differences():
    rng = np.random.default_rng(13)
    wl = make_workload("tiny", seed=13, n_ant=12)
    N = 256
    w = rng.uniform(0.5, 1.5, wl.weights.shape)
    g = O.Geometry(wl.uvw_m, wl.freq_hz, w, N, wl.cell_lambda)
    Gt = rng.standard_normal((1, N, N)) + 1j * rng.standard_normal((1, N, N))
    V = wl.vis.astype(np.complex128)

    def L2(V=V, ww=w):
        gg = O.Geometry(wl.uvw_m, wl.freq_hz, ww, N, wl.cell_lambda)
        return float(np.sum(np.abs(O.grid(gg, V, ww) - Gt) ** 2))

    gG = 2.0 * (O.grid(g, V, w) - Gt)
    gV, gw = O.grid_vjp(g, V, w, gG)
    for b in rng.choice(w.shape[1], 12, replace=False):
        for unit in (1.0, 1j):
            Vp = V.copy(); Vp[0, b, 0] += 1e-4 * unit
            Vm = V.copy(); Vm[0, b, 0] -= 1e-4 * unit
            fd = (L2(V=Vp) - L2(V=Vm)) / 2e-4
            an = gV[0, b, 0].real if unit == 1.0 else gV[0, b, 0].imag
            assert fd == pytest.approx(an, rel=1e-6, abs=1e-7)
        wp = w.copy(); wp[0, b, 0] += 1e-4
        wm = w.copy(); wm[0, b, 0] -= 1e-4
        fd = (L2(ww=wp) - L2(ww=wm)) / 2e-4
        assert fd == pytest.approx(gw[0, b, 0], rel=1e-6, abs=1e-7)


# ------------------------------------------------------- polarisation conversion
def _stokes_to_linear(I, Q, U, V):
    """Observed products of ideal linear feeds: XX = I + Q, XY = U + iV,
    YX = U - iV, YY = I - Q (the textbook relation, independent of the oracle)."""
    return np.stack([I + Q, U + 1j * V, U - 1j * V, I - Q])


def test_polconvert_identity_returns_input():
    rng = np.random.default_rng(11)
    P = rng.standard_normal((3, 4, 37)) + 1j * rng.standard_normal((3, 4, 37))
    A = np.zeros((4, 4, 37), np.complex128)
    for r in range(4):
        A[r, r] = 1.0
    assert np.array_equal(O.polconvert(A, P), P)


def test_polconvert_recovers_stokes_from_linear_feeds():
    """A = the inverse of the linear-feed relation, written row by row:
    I = (XX + YY)/2, Q = (XX - YY)/2, U = (XY + YX)/2, V = -i (XY - YX)/2.
    The matrix is not symmetric, so a transposed operand fails here."""
    rng = np.random.default_rng(12)
    n = 50
    stokes = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for _ in range(4)]
    P = _stokes_to_linear(*stokes)[None]
    M = np.array([[0.5, 0, 0, 0.5], [0.5, 0, 0, -0.5], [0, 0.5, 0.5, 0], [0, -0.5j, 0.5j, 0]])
    A = np.repeat(M[:, :, None], n, axis=2)
    S = O.polconvert(A, P)
    for r in range(4):
        np.testing.assert_allclose(S[0, r], stokes[r], rtol=0, atol=1e-14)


def test_polconvert_composition_and_per_channel_matrices():
    """Converting with B after A equals converting once with the per-pixel
    product B A (formed by explicit loops); per-channel matrices (c+1) I scale
    channel c by c+1; a shared matrix equals the same matrix given per channel."""
    rng = np.random.default_rng(13)
    n, C = 9, 3
    A = rng.standard_normal((4, 4, n)) + 1j * rng.standard_normal((4, 4, n))
    B = rng.standard_normal((4, 4, n)) + 1j * rng.standard_normal((4, 4, n))
    P = rng.standard_normal((C, 4, n)) + 1j * rng.standard_normal((C, 4, n))
    BA = np.zeros((4, 4, n), np.complex128)
    for i in range(n):
        for r in range(4):
            for k in range(4):
                BA[r, k, i] = sum(B[r, m, i] * A[m, k, i] for m in range(4))
    np.testing.assert_allclose(O.polconvert(B, O.polconvert(A, P)), O.polconvert(BA, P), rtol=1e-12, atol=1e-12)
    Ac = np.zeros((C, 4, 4, n), np.complex128)
    for c in range(C):
        for r in range(4):
            Ac[c, r, r] = c + 1
    S = O.polconvert(Ac, P)
    for c in range(C):
        np.testing.assert_array_equal(S[c], (c + 1) * P[c])
    np.testing.assert_array_equal(O.polconvert(np.stack([A] * C), P), O.polconvert(A, P))


def test_polconvert_pixels_are_independent():
    rng = np.random.default_rng(14)
    n = 21
    A = rng.standard_normal((4, 4, n)) + 1j * rng.standard_normal((4, 4, n))
    P = rng.standard_normal((2, 4, n)) + 1j * rng.standard_normal((2, 4, n))
    perm = rng.permutation(n)
    np.testing.assert_array_equal(O.polconvert(A[..., perm], P[..., perm]), O.polconvert(A, P)[..., perm])


# ------------------------------------------------ per-visibility (per-baseline) kernels
def _small_pb(W, OS, conj=False, seed=0):
    wl = make_workload("tiny", seed=seed)
    freq = wl.freq_hz[wl.channels]
    rng = np.random.default_rng(seed + 50)
    w = rng.uniform(0.5, 1.5, wl.weights.shape)
    geom = O.Geometry(wl.uvw_m, freq, w, 256, wl.cell_lambda, W, OS, conjugate=conj)
    return wl, w, geom


@pytest.mark.parametrize("W,OS,conj", [(7, 8, False), (24, 8, True), (8, 4, True)])
def test_per_baseline_with_the_shared_table_is_plain_gridding(W, OS, conj):
    """Every baseline given the Kaiser-Bessel table: identical to the pinned
    shared-kernel gridding and degridding."""
    wl, w, geom = _small_pb(W, OS, conj)
    B = wl.uvw_m.shape[0]
    tabs = np.broadcast_to(geom.tab, (B,) + geom.tab.shape)
    np.testing.assert_array_equal(O.grid_per_baseline(geom, wl.vis, w, tabs), O.grid(geom, wl.vis, w))
    G = np.random.default_rng(2).standard_normal((1, 256, 256)) + 0j
    np.testing.assert_array_equal(O.degrid_per_baseline(geom, G, tabs), O.degrid(geom, G))


@pytest.mark.parametrize("W,OS", [(7, 8), (24, 8)])
def test_per_baseline_scaling_selects_each_baseline_and_phase(W, OS):
    """Baseline b's table = s_b g[p] x (shared table row p): each sample's
    contribution is scaled by s_b^2 g[r_y] g[r_x], i.e. shared-kernel gridding with
    those factors folded into the weights.  A table taken from the wrong baseline
    or the wrong phase row fails here."""
    wl, w, geom = _small_pb(W, OS, seed=3)
    B = wl.uvw_m.shape[0]
    rng = np.random.default_rng(4)
    s = rng.uniform(0.5, 2.0, B)
    g = rng.uniform(0.5, 2.0, OS)
    tabs = s[:, None, None] * (g[:, None] * geom.tab)[None]
    cx, cy, rx, ry, valid = geom.copies[0]
    r0 = geom.r[0]
    w2 = w * (s[None, :, None] ** 2) * g[rx - r0] * g[ry - r0]
    np.testing.assert_allclose(O.grid_per_baseline(geom, wl.vis, w, tabs), O.grid(geom, wl.vis, w2),
                               rtol=1e-12, atol=1e-12)


def test_per_baseline_adjoint_identity():
    """<grid(V), G> = <V, degrid(G)> with unit weights and random per-baseline tables."""
    wl, _, geom = _small_pb(24, 8, seed=5)
    B = wl.uvw_m.shape[0]
    rng = np.random.default_rng(6)
    tabs = rng.uniform(0.0, 1.0, (B, 8, 24))
    ones = np.ones(wl.weights.shape)
    geom1 = O.Geometry(wl.uvw_m, wl.freq_hz[wl.channels], ones, 256, wl.cell_lambda, 24, 8)
    G = rng.standard_normal((1, 256, 256)) + 1j * rng.standard_normal((1, 256, 256))
    lhs = np.vdot(O.grid_per_baseline(geom1, wl.vis, ones, tabs).ravel(), G.ravel())
    rhs = np.vdot(np.asarray(wl.vis, np.complex128).ravel(), O.degrid_per_baseline(geom1, G, tabs).ravel())
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
