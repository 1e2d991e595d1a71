"""Plain, slow, FP64 definition of what the gridding hot path computes.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function follows the
paper (Edgar et al., "Enabling a High Throughput Real Time Data Pipeline for a Large
Radio Telescope Array with GPUs") and states the passage it restates:

  * Section 5, Eq. (1): the gridded value is the sum over visibilities of the
    gridding convolution function centred on each visibility times its value; the
    function vanishes beyond a cut-off radius.
  * Section 5, following Eq. (1): each visibility adds its weighted values to the
    pixels of the patch it covers (the scatter form the C code used), the weight
    being the function evaluated at the distance from the visibility to the pixel
    centre.  Section 5.2: the same sum taken per pixel (the gather form).

The anti-aliasing function is a separable Kaiser-Bessel window of support W
sampled at OS phases per cell (the paper's spheroidal function is replaced by this
window; the paper gives no coefficients for it).  Readings where the paper is
silent are marked READING and collected in the design notes.

Conventions: grids are complex [C][N][N] indexed [channel][v][u]; pixel N/2 is
u = 0; visibilities, weights and models are [C][B][T]; uvw is [B][T][3] metres.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299_792_458.0


# --------------------------------------------------------------------------- kernel
def default_beta(W: int) -> float:
    """READING: Kaiser-Bessel shape parameter 2.34 * W."""
    return 2.34 * W


def kb(t, W: int, beta: float) -> np.ndarray:
    """1-D gridding convolution function k(t) = I0(beta sqrt(1-(2t/W)^2)) / I0(beta).

    Zero for |t| >= W/2: Eq. (1) states the function vanishes beyond r_max; the
    edge itself is set to zero (READING), which makes conjugate gridding exactly
    Hermitian.
    """
    t = np.asarray(t, dtype=np.float64)
    a = 2.0 * t / W
    inside = np.abs(t) < W / 2.0
    arg = beta * np.sqrt(np.where(inside, 1.0 - a * a, 0.0))
    return np.where(inside, np.i0(arg) / np.i0(beta), 0.0)


def kb_hat(nu, W: int, beta: float) -> np.ndarray:
    """Fourier transform of kb: W sinh(sqrt(b^2-(pi W nu)^2)) / (sqrt(.) I0(beta)).

    Used only for the image-domain grid correction of the DFT check.
    """
    nu = np.asarray(nu, dtype=np.float64)
    z2 = beta * beta - (math.pi * W * nu) ** 2
    out = np.empty_like(nu)
    pos = z2 > 0
    z = np.sqrt(np.abs(z2))
    out[pos] = W * np.sinh(z[pos]) / z[pos]
    neg = z2 < 0
    out[neg] = W * np.sin(z[neg]) / z[neg]
    out[z2 == 0] = W
    return out / np.i0(beta)


def phase_range(W: int, OS: int):
    """Phase offsets r (in 1/OS cells) and tap offsets t of the sampled kernel.

    Odd W: the visibility snaps to the nearest cell, r in [-(OS//2), OS - OS//2),
    taps t in [-(W-1)/2, (W-1)/2].  Even W: the cell to the left, r in [0, OS),
    taps t in [-W/2+1, W/2].  In both cases every tap lies within W/2 of the
    snapped position (READING of "distance from the visibility to the centre of a
    given pixel", Section 5).
    """
    if W % 2:
        r0, t0 = -(OS // 2), -(W - 1) // 2
    else:
        r0, t0 = 0, -(W // 2) + 1
    return np.arange(r0, r0 + OS), np.arange(t0, t0 + W)


def table(W: int, OS: int, beta: float) -> np.ndarray:
    """tab[p][j] = k(t_j - r_p/OS), the kernel sampled at OS phases (READING: nearest
    phase, no interpolation)."""
    r, t = phase_range(W, OS)
    return kb(t[None, :] - r[:, None] / OS, W, beta)


# ----------------------------------------------------------------------- coordinates
def snapped(uvw_m, freq_hz, N: int, du: float, OS: int, conjugate_copy: bool = False):
    """Oversampled integer grid coordinates (xs, ys) [C][B][T] and a finite mask.

    x = u f / (c du) + N/2 in cells, snapped to 1/OS cell by rounding half up
    (READING).  Section 5: the pixel a visibility affects follows from its
    distance to the pixel centres; pixel N/2 is u = 0 (READING).
    The products are evaluated in the order s = f/(c du); x = u*s + N/2;
    xs = floor(x*OS + 0.5), each step rounded once.
    """
    uvw_m = np.asarray(uvw_m, np.float64)
    sgn = -1.0 if conjugate_copy else 1.0
    s = np.asarray(freq_hz, np.float64) / (C_LIGHT * du)            # [C]
    u = sgn * uvw_m[None, :, :, 0]
    v = sgn * uvw_m[None, :, :, 1]
    x = u * s[:, None, None] + N / 2
    y = v * s[:, None, None] + N / 2
    xo = np.floor(x * OS + 0.5)
    yo = np.floor(y * OS + 0.5)
    lim = 2.0 ** 30
    finite = np.isfinite(xo) & np.isfinite(yo) & (np.abs(xo) < lim) & (np.abs(yo) < lim)
    xs = np.where(finite, xo, 0).astype(np.int64)
    ys = np.where(finite, yo, 0).astype(np.int64)
    return xs, ys, finite


def cell_phase(xs, W: int, OS: int):
    """Split an oversampled coordinate into (cell, phase r) per phase_range."""
    r0 = phase_range(W, OS)[0][0]
    c = np.floor_divide(xs - r0, OS)
    return c, xs - c * OS


def coords(uvw_m, freq_hz, weights, N: int, du: float, W: int, OS: int, conjugate_copy=False):
    """(cx, cy, rx, ry, valid), all [C][B][T].

    READING: a sample is valid iff its weight is non-zero and every tap lies on the
    grid; invalid samples contribute nothing and predict 0.
    """
    xs, ys, fin = snapped(uvw_m, freq_hz, N, du, OS, conjugate_copy)
    cx, rx = cell_phase(xs, W, OS)
    cy, ry = cell_phase(ys, W, OS)
    t = phase_range(W, OS)[1]
    lo, hi = t[0], t[-1]
    ok = fin & (cx + lo >= 0) & (cx + hi <= N - 1) & (cy + lo >= 0) & (cy + hi <= N - 1)
    w = np.asarray(weights)
    valid = ok & (w != 0)
    return cx, cy, rx, ry, valid


# ------------------------------------------------------------------- grid / degrid
class Geometry:
    """Everything the scatter needs that depends only on uvw, frequencies and flags."""

    def __init__(self, uvw_m, freq_hz, weights, N, du, W=7, OS=8, beta=None, conjugate=False):
        self.N, self.W, self.OS = int(N), int(W), int(OS)
        self.beta = default_beta(W) if beta is None or beta <= 0 else float(beta)
        self.tab = table(self.W, self.OS, self.beta)
        self.r, self.t = phase_range(self.W, self.OS)
        self.copies = [coords(uvw_m, freq_hz, weights, N, du, W, OS, False)]
        if conjugate:
            self.copies.append(coords(uvw_m, freq_hz, weights, N, du, W, OS, True))
        self.C = len(freq_hz)

    @property
    def valid(self):
        return self.copies[0][4]

    def _taps(self, k):
        cx, cy, rx, ry, valid = self.copies[k]
        c = np.broadcast_to(np.arange(self.C)[:, None, None], cx.shape)[valid]
        kx = self.tab[(rx - self.r[0])[valid]]        # [n][W]
        ky = self.tab[(ry - self.r[0])[valid]]
        return c, cx[valid], cy[valid], kx, ky, valid


def grid(geom: Geometry, vis, weights) -> np.ndarray:
    """Eq. (1) in scatter form: G[c][cy+ty][cx+tx] += w V k_y k_x over valid samples.

    With a conjugate copy, conj(V) is also gridded at (-u, -v).  Output overwritten.
    """
    N, t = geom.N, geom.t
    G = np.zeros((geom.C, N, N), np.complex128)
    vis = np.asarray(vis, np.complex128)
    w = np.asarray(weights, np.float64)
    for k in range(len(geom.copies)):
        c, cx, cy, kx, ky, valid = geom._taps(k)
        a = (w * vis)[valid]
        if k == 1:
            a = np.conj(a)
        for jy, ty in enumerate(t):
            for jx, tx in enumerate(t):
                np.add.at(G, (c, cy + ty, cx + tx), a * ky[:, jy] * kx[:, jx])
    return G


def degrid(geom: Geometry, G, copy: int = 0) -> np.ndarray:
    """Adjoint of gridding (no weights): M = sum over taps of k_y k_x G at the sample.

    Uses the +uv copy only; invalid samples predict 0.  ``copy=1`` evaluates the
    prediction at the conjugate positions (-u, -v), used for the adjoint check.
    """
    t = geom.t
    c, cx, cy, kx, ky, valid = geom._taps(copy)
    m = np.zeros(valid.shape, np.complex128)
    acc = np.zeros(c.shape, np.complex128)
    for jy, ty in enumerate(t):
        for jx, tx in enumerate(t):
            acc += ky[:, jy] * kx[:, jx] * G[c, cy + ty, cx + tx]
    m[valid] = acc
    return m


def grid_degrid(geom: Geometry, vis, weights, G_in):
    """Fused residual step: M = degrid(G_in); r = V - M; G_out = grid(r); chi2 = sum w |r|^2.

    Returns (M, G_out, chi2, r); r is zero for invalid samples.
    """
    M = degrid(geom, G_in)
    valid = geom.valid
    r = np.where(valid, np.asarray(vis, np.complex128) - M, 0.0)
    G_out = grid(geom, r, weights)
    w = np.asarray(weights, np.float64)
    chi2 = float(np.sum(np.where(valid, w * np.abs(r) ** 2, 0.0)))
    return M, G_out, chi2, r


def grid_adjoint(geom: Geometry, y, weights) -> np.ndarray:
    """Adjoint of ``grid`` w.r.t. the real inner product Re<.,.>: w (D+ y + conj(D- y)).

    Without a conjugate copy it is w * degrid(y).
    """
    w = np.asarray(weights, np.float64)
    out = degrid(geom, y, 0)
    if len(geom.copies) > 1:
        out = out + np.conj(degrid(geom, y, 1))
    return np.where(geom.valid, w * out, 0.0)


# -------------------------------------------------------------------- gradients
def chi2_gradients(geom: Geometry, vis, weights, G):
    """Gradients of L = sum w |V - degrid(G)|^2 (PyTorch convention dL/dRe + i dL/dIm).

    dL/dG = -2 grid(r, w); dL/dw = |r|^2; dL/dV = 2 w r (zero where invalid).
    """
    M, G_out, chi2, r = grid_degrid(geom, vis, weights, G)
    w = np.asarray(weights, np.float64)
    gG = -2.0 * G_out
    gw = np.where(geom.valid, np.abs(r) ** 2, 0.0)
    gV = np.where(geom.valid, 2.0 * w * r, 0.0)
    return chi2, gG, gw, gV


def grid_vjp(geom: Geometry, vis, weights, gG):
    """Vector-Jacobian product of G = grid(V, w) for an upstream gradient gG.

    dL/dV = w * degrid(gG); dL/dw = Re(conj(V) degrid(gG)) (zero where invalid).
    """
    d = degrid(geom, gG)
    w = np.asarray(weights, np.float64)
    v = np.asarray(vis, np.complex128)
    gV = np.where(geom.valid, w * d, 0.0)
    gw = np.where(geom.valid, np.real(np.conj(v) * d), 0.0)
    return gV, gw


# ------------------------------------------------------------ brute-force checks
def gather_grid(uvw_m, freq_hz, vis, weights, N, du, W, OS, beta=None, conjugate=False):
    """Section 5.2 naive gather: every pixel scans every visibility.

    Uses the closed-form kernel at the distance from the snapped position
    xs/OS to the pixel centre, with no phase table and no cell split, so it checks
    the table and the tap bookkeeping of ``grid``.  Tiny inputs only.
    """
    beta = default_beta(W) if beta is None or beta <= 0 else beta
    G = np.zeros((len(freq_hz), N, N), np.complex128)
    pix = np.arange(N, dtype=np.float64)
    copies = [False, True] if conjugate else [False]
    for conj in copies:
        _, _, _, _, valid = coords(uvw_m, freq_hz, weights, N, du, W, OS, conj)
        xs, ys, _ = snapped(uvw_m, freq_hz, N, du, OS, conj)
        for c in range(len(freq_hz)):
            sel = valid[c]
            xq = xs[c][sel] / OS
            yq = ys[c][sel] / OS
            a = (np.asarray(weights, np.float64)[c] * np.asarray(vis, np.complex128)[c])[sel]
            if conj:
                a = np.conj(a)
            for py in range(N):
                ky = kb(py - yq, W, beta)
                if not np.any(ky):
                    continue
                kx = kb(pix[:, None] - xq[None, :], W, beta)     # [N][n]
                G[c, py] += kx @ (a * ky)
    return G


def image(G, W: int, beta: float) -> np.ndarray:
    """Grid -> dirty image: centred inverse FFT scaled by N^2, divided by the
    separable grid correction khat(nu_x) khat(nu_y), nu = (q - N/2)/N."""
    N = G.shape[-1]
    img = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(G, axes=(-2, -1))), axes=(-2, -1)) * (N * N)
    nu = (np.arange(N) - N // 2) / N
    corr = kb_hat(nu, W, beta)
    return img / (corr[:, None] * corr[None, :])


def direct_dft(xs_snapped, ys_snapped, a, N, OS, region):
    """I(l, m) = sum_i a_i exp(+2 pi i (u_q l + v_q m)) on image pixels ``region``
    (iterable of (qy, qx)), with u_q = (xs/OS - N/2) du and l = (qx - N/2)/(N du);
    du cancels.  Brute force over all samples."""
    xq = xs_snapped / OS - N / 2
    yq = ys_snapped / OS - N / 2
    out = np.empty(len(region), np.complex128)
    for k, (qy, qx) in enumerate(region):
        ph = 2.0 * np.pi * (xq * (qx - N / 2) + yq * (qy - N / 2)) / N
        out[k] = np.sum(a * np.exp(1j * ph))
    return out


# ------------------------------------------------------- polarisation conversion
def polconvert(A, P) -> np.ndarray:
    """Section 3, the polarisation convertor stage: for every pixel i, S_i = A_i P_i,
    where P_i holds the four observed polarisation products of the pixel, A_i is a
    4x4 complex matrix (supplied by a precomputation) and S_i the converted vector.

    A: complex [4][4][n_pix], one matrix per pixel shared by every channel, or
    [C][4][4][n_pix], one per channel and pixel.  P: complex [C][4][n_pix].
    Returns complex128 S [C][4][n_pix] with S[c][r][i] = sum_k A[r][k][i] P[c][k][i]."""
    P = np.asarray(P, np.complex128)
    A = np.asarray(A, np.complex128)
    C = P.shape[0]
    S = np.zeros(P.shape, np.complex128)
    for c in range(C):
        Ac = A if A.ndim == 3 else A[c]
        for r in range(4):
            for k in range(4):
                S[c, r] += Ac[r, k] * P[c, k]
    return S


# ------------------------------------------- per-visibility (per-baseline) kernels
def _baseline_taps(geom: Geometry, k: int, bl_tab):
    """Like Geometry._taps, but each sample's kernel rows come from the table of its
    baseline: bl_tab[b] is [OS][W] in the phase / tap layout of ``table``."""
    cx, cy, rx, ry, valid = geom.copies[k]
    tab = np.asarray(bl_tab, np.float64)
    c = np.broadcast_to(np.arange(valid.shape[0])[:, None, None], valid.shape)[valid]
    b = np.broadcast_to(np.arange(valid.shape[1])[None, :, None], valid.shape)[valid]
    r0 = geom.r[0]
    kx = tab[b, (rx - r0)[valid]]                 # [n][W]
    ky = tab[b, (ry - r0)[valid]]
    return c, cx[valid], cy[valid], kx, ky, valid


def grid_per_baseline(geom: Geometry, vis, weights, bl_tab) -> np.ndarray:
    """Eq. (1) with a kernel specific to each visibility (Section 3, the gridder: the
    kernel follows from the calibration of the two tiles of the visibility's
    baseline; Table 4 uses a 24 x 24 kernel).  READING: the kernel of baseline b is
    separable, the same along u and v and across channels, and given sampled as
    bl_tab[b][p][j] = k_b(t_j - r_p / OS) (the layout of ``table``):
    G[c][cy+t_v][cx+t_u] += w V bl_tab[b][r_y][t_v] bl_tab[b][r_x][t_u].
    Conjugate copies use their baseline's table at their own phases."""
    N, t = geom.N, geom.t
    G = np.zeros((geom.C, N, N), np.complex128)
    vis = np.asarray(vis, np.complex128)
    w = np.asarray(weights, np.float64)
    for k in range(len(geom.copies)):
        c, cx, cy, kx, ky, valid = _baseline_taps(geom, k, bl_tab)
        a = (w * vis)[valid]
        if k == 1:
            a = np.conj(a)
        for jy, ty in enumerate(t):
            for jx, tx in enumerate(t):
                np.add.at(G, (c, cy + ty, cx + tx), a * ky[:, jy] * kx[:, jx])
    return G


def degrid_per_baseline(geom: Geometry, G, bl_tab) -> np.ndarray:
    """Adjoint of grid_per_baseline without weights (the +uv copy; invalid samples
    predict 0): M = sum over taps of bl_tab[b][r_y][t_v] bl_tab[b][r_x][t_u] G."""
    t = geom.t
    c, cx, cy, kx, ky, valid = _baseline_taps(geom, 0, bl_tab)
    m = np.zeros(valid.shape, np.complex128)
    acc = np.zeros(c.shape, np.complex128)
    for jy, ty in enumerate(t):
        for jx, tx in enumerate(t):
            acc += ky[:, jy] * kx[:, jx] * G[c, cy + ty, cx + tx]
    m[valid] = acc
    return m
