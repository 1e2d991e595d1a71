"""Seeded inputs for the polarisation conversion stage: per-pixel 4x4 complex
matrices and four observed polarisation products per pixel and channel.

Only inputs are built here; the conversion itself (S = A P) is not.
"""
from __future__ import annotations

import numpy as np


def make_polconv_inputs(n_pix: int, n_chan: int, seed: int = 0, per_channel: bool = False, spread: float = 0.05):
    """Returns (A, P) as complex64 arrays.

    A: [16][n_pix] (or [n_chan][16][n_pix] with ``per_channel``): entry r*4+k of
    each pixel's matrix, the linear-feed to Stokes transform plus a seeded
    direction-dependent perturbation of relative size ``spread``.
    P: [n_chan][4][n_pix]: XX, XY, YX, YY of a sky of point sources on a noise
    floor (I > 0, |Q|, |U|, |V| up to 30% of I), XX = I + Q, XY = U + iV,
    YX = U - iV, YY = I - Q.
    """
    rng = np.random.default_rng(seed)
    base = np.array([[0.5, 0, 0, 0.5], [0.5, 0, 0, -0.5], [0, 0.5, 0.5, 0], [0, -0.5j, 0.5j, 0]],
                    np.complex128).reshape(16, 1)

    def matrices():
        pert = rng.standard_normal((16, n_pix)) + 1j * rng.standard_normal((16, n_pix))
        return (base + spread * 0.5 * pert).astype(np.complex64)

    A = np.stack([matrices() for _ in range(n_chan)]) if per_channel else matrices()
    P = np.empty((n_chan, 4, n_pix), np.complex64)
    n_src = max(1, n_pix // 5000)
    for c in range(n_chan):
        I = np.abs(rng.normal(0.01, 0.005, n_pix))
        idx = rng.integers(0, n_pix, n_src)
        I[idx] += rng.uniform(0.5, 5.0, n_src)
        frac = rng.uniform(-0.3, 0.3, (3, n_pix))
        Q, U, V = frac[0] * I, frac[1] * I, frac[2] * I
        P[c, 0] = I + Q
        P[c, 1] = U + 1j * V
        P[c, 2] = U - 1j * V
        P[c, 3] = I - Q
    return A, P
