"""Seeded per-baseline gridding kernels (stand-ins for kernels derived from the
calibration of each baseline's two tiles): smooth positive bumps of per-baseline
width, tapered to zero at the edges of the support.

Only the caller-side table values are built here, in the [B][OS][W] layout the
library takes (row p: kernel phase p, column j: tap j); how a table is applied
to the visibilities is not.
"""
from __future__ import annotations

import numpy as np


def make_baseline_kernels(n_base: int, W: int, OS: int, seed: int = 0) -> np.ndarray:
    """float32 [n_base][OS][W]: tab[b][p][j] = exp(-x^2 / (2 s_b^2)) cos^2(pi x),
    x = (j + 0.5 - p / OS) / W - 0.5, with s_b ~ U(0.12, 0.25) per baseline."""
    rng = np.random.default_rng(seed)
    s = rng.uniform(0.12, 0.25, n_base)
    j = np.arange(W)[None, :]
    p = np.arange(OS)[:, None]
    x = (j + 0.5 - p / OS) / W - 0.5                      # [OS][W]
    bump = np.exp(-(x[None] ** 2) / (2.0 * s[:, None, None] ** 2)) * np.cos(np.pi * x)[None] ** 2
    return bump.astype(np.float32)
