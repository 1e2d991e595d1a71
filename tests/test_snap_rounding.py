"""Snapping samples whose u s + N/2 sits at a rounding midpoint next to a phase boundary.

The snapped coordinate is xs = floor(x OS + 1/2) with x = u s + N/2, each step
rounded once (the oracle's reading of the uv -> grid conversion).  Evaluated as
one fused multiply-add, x is rounded once instead of twice, and for samples whose
exact u s + N/2 lies within the product's rounding error of a midpoint between
two doubles that straddle x* = (m - 1/2) / OS, the two evaluations land on
different sides of x* and the sample snaps to a neighbouring phase.  Random
inputs hit such a sample about once in 1e12; the inputs here are searched for
on purpose (exact rational arithmetic for the fused value), so an implementation
that contracts the two steps fails them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

N, OS, W, DU = 256, 8, 7, 2.0
FREQ = 150e6


def _sep(u, s):
    x = u * s + N / 2                          # Python floats: two roundings
    return math.floor(x * OS + 0.5)


def _fused(u, s):
    x = float(Fraction(u) * Fraction(s) + Fraction(N // 2))   # one rounding
    return math.floor(x * OS + 0.5)


def boundary_samples(s, count):
    """u values (metres) near phase boundaries where the two evaluations differ."""
    out = []
    for m in range(8 * 100, 8 * 156):
        u0 = ((m - 0.5) / OS - N / 2) / s
        for direction in (np.inf, -np.inf):
            u = u0
            for _ in range(2000):
                if _sep(u, s) != _fused(u, s):
                    out.append(u)
                    break
                u = float(np.nextafter(u, direction))
        if len(out) >= count:
            break
    return out[:count]


def _scale():
    return FREQ / (O.C_LIGHT * DU)


def _uvw(us):
    """One time step per baseline: the searched values on u, and on v for the second half."""
    n = len(us)
    uvw = np.zeros((2 * n, 1, 3))
    uvw[:n, 0, 0] = us
    uvw[n:, 0, 1] = us
    uvw[:n, 0, 1] = 3.7                        # keep the other axis away from boundaries
    uvw[n:, 0, 0] = -5.3
    return uvw


def test_boundary_samples_pin_the_oracle_to_two_roundings():
    """The oracle's snapped coordinates are the two-rounding values on every
    searched sample, which the one-rounding evaluation misses."""
    s = _scale()
    us = boundary_samples(s, 24)
    assert len(us) == 24
    xs, ys, fin = O.snapped(_uvw(us), [FREQ], N, DU, OS)
    n = len(us)
    assert fin.all()
    for i, u in enumerate(us):
        assert xs[0, i, 0] == _sep(u, s) != _fused(u, s)
        assert ys[0, n + i, 0] == _sep(u, s)


@pytest.mark.gpu
def test_gpu_snapping_matches_oracle_at_rounding_midpoints():
    """The library's coordinates (rts_compute_coords) and the plan's gridding
    (which snaps in its own kernels) agree with the oracle on the searched
    samples: bit-exact coordinates, and a grid within the FP32 bound (a sample
    snapped to a neighbouring phase would move its weights by a sixteenth of a
    cell and the grid by about 1e-2 relative)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_5575_amd as rts
    from tests.gpu_helpers import RTOL_L2, rel_l2
    us = boundary_samples(_scale(), 24)
    uvw = _uvw(us)
    B = uvw.shape[0]
    w = np.ones((1, B, 1), np.float32)
    rng = np.random.default_rng(5)
    vis = (rng.standard_normal((1, B, 1)) + 1j * rng.standard_normal((1, B, 1))).astype(np.complex64)
    dev = torch.device("cuda:0")
    uvw_d = torch.from_numpy(uvw).to(dev)
    w_d = torch.from_numpy(w).to(dev)
    out = rts.compute_coords(uvw_d, [FREQ], w_d, N, DU, W, OS).cpu().numpy()
    xs, ys, fin = O.snapped(uvw, [FREQ], N, DU, OS)
    assert np.array_equal(out[..., 0], xs) and np.array_equal(out[..., 1], ys)
    plan = rts.GridPlan(uvw_d, [FREQ], w_d, N, DU, support=W, oversample=OS)
    G = plan.grid(torch.from_numpy(vis).to(dev), w_d).cpu().numpy()
    ref = O.grid(O.Geometry(uvw, [FREQ], w, N, DU, W, OS), vis, w)
    assert rel_l2(G[0], ref[0]) <= RTOL_L2
