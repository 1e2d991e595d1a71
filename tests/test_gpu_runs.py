"""Runs of equal snapped positions inside a segment, against the FP64 oracle.

Consecutive samples of a track that snap to the same oversampled position have
the same kernel rows; the tile kernel degrids such a run once and grids its summed
weighted (residual) visibility with one outer product (Eq. (1) regrouped).  These
cases force the run shapes a four- or eight-sample segment can have: one run, two,
alternating positions (A B A B ...: a run per sample), flagged samples inside,
before and after a run, an all-flagged track, and a second position one cell
away on either axis (the window's last column or row is then reached and must be
added by the flush).  Both tile sizes (128- and 512-thread workgroups) and the
-uv copy of gridding are covered.

Bar: relative L2 1e-5 per channel against the oracle (grid, degrid, fused grid
and model, chi-squared); model values of flagged samples exactly 0.
"""
import numpy as np
import pytest

import oracle as O
from tests.gpu_helpers import RTOL_L2, rel_l2, small_case, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 256
N_PATTERNS = 10


@pytest.fixture(scope="module")
def rts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_5575_amd as rts
    rts._lib.load()
    return rts


def shaped_tracks(wl, freq, du, seed):
    """Rewrite each baseline's track into one of N_PATTERNS run shapes (baseline
    index mod N_PATTERNS) built from two positions A (the track's first sample) and
    B (A moved by a fraction of a cell, or by one whole cell on one axis), with
    weights U(0.5, 1.5) and the pattern's flags."""
    uvw = wl.uvw_m.copy()
    B, T = uvw.shape[0], uvw.shape[1]
    cell_m = du * O.C_LIGHT / float(np.mean(freq))       # one cell in metres, mid band
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, (len(freq), B, T)).astype(np.float32)
    for b in range(B):
        p = b % N_PATTERNS
        A = uvw[b, 0].copy()
        step = {8: (1.0, 0.0), 9: (0.0, 1.0)}.get(p, (0.45, 0.3))
        Bp = A + np.array([step[0] * cell_m, step[1] * cell_m, 0.0])
        if p == 3:
            continue                                     # natural motion
        seq = {0: "A" * T, 1: "A" * (T // 2) + "B" * (T - T // 2), 2: "AB" * (T // 2) + "A" * (T % 2),
               4: "A" * (T - 1) + "B", 5: "A" * T, 6: "A" + "B" * (T - 1), 7: "AB" * (T // 2) + "A" * (T % 2),
               8: "AABB" * (T // 4) + "A" * (T % 4), 9: "ABBA" * (T // 4) + "A" * (T % 4)}[p]
        for t, ch in enumerate(seq):
            uvw[b, t] = A if ch == "A" else Bp
        if p == 4:
            w[:, b, 1] = 0.0                             # flagged inside a run
        elif p == 5:
            w[:, b, 0] = 0.0                             # flagged before the run
        elif p == 6:
            w[:, b, T - 2:] = 0.0                        # flagged at the end
        elif p == 7:
            w[:, b, :] = 0.0                             # all flagged
    return uvw, w


def run_counts(uvw, freq, w, du, OS=8):
    """Runs per track of channel 0 (oracle coordinates): maximal stretches of valid
    samples with one snapped position."""
    xs, ys, fin = O.snapped(uvw, freq[:1], N, du, OS)
    valid = (w[0] != 0) & fin[0]
    key = xs[0] * (1 << 24) + ys[0]
    n = np.zeros(uvw.shape[0], int)
    last = np.full(uvw.shape[0], -1, np.int64)
    for t in range(uvw.shape[1]):
        new = valid[:, t] & (key[:, t] != last)
        n += new
        last = np.where(valid[:, t], key[:, t], last)
    return n


@pytest.mark.parametrize("name,tile", [("batched", 64), ("batched", 32), ("single_cadence", 64)])
def test_run_shapes_match_oracle(rts, name, tile):
    channels = (0, 383, 767) if name == "batched" else (0, 13, 31)
    wl, freq, du = small_case(name, seed=4, n_ant=40, channels=channels, N=N)
    T = wl.n_time
    uvw_np, w_np = shaped_tracks(wl, freq, du, seed=11)
    runs = run_counts(uvw_np, freq, w_np, du)
    assert (runs == 1).any() and (runs == 0).any() and (runs == T).any() and (runs == 2).any()
    wl.uvw_m, wl.weights = uvw_np, w_np
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, tile=tile)
    assert plan.info["tile"] == tile
    rng = np.random.default_rng(6)
    gin_np = (0.1 * (rng.standard_normal((len(freq), N, N)) + 1j * rng.standard_normal((len(freq), N, N)))
              ).astype(np.complex64)
    gin = torch.from_numpy(gin_np).cuda()
    G = plan.grid(vis, w).cpu().numpy()
    M = plan.degrid(gin).cpu().numpy()
    Mf, Gf, chi2 = (x.cpu().numpy() for x in plan.grid_degrid(vis, w, gin))
    geom = O.Geometry(uvw_np, freq, w_np, N, du)
    Gref = O.grid(geom, wl.vis, w_np)
    Mref = O.degrid(geom, gin_np.astype(np.complex128))
    Mo, Go, chi2o, _ = O.grid_degrid(geom, wl.vis, w_np, gin_np.astype(np.complex128))
    assert np.all(M[~geom.valid] == 0) and np.all(Mf[~geom.valid] == 0)
    for c in range(len(freq)):
        assert rel_l2(G[c], Gref[c]) <= RTOL_L2, ("grid", c)
        assert rel_l2(M[c], Mref[c]) <= RTOL_L2, ("degrid", c)
        assert rel_l2(Gf[c], Go[c]) <= RTOL_L2, ("fused grid", c)
        assert rel_l2(Mf[c], Mo[c]) <= RTOL_L2, ("fused model", c)
    assert abs(float(chi2) - chi2o) <= RTOL_L2 * abs(chi2o)


def test_run_shapes_conjugate_gridding(rts):
    """Gridding with the -uv copy: each copy's runs are found from its own
    coordinates, and the copy adds the conjugate of its summed weighted
    visibility."""
    wl, freq, du = small_case("batched", seed=5, n_ant=40, channels=(0, 767), N=N)
    uvw_np, w_np = shaped_tracks(wl, freq, du, seed=12)
    wl.uvw_m, wl.weights = uvw_np, w_np
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, conjugate=True)
    G = plan.grid(vis, w).cpu().numpy()
    Gref = O.grid(O.Geometry(uvw_np, freq, w_np, N, du, conjugate=True), wl.vis, w_np)
    for c in range(len(freq)):
        assert rel_l2(G[c], Gref[c]) <= RTOL_L2, c
