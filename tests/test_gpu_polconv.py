"""Polarisation conversion S_i = A_i P_i (rts_polconvert) against the FP64 oracle.

The oracle is pinned in tests/test_oracle_pins.py (identity, Stokes recovery from
linear feeds, composition, per-channel matrices, pixel independence).  Bound per
element: each output is a sum of four complex products computed in FP32 from
complex64 inputs; a complex product and each addition round with relative error
at most 2^-24 per real operation, so |S - S_ref| <= 8 * 2^-24 * sum_k |A_rk| |P_k|
(about 4.8e-7 of the magnitudes), which the test uses with a margin of 2."""
import numpy as np
import pytest

import oracle as O
from synth import make_polconv_inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def rts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_5575_amd as rts
    rts._lib.load()
    return rts


def check(S, A, P):
    """Element-wise comparison with the oracle within the FP32 bound."""
    n = P.shape[-1]
    A4 = A.reshape(A.shape[:-2] + (4, 4, n))
    ref = O.polconvert(A4, P)
    absA = np.abs(A4.astype(np.complex128))
    absP = np.abs(P.astype(np.complex128))
    mag = np.zeros(ref.shape)
    for c in range(P.shape[0]):
        Ac = absA if absA.ndim == 3 else absA[c]
        for r in range(4):
            for k in range(4):
                mag[c, r] += Ac[r, k] * absP[c, k]
    err = np.abs(S.astype(np.complex128) - ref)
    assert np.all(err <= 2 * 8 * U32 * mag + 1e-30), float(np.max(err / (mag + 1e-30)))


@pytest.mark.parametrize("n_pix,C", [(4096, 3), (4095, 3), (1, 1), (2, 5), (70001, 2)])
def test_polconvert_matches_oracle(rts, n_pix, C):
    """Even counts take the two-pixel path, odd counts the one-pixel path; 70001
    spans many workgroups with a ragged tail."""
    A, P = make_polconv_inputs(n_pix, C, seed=n_pix)
    S = rts.polconvert(torch.from_numpy(A).cuda(), torch.from_numpy(P).cuda()).cpu().numpy()
    check(S, A, P)


def test_polconvert_per_channel_matrices(rts):
    A, P = make_polconv_inputs(3000, 4, seed=7, per_channel=True)
    S = rts.polconvert(torch.from_numpy(A).cuda(), torch.from_numpy(P).cuda()).cpu().numpy()
    check(S, A, P)


def test_polconvert_in_place_and_misaligned(rts):
    A, P = make_polconv_inputs(2000, 2, seed=3)
    Ad = torch.from_numpy(A).cuda()
    Pd = torch.from_numpy(P).cuda()
    out = rts.polconvert(Ad, Pd, out=Pd)           # in place
    assert out.data_ptr() == Pd.data_ptr()
    check(Pd.cpu().numpy(), A, P)
    # planes that start 8 bytes past a 16-byte boundary take the one-pixel path
    n = 1999
    A2, P2 = make_polconv_inputs(n, 2, seed=4)
    bufA = torch.zeros(16 * n + 1, dtype=torch.complex64, device="cuda")
    bufP = torch.zeros(2 * 4 * n + 1, dtype=torch.complex64, device="cuda")
    Av = bufA[1:].view(16, n)
    Pv = bufP[1:].view(2, 4, n)
    Av.copy_(torch.from_numpy(A2))
    Pv.copy_(torch.from_numpy(P2))
    assert Av.data_ptr() % 16 == 8
    S = rts.polconvert(Av, Pv).cpu().numpy()
    check(S, A2, P2)


def test_polconvert_recovers_stokes(rts):
    """With the unperturbed linear-feed inverse, the output is the sky's Stokes
    images (I, Q, U, V) to FP32 rounding."""
    n = 5000
    _, P = make_polconv_inputs(n, 2, seed=9)
    M = np.array([[0.5, 0, 0, 0.5], [0.5, 0, 0, -0.5], [0, 0.5, 0.5, 0], [0, -0.5j, 0.5j, 0]], np.complex64)
    A = np.repeat(M.reshape(16, 1), n, axis=1)
    S = rts.polconvert(torch.from_numpy(A).cuda(), torch.from_numpy(P).cuda()).cpu().numpy()
    P64 = P.astype(np.complex128)
    I = (P64[:, 0] + P64[:, 3]) / 2
    V = (P64[:, 1] - P64[:, 2]) / 2j
    np.testing.assert_allclose(S[:, 0], I, rtol=0, atol=4 * U32 * np.abs(P64).max())
    np.testing.assert_allclose(S[:, 3], V, rtol=0, atol=4 * U32 * np.abs(P64).max())


def test_polconvert_full_size_sampled(rts):
    """The bench configuration (12 channels of 1125 x 1125 pixels, one matrix set):
    sampled pixels against the oracle evaluated on those pixels only."""
    n, C = 1125 * 1125, 12
    A, P = make_polconv_inputs(n, C, seed=21)
    S = rts.polconvert(torch.from_numpy(A).cuda(), torch.from_numpy(P).cuda()).cpu().numpy()
    idx = np.random.default_rng(0).choice(n, 4000, replace=False)
    idx = np.concatenate([idx, [0, 1, n - 2, n - 1]])
    check(S[..., idx], A[..., idx], P[..., idx])


def test_polconvert_empty(rts):
    A = torch.zeros((16, 0), dtype=torch.complex64, device="cuda")
    P = torch.zeros((3, 4, 0), dtype=torch.complex64, device="cuda")
    assert rts.polconvert(A, P).shape == (3, 4, 0)


@pytest.mark.parametrize("gap", [0, 2, 3])
def test_polconvert_channel_stride_through_the_abi(rts, gap):
    """Per-channel matrix blocks a_chan_stride = 16 n + gap complex elements apart
    (gap 3 makes the stride odd: the one-pixel path), called through the C ABI."""
    n, C = 1000, 3
    A, P = make_polconv_inputs(n, C, seed=30 + gap, per_channel=True)
    stride = 16 * n + gap
    buf = torch.zeros(C * stride, dtype=torch.complex64, device="cuda")
    for c in range(C):
        buf[c * stride:c * stride + 16 * n] = torch.from_numpy(A[c].ravel()).cuda()
    Pd = torch.from_numpy(P).cuda()
    S = torch.empty_like(Pd)
    lib = rts._lib.load()
    st = lib.rts_polconvert(buf.data_ptr(), Pd.data_ptr(), S.data_ptr(), n, C, stride, None)
    torch.cuda.synchronize()
    assert st == 0
    check(S.cpu().numpy(), A, P)
