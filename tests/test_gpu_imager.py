"""Imager (grid -> dirty image, the step after gridding) against the FP64 oracle.

The oracle's image is pinned in tests/test_oracle_pins.py against a brute-force
direct DFT; here the GPU image (hipFFT batched inverse transform between the
library's sign and grid-correction passes) must match it per channel, for odd and
even supports, in place (quadrant-swap pass after transforming the grid
itself) and out of place (sign pass into the output, transform, correction).

Bounds (relative L2 per channel):
  * central region |nu_x|, |nu_y| <= 1/4: <= 1e-5.  There the correction divides
    by khat(nu) >= 0.12 khat(0) (W = 16; 0.55 at W = 7), so FP32 rounding of the
    transform is amplified at most eightfold.
  * whole field with the correction undone on both sides (multiplied back by the
    exact FP64 khat(nu_y) khat(nu_x)): <= 1e-5.  This checks the transform, the
    two centring sign passes and every correction value over all pixels, without
    the division by khat values down to 1e-4 of khat(0) at the field edge (W = 16),
    which lifts the single-precision rounding of any FP32 implementation there.
"""
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


@pytest.mark.parametrize("W,OS,N,conj", [(7, 8, 256, True), (8, 8, 128, False), (16, 16, 256, True)])
def test_image_matches_oracle(rts, W, OS, N, conj):
    wl, freq, du = small_case(n_ant=40, channels=(0, 13, 31), N=N, W=W, OS=OS, weights="uniform", flag_frac=0.1)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, support=W, oversample=OS, conjugate=conj)
    G = plan.grid(vis, w)
    img = plan.image(G).cpu().numpy()
    H = G.clone()
    img_ip = plan.image(H, out=H).cpu().numpy()      # in place: quadrant-swap pass
    G64 = G.cpu().numpy().astype(np.complex128)
    ref = O.image(G64, W, O.default_beta(W))
    # A plain complex64 CPU pipeline of the same operation (numpy's FFT in single
    # precision) is printed beside the GPU errors for comparison.
    nu = (np.arange(N) - N // 2) / N
    corr = O.kb_hat(nu, W, O.default_beta(W)).astype(np.float32)
    G32 = G.cpu().numpy()
    ref32 = (np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(G32, axes=(-2, -1)).astype(np.complex64)).astype(np.complex64),
                             axes=(-2, -1)) * np.float32(N * N)) / (corr[:, None] * corr[None, :])
    q = slice(N // 4, 3 * N // 4 + 1)                    # |nu| <= 1/4
    k64 = O.kb_hat(nu, W, O.default_beta(W))
    kk = k64[:, None] * k64[None, :]
    for c in range(len(freq)):
        e32 = rel_l2(ref32[c], ref[c])
        for name, im in (("out of place", img), ("in place", img_ip)):
            err = rel_l2(im[c], ref[c])
            err_c = rel_l2(im[c][q, q], ref[c][q, q])
            err_u = rel_l2(im[c] * kk, ref[c] * kk)
            print(f"imager W={W} N={N} channel {c} {name}: central {err_c:.2e}, uncorrected {err_u:.2e}, "
                  f"whole field {err:.2e} (complex64 CPU FFT: {e32:.2e})")
            assert err_c <= RTOL_L2, f"channel {c} {name}: central region"
            assert err_u <= RTOL_L2, f"channel {c} {name}: whole field without the correction"
    if conj:
        # Hermitian grid -> real image.  Checked on the central half of the field:
        # towards the edges the grid correction divides by khat values down to
        # 1e-4 of khat(0) (W=16), which lifts single-precision rounding there.
        q = slice(N // 4, 3 * N // 4)
        inner = img[:, q, q]
        assert np.linalg.norm(inner.imag) <= 1e-5 * np.linalg.norm(inner.real)


@pytest.mark.parametrize("N,tile", [(128, 0), (132, 12), (130, 10)])
def test_image_in_place_and_repeat(rts, N, tile):
    """Repeated calls are bitwise identical.  In place, N a multiple of 4 takes the
    quadrant-swap pass after transforming the grid itself; N = 130 (N/2 odd) keeps
    the sign pass, run in place.  Both orders of evaluation are FP32 rounding of
    the same sum: in place and out of place agree to 1e-6 relative L2 on the
    central region |nu| <= 1/4 (the whole field differs by a few 1e-6, where the
    correction divides by small khat values at the edge), and the in place image
    matches the oracle's on the central region and, with the correction undone,
    over the whole field, to 1e-5."""
    wl, freq, du = small_case(n_ant=32, channels=(4, 20), N=N, W=7, OS=8)
    uvw, vis, w = to_dev(torch, wl)
    plan = rts.GridPlan(uvw, freq, w, N, du, tile=tile) if tile else rts.GridPlan(uvw, freq, w, N, du)
    G = plan.grid(vis, w)
    a = plan.image(G).cpu().numpy()
    b = plan.image(G).cpu().numpy()
    assert np.array_equal(a, b)
    H = G.clone()
    plan.image(H, out=H)
    h = H.cpu().numpy()
    q = slice(N // 4, 3 * N // 4 + 1)
    assert rel_l2(h[:, q, q], a[:, q, q]) <= 1e-6
    H2 = G.clone()
    plan.image(H2, out=H2)
    assert np.array_equal(H2.cpu().numpy(), h)
    ref = O.image(G.cpu().numpy().astype(np.complex128), 7, O.default_beta(7))
    k64 = O.kb_hat((np.arange(N) - N // 2) / N, 7, O.default_beta(7))
    kk = k64[:, None] * k64[None, :]
    for c in range(len(freq)):
        assert rel_l2(h[c][q, q], ref[c][q, q]) <= RTOL_L2
        assert rel_l2(h[c] * kk, ref[c] * kk) <= RTOL_L2


def test_point_source_image_peaks_at_its_pixel(rts):
    """One visibility of a unit point source at pixel (qy, qx) on every baseline:
    the image peaks at that pixel."""
    from synth import make_workload
    N, W = 256, 7
    wl = make_workload("tiny", seed=3)
    freq = wl.freq_hz[wl.channels]
    du = wl.cell_lambda
    qy, qx = N // 2 + 9, N // 2 - 14
    l, m = (qx - N // 2) / (N * du), (qy - N // 2) / (N * du)
    lam = O.C_LIGHT / freq[0]
    u = wl.uvw_m[:, :, 0] / lam
    v = wl.uvw_m[:, :, 1] / lam
    vis = np.exp(-2j * np.pi * (u * l + v * m))[None].astype(np.complex64)
    weights = np.ones_like(vis.real, dtype=np.float32)
    dev = torch.device("cuda:0")
    uvw_d = torch.from_numpy(np.ascontiguousarray(wl.uvw_m)).to(dev)
    plan = rts.GridPlan(uvw_d, freq, torch.from_numpy(weights).to(dev), N, du, support=W, oversample=8, conjugate=True)
    G = plan.grid(torch.from_numpy(vis).to(dev), torch.from_numpy(weights).to(dev))
    img = plan.image(G).cpu().numpy()[0].real
    assert np.unravel_index(np.argmax(img), img.shape) == (qy, qx)
