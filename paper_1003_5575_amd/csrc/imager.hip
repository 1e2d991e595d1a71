// Imager: uv grid -> dirty image for every channel (the imaging step that
// follows gridding in the paper's pipeline, Section 3).  The image is the
// centred inverse 2-D FFT of the grid divided by the separable grid correction
// khat(nu_x) khat(nu_y), nu = (q - N/2) / N, where khat is the Fourier transform
// of the gridding kernel.  For even N the centring shifts are folded into sign
// factors: with s(x, y) = (-1)^(x+y), shift(IFFT(shift(G))) = s . IFFT(s . G)
// = s . shift(IFFT(G)).
// The FFT itself is hipFFT's batched in-place transform (all channels in one
// call); the sign and correction passes are the kernels below.  Out of place,
// the sign pass copies s . G into the output, which is then transformed in place
// and corrected.  In place (image over the grid, N a multiple of 4), the grid is
// transformed as it is and one pass swaps the quadrants while it applies the
// sign and the correction, so the image costs one full-grid pass less.
#include <hipfft/hipfft.h>

#include <cmath>
#include <vector>

#include "internal.h"

namespace rts {
namespace {

// Fourier transform of the Kaiser-Bessel window at nu cycles per cell:
// W sinh(sqrt(beta^2 - (pi W nu)^2)) / (sqrt(.) I0(beta)), sin for negative radicand.
double kb_hat(double nu, int W, double beta) {
  const double t = M_PI * W * nu;
  const double z2 = beta * beta - t * t;
  double s = 1.0;
  if (z2 > 0.0) {
    const double z = std::sqrt(z2);
    s = std::sinh(z) / z;
  } else if (z2 < 0.0) {
    const double z = std::sqrt(-z2);
    s = std::sin(z) / z;
  }
  return W * s / bessel_i0(beta);
}

// Two cells (x, x+1) per thread, x even: out = s . g.
__global__ __launch_bounds__(kBlock) void k_image_pre(const float4 *g, float4 *out, int64_t npairs, int N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  const int64_t cell = 2 * i;
  const int x = (int)(cell % N), y = (int)((cell / N) % N);
  const float s = ((x + y) & 1) ? -1.0f : 1.0f;
  const float4 v = g[i];
  out[i] = make_float4(s * v.x, s * v.y, -s * v.z, -s * v.w);
}

// img = s . img / (khat_y khat_x), with rc = 1 / khat.
__global__ __launch_bounds__(kBlock) void k_image_post(float4 *img, const float *rc, int64_t npairs, int N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  const int64_t cell = 2 * i;
  const int x = (int)(cell % N), y = (int)((cell / N) % N);
  const float sy = (((x + y) & 1) ? -1.0f : 1.0f) * rc[y];
  const float f0 = sy * rc[x], f1 = -sy * rc[x + 1];
  const float4 v = img[i];
  img[i] = make_float4(f0 * v.x, f0 * v.y, f1 * v.z, f1 * v.w);
}

// In place, after the transform of the unmodulated grid (F = IFFT(G)):
// img(p) = s(p) F(p') / (khat khat)(p) with p' = p + (N/2, N/2) mod N, the
// centring shift.  The map p -> p' pairs pixels of the upper and lower halves, so
// each thread reads both members of two such pairs (pixels x, x+1 of row y < N/2
// and pixels x', x'+1 of row y + N/2, x' = (x + N/2) mod N) and writes them
// exchanged.  s(p') = s(p) since N is even; x' is even since N/2 is.
__global__ __launch_bounds__(kBlock) void k_image_swap(float4 *img, const float *rc, int64_t nquads, int N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nquads) return;
  const int h = N / 2;
  const int64_t per_c = (int64_t)h * h;   // threads per channel: N/2 rows x N/2 pixel pairs
  const int64_t c = i / per_c;
  const int rem = (int)(i - c * per_c);
  const int y = rem / h, x = 2 * (rem - y * h);
  const int x2 = (x + h) % N, y2 = y + h;
  float4 *plane = img + c * ((int64_t)N * N / 2);
  const int64_t ia = ((int64_t)y * N + x) / 2, ib = ((int64_t)y2 * N + x2) / 2;
  const float4 a = plane[ia], b = plane[ib];
  const float s0 = ((x + y) & 1) ? -1.0f : 1.0f;
  const float fa = s0 * rc[y], fb = s0 * rc[y2];
  const float a0 = fa * rc[x], a1 = -fa * rc[x + 1];
  const float b0 = fb * rc[x2], b1 = -fb * rc[x2 + 1];
  plane[ia] = make_float4(a0 * b.x, a0 * b.y, a1 * b.z, a1 * b.w);
  plane[ib] = make_float4(b0 * a.x, b0 * a.y, b1 * a.z, b1 * a.w);
}

const char *fft_error(hipfftResult r) {
  switch (r) {
    case HIPFFT_ALLOC_FAILED: return "allocation failed";
    case HIPFFT_INVALID_VALUE: return "invalid value";
    case HIPFFT_INVALID_SIZE: return "invalid size";
    case HIPFFT_EXEC_FAILED: return "execution failed";
    case HIPFFT_SETUP_FAILED: return "setup failed";
    default: return "error";
  }
}

// Correction table and FFT plan, built on first use (allocates device memory).
rts_status ensure_imager(Plan &P) {
  if (P.fft) return RTS_OK;
  std::vector<float> rc(P.N);
  for (int i = 0; i < P.N; ++i) rc[i] = (float)(1.0 / kb_hat((double)(i - P.N / 2) / P.N, P.W, P.beta));
  if (!P.d_rcorr) {
    hipError_t e = hipMalloc((void **)&P.d_rcorr, (size_t)P.N * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(P.d_rcorr, rc.data(), rc.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      set_error("imager correction table: %s", hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? RTS_E_NOMEM : RTS_E_HIP;
    }
  }
  hipfftHandle h = nullptr;
  int n[2] = {P.N, P.N};
  const hipfftResult r = hipfftPlanMany(&h, 2, n, nullptr, 1, P.N * P.N, nullptr, 1, P.N * P.N, HIPFFT_C2C, P.C);
  if (r != HIPFFT_SUCCESS) {
    set_error("hipfftPlanMany(%d x %d, batch %d): %s", P.N, P.N, P.C, fft_error(r));
    return r == HIPFFT_ALLOC_FAILED ? RTS_E_NOMEM : RTS_E_HIP;
  }
  P.fft = (void *)h;
  return RTS_OK;
}

}  // namespace

void destroy_imager(Plan *P) {
  if (P->fft) hipfftDestroy((hipfftHandle)P->fft);
  P->fft = nullptr;
  hipFree(P->d_rcorr);
  P->d_rcorr = nullptr;
}

}  // namespace rts

using namespace rts;

extern "C" rts_status rts_image(rts_plan_t plan, const float *grid, float *image_out, void *stream) {
  if (!plan) {
    set_error("plan is NULL");
    return RTS_E_INVALID;
  }
  if (!grid || !image_out) {
    set_error("grid and image_out must be non-NULL");
    return RTS_E_INVALID;
  }
  if (((uintptr_t)grid % 16) || ((uintptr_t)image_out % 16)) {
    set_error("grid and image_out must be 16-byte aligned");
    return RTS_E_INVALID;
  }
  Plan &P = *plan;
  if (rts_status st = ensure_imager(P)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t npairs = (int64_t)P.C * P.N * P.N / 2;
  const unsigned nb = (unsigned)((npairs + kBlock - 1) / kBlock);
  const bool swap = (const float *)image_out == grid && P.N % 4 == 0;
  hipError_t e = hipSuccess;
  if (!swap) {
    hipLaunchKernelGGL(k_image_pre, dim3(nb), dim3(kBlock), 0, s, (const float4 *)grid, (float4 *)image_out, npairs,
                       P.N);
    e = hipGetLastError();
    if (e != hipSuccess) {
      set_error("imager sign pass: %s", hipGetErrorString(e));
      return RTS_E_HIP;
    }
  }
  hipfftHandle h = (hipfftHandle)P.fft;
  hipfftResult r = hipfftSetStream(h, s);
  if (r == HIPFFT_SUCCESS)
    r = hipfftExecC2C(h, (hipfftComplex *)image_out, (hipfftComplex *)image_out, HIPFFT_BACKWARD);
  if (r != HIPFFT_SUCCESS) {
    set_error("hipfftExecC2C: %s", fft_error(r));
    return RTS_E_HIP;
  }
  if (swap) {
    const int64_t nquads = npairs / 2;
    const unsigned nq = (unsigned)((nquads + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_image_swap, dim3(nq), dim3(kBlock), 0, s, (float4 *)image_out, (const float *)P.d_rcorr,
                       nquads, P.N);
  } else {
    hipLaunchKernelGGL(k_image_post, dim3(nb), dim3(kBlock), 0, s, (float4 *)image_out, (const float *)P.d_rcorr,
                       npairs, P.N);
  }
  e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("imager correction pass: %s", hipGetErrorString(e));
    return RTS_E_HIP;
  }
  return RTS_OK;
}
