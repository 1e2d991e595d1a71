// Polarisation conversion (the polarisation convertor stage of the paper's
// pipeline, Section 3; timed in Tables 3 and 4): for every pixel i of every
// channel, S_i = A_i P_i with P_i the four observed polarisation products of
// the pixel and A_i a 4x4 complex matrix from a precomputation.
//
// Layouts (complex64 as interleaved float pairs, planar so that every load and
// store is coalesced):
//   A  [16][n_pix]  entry r*4 + k of each pixel's matrix, plane by plane; with a
//                   channel stride, channel c's matrices start a_chan_stride
//                   complex elements further on
//   P  [C][4][n_pix]  the four observed products of each pixel, per channel
//   S  [C][4][n_pix]  S[c][r][i] = sum_k A[r*4+k][i] P[c][k][i]
//
// The operation is HBM-bound (64 bytes of P and S per pixel and channel, plus
// the 128-byte matrix): one thread converts two neighbouring pixels with 16-byte
// loads and stores, keeping a shared matrix in registers across the channels.
#include "internal.h"

namespace rts {
namespace {

constexpr int kPolBlock = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}

// Pixel pairs: thread t owns pixels 2t and 2t+1 (n_pix even, 16-byte aligned
// planes).  S may alias P: each thread reads all four products of its pixels
// before writing any of them.
__global__ __launch_bounds__(kPolBlock) void k_polconv_pairs(const float4 *__restrict__ A, const float4 *P, float4 *S,
                                                          int64_t npair, int C, int64_t a_stride_pairs) {
  const int64_t t = (int64_t)blockIdx.x * kPolBlock + threadIdx.x;
  if (t >= npair) return;
  float4 a[16];
  for (int c = 0; c < C; ++c) {
    if (c == 0 || a_stride_pairs != 0) {
      const float4 *Ac = A + (int64_t)c * a_stride_pairs + t;
#pragma unroll
      for (int e = 0; e < 16; ++e) a[e] = Ac[(int64_t)e * npair];
    }
    const float4 *Pc = P + (int64_t)c * 4 * npair + t;
    float4 p[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = Pc[(int64_t)k * npair];
    float4 *Sc = S + (int64_t)c * 4 * npair + t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float2 s0 = make_float2(0.0f, 0.0f), s1 = make_float2(0.0f, 0.0f);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 ae = a[r * 4 + k];
        s0 = cfma(make_float2(ae.x, ae.y), make_float2(p[k].x, p[k].y), s0);
        s1 = cfma(make_float2(ae.z, ae.w), make_float2(p[k].z, p[k].w), s1);
      }
      Sc[(int64_t)r * npair] = make_float4(s0.x, s0.y, s1.x, s1.y);
    }
  }
}

// Any pixel count or alignment: one pixel per thread with 8-byte accesses.
__global__ __launch_bounds__(kPolBlock) void k_polconv_single(const float2 *__restrict__ A, const float2 *P, float2 *S,
                                                           int64_t npix, int C, int64_t a_stride) {
  const int64_t i = (int64_t)blockIdx.x * kPolBlock + threadIdx.x;
  if (i >= npix) return;
  float2 a[16];
  for (int c = 0; c < C; ++c) {
    if (c == 0 || a_stride != 0) {
      const float2 *Ac = A + (int64_t)c * a_stride + i;
#pragma unroll
      for (int e = 0; e < 16; ++e) a[e] = Ac[(int64_t)e * npix];
    }
    const float2 *Pc = P + (int64_t)c * 4 * npix + i;
    float2 p[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = Pc[(int64_t)k * npix];
    float2 *Sc = S + (int64_t)c * 4 * npix + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float2 s = cmul(a[r * 4], p[0]);
#pragma unroll
      for (int k = 1; k < 4; ++k) s = cfma(a[r * 4 + k], p[k], s);
      Sc[(int64_t)r * npix] = s;
    }
  }
}

}  // namespace
}  // namespace rts

using namespace rts;

extern "C" rts_status rts_polconvert(const float *A, const float *P, float *S, int64_t n_pix, int n_chan,
                                     int64_t a_chan_stride, void *stream) {
  if (n_pix < 0 || n_chan < 0) {
    set_error("n_pix and n_chan must be >= 0 (got %lld, %d)", (long long)n_pix, n_chan);
    return RTS_E_INVALID;
  }
  if (n_pix > ((int64_t)1 << 40) / 16) {
    set_error("n_pix too large (%lld)", (long long)n_pix);
    return RTS_E_INVALID;
  }
  if (a_chan_stride != 0 && a_chan_stride < 16 * n_pix) {
    set_error("a_chan_stride must be 0 (one matrix set for all channels) or >= 16*n_pix (got %lld)",
              (long long)a_chan_stride);
    return RTS_E_INVALID;
  }
  if (n_pix == 0 || n_chan == 0) return RTS_OK;
  if (!A || !P || !S) {
    set_error("A, P and S must be non-NULL");
    return RTS_E_INVALID;
  }
  if (((uintptr_t)A % 8) || ((uintptr_t)P % 8) || ((uintptr_t)S % 8)) {
    set_error("A, P and S must be 8-byte aligned");
    return RTS_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool pairs = n_pix % 2 == 0 && a_chan_stride % 2 == 0 && (uintptr_t)A % 16 == 0 &&
                     (uintptr_t)P % 16 == 0 && (uintptr_t)S % 16 == 0;
  if (pairs) {
    const int64_t npair = n_pix / 2;
    const unsigned nb = (unsigned)((npair + kPolBlock - 1) / kPolBlock);
    hipLaunchKernelGGL(k_polconv_pairs, dim3(nb), dim3(kPolBlock), 0, s, (const float4 *)A, (const float4 *)P,
                       (float4 *)S, npair, n_chan, a_chan_stride / 2);
  } else {
    const unsigned nb = (unsigned)((n_pix + kPolBlock - 1) / kPolBlock);
    hipLaunchKernelGGL(k_polconv_single, dim3(nb), dim3(kPolBlock), 0, s, (const float2 *)A, (const float2 *)P,
                       (float2 *)S, n_pix, n_chan, a_chan_stride);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("polarisation conversion: %s", hipGetErrorString(e));
    return RTS_E_HIP;
  }
  return RTS_OK;
}
