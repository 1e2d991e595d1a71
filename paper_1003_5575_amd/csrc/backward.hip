// Element-wise terms of the gradients through gridding and through the
// chi-squared step (Eq. (1) and its adjoint; the products of the adjoint pass
// itself run in the tile kernels).
//
//   grid backward:  d = D(dL/dG) (degridding, 0 at invalid samples);
//                   dL/dV = w d,  dL/dw = Re(conj(V) d)
//   chi2 backward:  r = V - M at valid samples (0 elsewhere), g = dL/dchi2;
//                   dL/dV = 2 g w r,  dL/dw = g |r|^2,  dL/dG = -2 g G_resid
// with G_resid = D^T (w r), the grid the fused step wrote.
#include "internal.h"

namespace rts {
namespace {

__global__ __launch_bounds__(kBlock) void k_grid_backward(const float2 *__restrict__ vis, const float *__restrict__ w,
                                                          float2 *__restrict__ d, float *__restrict__ gw,
                                                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float2 di = d[i];
  if (gw) {
    const float2 v = vis[i];
    gw[i] = fmaf(v.x, di.x, v.y * di.y);
  }
  const float wi = w[i];
  d[i] = make_float2(wi * di.x, wi * di.y);
}

__global__ __launch_bounds__(kBlock) void k_chi2_backward(const float2 *__restrict__ vis, const float *__restrict__ w,
                                                          const float2 *__restrict__ model,
                                                          const uint16_t *__restrict__ coords,
                                                          const double *__restrict__ gchi2, float2 *__restrict__ gv,
                                                          float *__restrict__ gw, int64_t n, int64_t per_chan,
                                                          int ncopy) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t c = i / per_chan;
  // the +uv copy's packed coordinates carry the plan's validity bit
  const bool ok = (coords[i + c * (int64_t)(ncopy - 1) * per_chan] & kCoordValid) != 0;
  const float g = (float)gchi2[0];
  float2 r = make_float2(0.0f, 0.0f);
  if (ok) {
    const float2 v = vis[i], m = model[i];
    r = make_float2(v.x - m.x, v.y - m.y);
  }
  if (gv) {
    const float s = 2.0f * g * w[i];
    gv[i] = make_float2(s * r.x, s * r.y);
  }
  if (gw) gw[i] = g * fmaf(r.x, r.x, r.y * r.y);
}

__global__ __launch_bounds__(kBlock) void k_scale_grid(const float4 *__restrict__ src, const double *__restrict__ gchi2,
                                                       float4 *__restrict__ dst, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n4) return;
  const float s = -2.0f * (float)gchi2[0];
  const float4 a = src[i];
  dst[i] = make_float4(s * a.x, s * a.y, s * a.z, s * a.w);
}

unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_grid_backward(const float2 *vis, const float *w, float2 *d, float *gw, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grid_backward, dim3(blocks(n)), dim3(kBlock), 0, s, vis, w, d, gw, n);
  return hipGetLastError();
}

hipError_t launch_chi2_backward(const Plan &P, const float2 *vis, const float *w, const float2 *model,
                                const double *gchi2, float2 *gv, float *gw, const float2 *gres, float2 *gg,
                                hipStream_t s) {
  const int64_t per_chan = (int64_t)P.B * P.T;
  const int64_t n = (int64_t)P.C * per_chan;
  if ((gv || gw) && n > 0)
    hipLaunchKernelGGL(k_chi2_backward, dim3(blocks(n)), dim3(kBlock), 0, s, vis, w, model, P.d_coords, gchi2, gv,
                       gw, n, per_chan, P.ncopy);
  if (gg) {
    const int64_t n4 = (int64_t)P.C * P.N * P.N / 2;   // N is even: two complex cells per float4
    hipLaunchKernelGGL(k_scale_grid, dim3(blocks(n4)), dim3(kBlock), 0, s, reinterpret_cast<const float4 *>(gres),
                       gchi2, reinterpret_cast<float4 *>(gg), n4);
  }
  return hipGetLastError();
}

}  // namespace rts
