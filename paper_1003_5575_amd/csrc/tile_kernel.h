// Tile kernels: one workgroup owns one (channel, uv tile) of the output grid.
//
// Section 5.2 of the paper gives each block of pixels to one thread block and lets
// it read only the visibilities binned near it, staging them in shared memory.
// Here a workgroup owns a tile x tile square of one channel's grid in LDS
// (complex FP32 accumulator, no global atomics on grid data) and walks the work
// list of segments whose (W+1)x(W+1) window touches the tile.  One lane handles
// one segment: up to SMAX consecutive samples of one baseline that share the
// window, so the kernel rows, the G_in window rows and the accumulated window
// rows are reused across the samples in registers.  A segment whose window
// crosses a tile edge is listed in every tile it touches; each copy adds only the
// cells of its own tile, so every output cell has exactly one writer.
//
// Modes:
//   kGrid:   G_out = sum_s w_s V_s k_y k_x                    (Eq. (1))
//   kDegrid: M_s = sum k_y k_x G_in, written by the home listing  (adjoint)
//   kFused:  M = degrid(G_in); r = V - M; G_out = grid(r, w); chi2 partials
#pragma once

#include "internal.h"

namespace rts {

// Consecutive workgroups are dispatched round-robin over the 8 XCDs, each with its
// own L2.  Remap so that every XCD walks one contiguous range of tiles: a tile's
// neighbours (whose windows overlap it) then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n >> 3, r = n & 7, xcd = bid & 7, slot = bid >> 3;
  return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

template <int WN, int SMAX, int MODE>
__global__ __launch_bounds__(kBlock) void k_tile(TileArgs a) {
  extern __shared__ float smem[];
  float *tabE = smem;                        // [2*OS][WNP]
  float *acc = smem + a.OS2 * a.WNP;         // [tile*tile][2]  (kGrid, kFused)
  const int key = xcd_remap(blockIdx.x, gridDim.x);
  const int c = key / a.nT2;
  const int rem = key - c * a.nT2;
  const int ty = rem / a.nT, tx = rem - ty * a.nT;
  const int T = a.tile;
  const int x0 = tx * T, y0 = ty * T;
  const int TT = T * T;

  for (int i = threadIdx.x; i < a.OS2 * a.WNP; i += kBlock) tabE[i] = a.tabE[i];
  if (MODE != kDegrid)
    for (int i = threadIdx.x; i < 2 * TT; i += kBlock) acc[i] = 0.0f;
  __syncthreads();

  const uint32_t beg = a.tile_off[key], end = a.tile_off[key + 1];
  const size_t copy_stride = (size_t)a.B * a.T;
  double chi2 = 0.0;

  for (uint32_t k = beg + threadIdx.x; k < end; k += kBlock) {
    const uint2 rec = a.list[k];
    const bool home = (rec.y >> kRecHomeBit) & 1u;
    if (MODE == kDegrid && !home) continue;
    const int X0 = (int)(rec.y & kRecXMask);
    const int Y0 = (int)((rec.y >> kRecYShift) & kRecXMask);
    const int nt = (int)((rec.y >> kRecNtShift) & 7u) + 1;
    const int copy = (int)((rec.y >> kRecCopyBit) & 1u);
    const bool any = (rec.y >> kRecAnyBit) & 1u;
    const size_t vi = rec.x;
    const bool put_model = home && copy == 0 && (MODE == kDegrid || (MODE == kFused && a.write_model));
    if (!any) {
      if (put_model)
        for (int s = 0; s < nt; ++s) a.model[vi + s] = make_float2(0.0f, 0.0f);
      continue;
    }
    const size_t ci = vi + (size_t)(c * (a.ncopy - 1) + copy) * copy_stride;

    float kx[SMAX][WN], ky[SMAX][WN];
    float2 val[SMAX];
    float wt[SMAX];
    bool ok[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      ok[s] = false;
      val[s] = make_float2(0.0f, 0.0f);
      wt[s] = 0.0f;
      int sx = 0, sy = 0;
      if (s < nt) {
        const uint16_t cw = a.coords[ci + s];
        ok[s] = (cw & kCoordValid) != 0;
        sx = cw & 0x7F;
        sy = (cw >> 7) & 0x7F;
        if (MODE != kDegrid && ok[s]) {
          val[s] = a.vis[vi + s];
          wt[s] = a.w[vi + s];
          if (copy) val[s].y = -val[s].y;
        }
      }
      const float *rx = tabE + sx * a.WNP;
      const float *ry = tabE + sy * a.WNP;
#pragma unroll
      for (int i = 0; i < WN; ++i) {
        kx[s][i] = rx[i];
        ky[s][i] = ok[s] ? ry[i] : 0.0f;
      }
    }

    float2 M[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) M[s] = make_float2(0.0f, 0.0f);
    if (MODE != kGrid) {
      const float2 *g = a.gin + ((size_t)c * a.N + Y0) * a.N + X0;
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        float2 row[WN];
#pragma unroll
        for (int i = 0; i < WN; ++i) row[i] = g[(size_t)j * a.N + i];
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
          if (s < nt) {
            float rr = 0.0f, ri = 0.0f;
#pragma unroll
            for (int i = 0; i < WN; ++i) {
              rr = fmaf(kx[s][i], row[i].x, rr);
              ri = fmaf(kx[s][i], row[i].y, ri);
            }
            M[s].x = fmaf(ky[s][j], rr, M[s].x);
            M[s].y = fmaf(ky[s][j], ri, M[s].y);
          }
        }
      }
    }

    float2 A[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      A[s] = make_float2(0.0f, 0.0f);
      if (ok[s]) {
        if (MODE == kGrid) {
          A[s] = make_float2(wt[s] * val[s].x, wt[s] * val[s].y);
        } else if (MODE == kFused) {
          const float rr = val[s].x - M[s].x, ri = val[s].y - M[s].y;
          A[s] = make_float2(wt[s] * rr, wt[s] * ri);
          if (home && copy == 0) chi2 += (double)wt[s] * ((double)rr * rr + (double)ri * ri);
        }
      }
      if (put_model && s < nt) a.model[vi + s] = ok[s] ? M[s] : make_float2(0.0f, 0.0f);
    }

    if (MODE != kDegrid) {
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int yy = Y0 + j - y0;
        if ((unsigned)yy < (unsigned)T) {
          float2 arow[WN];
#pragma unroll
          for (int i = 0; i < WN; ++i) arow[i] = make_float2(0.0f, 0.0f);
#pragma unroll
          for (int s = 0; s < SMAX; ++s) {
            if (s < nt) {
              const float br = A[s].x * ky[s][j], bi = A[s].y * ky[s][j];
#pragma unroll
              for (int i = 0; i < WN; ++i) {
                arow[i].x = fmaf(br, kx[s][i], arow[i].x);
                arow[i].y = fmaf(bi, kx[s][i], arow[i].y);
              }
            }
          }
          float *dst = acc + 2 * (yy * T + (X0 - x0));
#pragma unroll
          for (int i = 0; i < WN; ++i) {
            const int xx = X0 + i - x0;
            if ((unsigned)xx < (unsigned)T) {
              atomicAdd(dst + 2 * i, arow[i].x);
              atomicAdd(dst + 2 * i + 1, arow[i].y);
            }
          }
        }
      }
    }
  }

  if (MODE == kFused) {
    __shared__ double red[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) chi2 += __shfl_down(chi2, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = chi2;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < kBlock / 64; ++i) t += red[i];
      a.chi2_part[key] = t;
    }
  }
  if (MODE != kDegrid) {
    __syncthreads();
    float4 *out = reinterpret_cast<float4 *>(a.gout);
    const float4 *src = reinterpret_cast<const float4 *>(acc);
    const int half = T / 2;
    for (int i = threadIdx.x; i < TT / 2; i += kBlock) {
      const int yy = i / half, xx = i - yy * half;
      out[(((size_t)c * a.N + y0 + yy) * a.N + x0) / 2 + xx] = src[i];
    }
  }
}

}  // namespace rts
