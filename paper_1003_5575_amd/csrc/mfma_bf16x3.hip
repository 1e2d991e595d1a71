// Gridding as a dense per-tile contraction on the matrix cores, with BF16 hi+lo
// split operands and FP32 accumulation.
//
// For one 16x16-cell tile of one channel, Eq. (1) restricted to the tile is
//     G_re = Av^T diag(w Re V) Au,   G_im = Av^T diag(w Im V) Au,
// where Av[s][y] (Au[s][x]) is the kernel weight of sample s on tile row y
// (column x), zero outside its support.  K runs over the samples whose window
// touches the tile (the plan's work list), 32 at a time.  Every operand x is
// split as x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), and the product
// is taken as hi*hi + hi*lo + lo*hi (three v_mfma_f32_16x16x32_bf16 per output
// block, FP32 accumulation): about 16 significant bits per operand, relative
// error of a few 1e-6 on the grid.  The accumulators stay in registers for the
// whole tile, so there are no atomics; one wave owns one tile.
#include "internal.h"

namespace rts {
namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int kMT = 16;          // tile edge of this kernel (one MFMA output block)
constexpr int kChunk = 32;       // samples per MFMA K step
constexpr int kWaves = 4;        // tiles (waves) per workgroup

struct SampleSlot {
  int dx, dy;       // window origin relative to the tile origin (cells)
  int sx, sy;       // extended-table rows of the sample (-1: no sample)
  float ar, ai;     // w * V (zero for an empty or invalid slot)
};

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }   // round to nearest even

// hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = to_bf16(x);
  lo = to_bf16(x - (float)hi);
}

__global__ __launch_bounds__(64 * kWaves) void k_grid_mfma_bf16x3(TileArgs a, const uint16_t *tab_hi,
                                                                   const uint16_t *tab_lo) {
  __shared__ SampleSlot slots[kWaves][kChunk];
  extern __shared__ float4 smem4[];
  float *tabE = reinterpret_cast<float *>(smem4);                       // [2*OS][WNP] FP32
  uint16_t *thi = reinterpret_cast<uint16_t *>(tabE + a.OS2 * a.WNP);   // [2*OS][WNP] bf16 bits
  uint16_t *tlo = thi + a.OS2 * a.WNP;
  for (int i = threadIdx.x; i < a.OS2 * a.WNP; i += 64 * kWaves) {
    tabE[i] = a.tabE[i];
    thi[i] = tab_hi[i];
    tlo[i] = tab_lo[i];
  }
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ngroups = (a.nkeys + kWaves - 1) / kWaves;
  const int key = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave;
  if (blockIdx.x >= (unsigned)ngroups || key >= a.nkeys) return;   // whole wave leaves together
  const int c = key / a.nT2;
  const int rem = key - c * a.nT2;
  const int ty = rem / a.nT, tx = rem - ty * a.nT;
  const int x0 = tx * kMT, y0 = ty * kMT;
  const uint32_t cap = (uint32_t)a.list_cap;
  const uint32_t beg = min(a.tile_off[key], cap), end = min(a.tile_off[key + 1], cap);
  const size_t copy_stride = (size_t)a.B * a.T;

  f4_t acc_re = {0.0f, 0.0f, 0.0f, 0.0f}, acc_im = {0.0f, 0.0f, 0.0f, 0.0f};
  const int i16 = lane & 15, g = lane >> 4;        // MFMA operand row/column and K group
  SampleSlot *ss = slots[wave];

  // seg_max (2, 4 or 8) sample slots per listing, kChunk / seg_max listings per chunk
  const int lg = __builtin_ctz((unsigned)a.seg_max);
  const uint32_t per_chunk = (uint32_t)(kChunk >> lg);
  for (uint32_t k0 = beg; k0 < end; k0 += per_chunk) {
    // Stage the chunk: slot lane holds sample (lane mod seg_max) of listing
    // k0 + lane / seg_max; slots past a segment's end stay empty.
    if (lane < kChunk) {
      SampleSlot sl;
      sl.dx = sl.dy = 0;
      sl.sx = sl.sy = -1;
      sl.ar = sl.ai = 0.0f;
      const uint32_t k = k0 + (uint32_t)(lane >> lg);
      const int j = lane & (a.seg_max - 1);
      if (k < end) {
        const uint2 rec = a.list[k];
        const int nt = (int)((rec.y >> kRecNtShift) & 7u) + 1;
        const bool any = (rec.y >> kRecAnyBit) & 1u;
        if (any && j < nt) {
          const int copy = (int)((rec.y >> kRecCopyBit) & 1u);
          const size_t vi = rec.x + j;
          const size_t ci = vi + (size_t)(c * (a.ncopy - 1) + copy) * copy_stride;
          const uint16_t cw = a.coords[ci];
          if (cw & kCoordValid) {
            float2 v = a.vis[vi];
            const float wt = a.w[vi];
            if (copy) v.y = -v.y;
            sl.dx = (int)(rec.y & kRecXMask) - x0;
            sl.dy = (int)((rec.y >> kRecYShift) & kRecXMask) - y0;
            sl.sx = cw & 0x7F;
            sl.sy = (cw >> 7) & 0x7F;
            sl.ar = wt * v.x;
            sl.ai = wt * v.y;
          }
        }
      }
      ss[lane] = sl;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the slot writes are visible to the wave

    // Operands.  A[y][s] = ky_s(y0 + y), row y = i16, samples s = 8g + e.
    // B[s][x] = a_s kx_s(x0 + x), column x = i16, the same samples.
    bf8_t ah, al, brh, brl, bih, bil;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const SampleSlot sl = ss[8 * g + e];
      const int ry = i16 - sl.dy, rx = i16 - sl.dx;       // window row / column of this cell
      const bool has = sl.sx >= 0;
      const bool iny = has && ry >= 0 && ry < a.WN;
      const bool inx = has && rx >= 0 && rx < a.WN;
      const int ty_i = iny ? sl.sy * a.WNP + ry : 0;
      const int tx_i = inx ? sl.sx * a.WNP + rx : 0;
      const uint16_t hy = iny ? thi[ty_i] : (uint16_t)0, ly = iny ? tlo[ty_i] : (uint16_t)0;
      ah[e] = __builtin_bit_cast(__bf16, hy);
      al[e] = __builtin_bit_cast(__bf16, ly);
      const float kx = inx ? tabE[tx_i] : 0.0f;
      __bf16 h, l;
      split_bf16(sl.ar * kx, h, l);
      brh[e] = h;
      brl[e] = l;
      split_bf16(sl.ai * kx, h, l);
      bih[e] = h;
      bil[e] = l;
    }
    acc_re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, brh, acc_re, 0, 0, 0);
    acc_re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, brl, acc_re, 0, 0, 0);
    acc_re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, brh, acc_re, 0, 0, 0);
    acc_im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bih, acc_im, 0, 0, 0);
    acc_im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bil, acc_im, 0, 0, 0);
    acc_im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bih, acc_im, 0, 0, 0);
    __builtin_amdgcn_wave_barrier();   // the next chunk's slot writes follow these reads
  }

  // D[y][x] sits in lane x + 16 * (y / 4), register y % 4.
  float2 *out = a.gout + ((size_t)c * a.N + y0) * a.N + x0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int y = 4 * g + r;
    out[(size_t)y * a.N + i16] = make_float2(acc_re[r], acc_im[r]);
  }
}

// Degridding of one 16x16 tile on the matrix cores.  For the samples of the
// tile's work list (16 at a time, rows of the MFMA), H = Av G_tile holds, per
// sample and tile column x, the sum over the tile's rows of k_y * G; the sample's
// partial model value over this tile is sum_x H[s][x] k_x(x).  The window of a
// sample that crosses tile edges is covered by its listings in each tile, so
// the partial values are added to the (zeroed) model with FP32 atomics.  Both
// operands of H are split hi+lo as in the gridding kernel; H is formed as one
// K=32 contraction per term with B = [Re G; Im G] stacked along K and A holding
// k_y in the half that selects the real or imaginary part.
struct DegridSlot {
  int dx, dy;     // window origin relative to the tile origin (cells)
  int sx, sy;     // extended-table rows (-1: no sample)
  int vi;         // model index
};

__global__ __launch_bounds__(64 * kWaves) void k_degrid_mfma_bf16x3(TileArgs a, const uint16_t *tab_hi,
                                                                     const uint16_t *tab_lo) {
  __shared__ DegridSlot dslots[kWaves][16];
  extern __shared__ float4 smem4[];
  float *tabE = reinterpret_cast<float *>(smem4);
  uint16_t *thi = reinterpret_cast<uint16_t *>(tabE + a.OS2 * a.WNP);
  uint16_t *tlo = thi + a.OS2 * a.WNP;
  for (int i = threadIdx.x; i < a.OS2 * a.WNP; i += 64 * kWaves) {
    tabE[i] = a.tabE[i];
    thi[i] = tab_hi[i];
    tlo[i] = tab_lo[i];
  }
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ngroups = (a.nkeys + kWaves - 1) / kWaves;
  const int key = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave;
  if (blockIdx.x >= (unsigned)ngroups || key >= a.nkeys) return;   // whole wave leaves together
  const int c = key / a.nT2;
  const int rem = key - c * a.nT2;
  const int ty = rem / a.nT, tx = rem - ty * a.nT;
  const int x0 = tx * kMT, y0 = ty * kMT;
  const uint32_t cap = (uint32_t)a.list_cap;
  const uint32_t beg = min(a.tile_off[key], cap), end = min(a.tile_off[key + 1], cap);
  if (beg >= end) return;
  const int i16 = lane & 15, g = lane >> 4;

  // B operand, loaded once: lane (x = i16, g) holds rows 8(g & 1) + e of Re G
  // (g < 2) or Im G (g >= 2) at tile column x.
  bf8_t bh, bl;
  {
    const float2 *gt = a.gin + ((size_t)c * a.N + y0) * a.N + x0 + i16;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float2 v = gt[(size_t)(8 * (g & 1) + e) * a.N];
      __bf16 h, l;
      split_bf16(g < 2 ? v.x : v.y, h, l);
      bh[e] = h;
      bl[e] = l;
    }
  }
  DegridSlot *ds = dslots[wave];
  const int lg = __builtin_ctz((unsigned)a.seg_max);
  const uint32_t per_chunk = (uint32_t)(16 >> lg);
  for (uint32_t k0 = beg; k0 < end; k0 += per_chunk) {
    // Stage 16 sample slots: slot j holds sample (j mod seg_max) of listing k0 + j / seg_max.
    if (lane < 16) {
      DegridSlot sl;
      sl.dx = sl.dy = 0;
      sl.sx = sl.sy = -1;
      sl.vi = 0;
      const uint32_t k = k0 + (uint32_t)(lane >> lg);
      const int j = lane & (a.seg_max - 1);
      if (k < end) {
        const uint2 rec = a.list[k];
        const int nt = (int)((rec.y >> kRecNtShift) & 7u) + 1;
        const bool any = (rec.y >> kRecAnyBit) & 1u;
        const int copy = (int)((rec.y >> kRecCopyBit) & 1u);
        if (any && copy == 0 && j < nt) {
          const size_t vi = rec.x + j;
          const uint16_t cw = a.coords[vi + (size_t)(c * (a.ncopy - 1)) * ((size_t)a.B * a.T)];
          if (cw & kCoordValid) {
            sl.dx = (int)(rec.y & kRecXMask) - x0;
            sl.dy = (int)((rec.y >> kRecYShift) & kRecXMask) - y0;
            sl.sx = cw & 0x7F;
            sl.sy = (cw >> 7) & 0x7F;
            sl.vi = (int)vi;
          }
        }
      }
      ds[lane] = sl;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the slot writes are visible to the wave

    // A operand: lane (s = i16, g) holds k_y of sample s at tile rows 8(g & 1) + e,
    // in the real half (g < 2) or the imaginary half (g >= 2) of K.
    bf8_t arh, arl, aih, ail;
    {
      const DegridSlot sl = ds[i16];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int ry = 8 * (g & 1) + e - sl.dy;
        const bool in = sl.sx >= 0 && ry >= 0 && ry < a.WN;
        const int ti = in ? sl.sy * a.WNP + ry : 0;
        const __bf16 h = __builtin_bit_cast(__bf16, in ? thi[ti] : (uint16_t)0);
        const __bf16 l = __builtin_bit_cast(__bf16, in ? tlo[ti] : (uint16_t)0);
        const __bf16 z = __builtin_bit_cast(__bf16, (uint16_t)0);
        arh[e] = g < 2 ? h : z;
        arl[e] = g < 2 ? l : z;
        aih[e] = g < 2 ? z : h;
        ail[e] = g < 2 ? z : l;
      }
    }
    f4_t hr = {0.0f, 0.0f, 0.0f, 0.0f}, hi = {0.0f, 0.0f, 0.0f, 0.0f};
    hr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bh, hr, 0, 0, 0);
    hr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bl, hr, 0, 0, 0);
    hr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, bh, hr, 0, 0, 0);
    hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bh, hi, 0, 0, 0);
    hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bl, hi, 0, 0, 0);
    hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, bh, hi, 0, 0, 0);

    // H[s][x] sits in lane x + 16 (s / 4), register s % 4: weight by k_x and sum
    // over the 16 columns of a row of lanes.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const DegridSlot sl = ds[4 * g + r];
      const int rx = i16 - sl.dx;
      const bool in = sl.sx >= 0 && rx >= 0 && rx < a.WN;
      const float kx = in ? tabE[sl.sx * a.WNP + rx] : 0.0f;
      float mr = hr[r] * kx, mi = hi[r] * kx;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        mr += __shfl_xor(mr, o, 16);
        mi += __shfl_xor(mi, o, 16);
      }
      if (i16 == 0 && sl.sx >= 0) {
        atomicAdd(&a.model[sl.vi].x, mr);
        atomicAdd(&a.model[sl.vi].y, mi);
      }
    }
    __builtin_amdgcn_wave_barrier();   // the next chunk's slot writes follow these reads
  }
}

}  // namespace

hipError_t launch_grid_mfma(const Plan &P, const TileArgs &a, hipStream_t s) {
  const int ngroups = (int)((P.nkeys + kWaves - 1) / kWaves);
  const size_t lds = (size_t)a.OS2 * a.WNP * (sizeof(float) + 2 * sizeof(uint16_t));
  hipLaunchKernelGGL(k_grid_mfma_bf16x3, dim3((unsigned)ngroups), dim3(64 * kWaves), lds, s, a, P.d_tab_hi,
                     P.d_tab_lo);
  return hipGetLastError();
}

hipError_t launch_degrid_mfma(const Plan &P, const TileArgs &a, hipStream_t s) {
  // the model is the sum of per-tile partial values: start from zero
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(a.model), (int64_t)2 * P.C * P.B * P.T, 0u, s);
  if (e != hipSuccess) return e;
  const int ngroups = (int)((P.nkeys + kWaves - 1) / kWaves);
  const size_t lds = (size_t)a.OS2 * a.WNP * (sizeof(float) + 2 * sizeof(uint16_t));
  hipLaunchKernelGGL(k_degrid_mfma_bf16x3, dim3((unsigned)ngroups), dim3(64 * kWaves), lds, s, a, P.d_tab_hi,
                     P.d_tab_lo);
  return hipGetLastError();
}

}  // namespace rts
