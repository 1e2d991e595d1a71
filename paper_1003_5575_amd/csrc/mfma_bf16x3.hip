// Gridding and degridding as dense per-tile contractions on the matrix cores,
// with BF16 hi+lo split operands and FP32 accumulation.
//
// For one 16x16-cell subtile of one channel, Eq. (1) restricted to the subtile is
//     G_re = Av^T diag(w Re V) Au,   G_im = Av^T diag(w Im V) Au,
// where Av[s][y] (Au[s][x]) is the kernel weight of sample s on subtile row y
// (column x), zero outside its support; degridding is its adjoint, H = Av G
// followed by the sum over columns weighted by Au.  Every operand x is split as
// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), and each product is taken
// as hi*hi + hi*lo + lo*hi (three v_mfma_f32_16x16x32_bf16 per block, FP32
// accumulation): about 16 significant bits per operand, relative error of a few
// 1e-6.
//
// A workgroup owns one tile of the plan (16, 32 or 64 cells, sorted by the
// plan's counting sort); each of its waves owns one 16x16 subtile and keeps a
// queue of the tile's listings whose window touches that subtile (ballot
// compaction), consuming it in chunks of sample slots.  Gridding accumulators
// stay in registers (no atomics); degridding adds each subtile's partial model
// values with FP32 atomics.
#include "internal.h"

namespace rts {
namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int kMT = 16;          // subtile edge (one MFMA output block)
constexpr int kMaxWaves = (kMaxTile / kMT) * (kMaxTile / kMT);
constexpr int kQueue = 128;      // listing queue per wave (at most chunk - 1 + 64 entries)

struct SampleSlot {
  int dx, dy;       // window origin relative to the subtile origin (cells)
  int sx, sy;       // extended-table rows of the sample (-1: no sample)
  float ar, ai;     // w * V (gridding) / unused (degridding)
  int vi;           // model index (degridding)
};

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }   // round to nearest even

// hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = to_bf16(x);
  lo = to_bf16(x - (float)hi);
}

// Table copy into LDS: FP32 rows, then the BF16 hi and lo parts.
__device__ __forceinline__ void load_tables(const TileArgs &a, const uint16_t *tab_hi, const uint16_t *tab_lo,
                                            float *&tabE, uint16_t *&thi, uint16_t *&tlo) {
  extern __shared__ float4 smem4[];
  tabE = reinterpret_cast<float *>(smem4);
  thi = reinterpret_cast<uint16_t *>(tabE + a.OS2 * a.WNP);
  tlo = thi + a.OS2 * a.WNP;
  for (int i = threadIdx.x; i < a.OS2 * a.WNP; i += blockDim.x) {
    tabE[i] = a.tabE[i];
    thi[i] = tab_hi[i];
    tlo[i] = tab_lo[i];
  }
  __syncthreads();
}

// Walk the tile's work list and call chunk(n) whenever the wave's queue holds
// `per_chunk` listings whose window overlaps the subtile at (x0, y0) (and once
// more for the remainder).  q: the wave's queue; chunk reads q[0..n).
template <class Chunk>
__device__ __forceinline__ void for_subtile_chunks(const TileArgs &a, uint32_t beg, uint32_t end, int x0, int y0,
                                                   bool with_copies, uint32_t *q, int per_chunk, Chunk chunk) {
  const int lane = threadIdx.x & 63;
  int qn = 0;                                        // wave-uniform
  for (uint32_t base = beg; base < end; base += 64) {
    const uint32_t k = base + (uint32_t)lane;
    bool ov = false;
    if (k < end) {
      const uint2 rec = a.list[k];
      const bool any = (rec.y >> kRecAnyBit) & 1u;
      const bool copy = (rec.y >> kRecCopyBit) & 1u;
      const int X0 = (int)(rec.y & kRecXMask), Y0 = (int)((rec.y >> kRecYShift) & kRecXMask);
      ov = any && (with_copies || !copy) && X0 < x0 + kMT && X0 + a.WN > x0 && Y0 < y0 + kMT && Y0 + a.WN > y0;
    }
    const unsigned long long m = __ballot(ov);
    const int pos = qn + __popcll(m & ((1ull << lane) - 1ull));
    if (ov) q[pos] = k;
    qn += __popcll(m);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
    while (qn >= per_chunk) {
      chunk(per_chunk);
      const int rest = qn - per_chunk;               // < 64
      const uint32_t t = lane < rest ? q[per_chunk + lane] : 0u;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);
      if (lane < rest) q[lane] = t;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);
      qn = rest;
    }
  }
  if (qn > 0) chunk(qn);
}

__global__ __launch_bounds__(64 * kMaxWaves) void k_grid_mfma_bf16x3(TileArgs a, const uint16_t *tab_hi,
                                                                     const uint16_t *tab_lo) {
  constexpr int kChunk = 32;                         // sample slots per MFMA K step
  __shared__ SampleSlot slots[kMaxWaves][kChunk];
  __shared__ uint32_t queue[kMaxWaves][kQueue];
  float *tabE;
  uint16_t *thi, *tlo;
  load_tables(a, tab_hi, tab_lo, tabE, thi, tlo);

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nsub = a.tile / kMT;
  const int key = xcd_remap(blockIdx.x, gridDim.x);
  const int c = key / a.nT2;
  const int rem = key - c * a.nT2;
  const int ty = rem / a.nT, tx = rem - ty * a.nT;
  const int x0 = tx * a.tile + kMT * (wave % nsub), y0 = ty * a.tile + kMT * (wave / nsub);
  const uint32_t cap = (uint32_t)a.list_cap;
  const uint32_t beg = min(a.tile_off[key], cap), end = min(a.tile_off[key + 1], cap);
  const size_t copy_stride = (size_t)a.B * a.T;

  f4_t acc_re = {0.0f, 0.0f, 0.0f, 0.0f}, acc_im = {0.0f, 0.0f, 0.0f, 0.0f};
  const int i16 = lane & 15, g = lane >> 4;        // MFMA operand row/column and K group
  SampleSlot *ss = slots[wave];
  uint32_t *q = queue[wave];
  // seg_max (2, 4 or 8) sample slots per listing, kChunk / seg_max listings per chunk
  const int lg = __builtin_ctz((unsigned)a.seg_max);

  for_subtile_chunks(a, beg, end, x0, y0, true, q, kChunk >> lg, [&](int n) {
    // Stage the chunk: slot lane holds sample (lane mod seg_max) of queued listing lane / seg_max.
    if (lane < kChunk) {
      SampleSlot sl;
      sl.dx = sl.dy = 0;
      sl.sx = sl.sy = -1;
      sl.ar = sl.ai = 0.0f;
      sl.vi = 0;
      const int li = lane >> lg;
      const int j = lane & (a.seg_max - 1);
      if (li < n) {
        const uint2 rec = a.list[q[li]];
        const int nt = (int)((rec.y >> kRecNtShift) & 7u) + 1;
        if (j < nt) {
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
  });

  // D[y][x] sits in lane x + 16 * (y / 4), register y % 4.
  float2 *out = a.gout + ((size_t)c * a.N + y0) * a.N + x0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int y = 4 * g + r;
    out[(size_t)y * a.N + i16] = make_float2(acc_re[r], acc_im[r]);
  }
}

// Degridding of one subtile: for the queued samples (16 at a time, rows of the
// MFMA), H = Av G_sub holds, per sample and subtile column x, the sum over the
// subtile's rows of k_y * G; the sample's partial model value over this subtile
// is sum_x H[s][x] k_x(x).  A window crossing subtile edges is covered by the
// subtiles it touches, so the partial values are added to the (zeroed) model
// with FP32 atomics.  H is formed as one K=32 contraction per term with
// B = [Re G; Im G] stacked along K and A holding k_y in the half that selects
// the real or imaginary part.
__global__ __launch_bounds__(64 * kMaxWaves) void k_degrid_mfma_bf16x3(TileArgs a, const uint16_t *tab_hi,
                                                                       const uint16_t *tab_lo) {
  constexpr int kChunk = 16;
  __shared__ SampleSlot dslots[kMaxWaves][kChunk];
  __shared__ uint32_t queue[kMaxWaves][kQueue];
  float *tabE;
  uint16_t *thi, *tlo;
  load_tables(a, tab_hi, tab_lo, tabE, thi, tlo);

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nsub = a.tile / kMT;
  const int key = xcd_remap(blockIdx.x, gridDim.x);
  const int c = key / a.nT2;
  const int rem = key - c * a.nT2;
  const int ty = rem / a.nT, tx = rem - ty * a.nT;
  const int x0 = tx * a.tile + kMT * (wave % nsub), y0 = ty * a.tile + kMT * (wave / nsub);
  const uint32_t cap = (uint32_t)a.list_cap;
  const uint32_t beg = min(a.tile_off[key], cap), end = min(a.tile_off[key + 1], cap);
  const int i16 = lane & 15, g = lane >> 4;

  // B operand, loaded once: lane (x = i16, g) holds rows 8(g & 1) + e of Re G
  // (g < 2) or Im G (g >= 2) at subtile column x.
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
  SampleSlot *ds = dslots[wave];
  uint32_t *q = queue[wave];
  const int lg = __builtin_ctz((unsigned)a.seg_max);

  for_subtile_chunks(a, beg, end, x0, y0, false, q, kChunk >> lg, [&](int n) {
    // Stage 16 sample slots: slot j holds sample (j mod seg_max) of queued listing j / seg_max.
    if (lane < kChunk) {
      SampleSlot sl;
      sl.dx = sl.dy = 0;
      sl.sx = sl.sy = -1;
      sl.ar = sl.ai = 0.0f;
      sl.vi = 0;
      const int li = lane >> lg;
      const int j = lane & (a.seg_max - 1);
      if (li < n) {
        const uint2 rec = a.list[q[li]];
        const int nt = (int)((rec.y >> kRecNtShift) & 7u) + 1;
        if (j < nt) {
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

    // A operand: lane (s = i16, g) holds k_y of sample s at subtile rows 8(g & 1) + e,
    // in the real half (g < 2) or the imaginary half (g >= 2) of K.
    bf8_t arh, arl, aih, ail;
    {
      const SampleSlot sl = ds[i16];
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
      const SampleSlot sl = ds[4 * g + r];
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
  });
}

}  // namespace

hipError_t launch_grid_mfma(const Plan &P, const TileArgs &a, hipStream_t s) {
  const size_t lds = (size_t)a.OS2 * a.WNP * (sizeof(float) + 2 * sizeof(uint16_t));
  const unsigned threads = 64u * (unsigned)((P.tile / kMT) * (P.tile / kMT));
  hipLaunchKernelGGL(k_grid_mfma_bf16x3, dim3((unsigned)P.nkeys), dim3(threads), lds, s, a, P.d_tab_hi,
                     P.d_tab_lo);
  return hipGetLastError();
}

hipError_t launch_degrid_mfma(const Plan &P, const TileArgs &a, hipStream_t s) {
  // the model is the sum of per-subtile partial values: start from zero
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(a.model), (int64_t)2 * P.C * P.B * P.T, 0u, s);
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)a.OS2 * a.WNP * (sizeof(float) + 2 * sizeof(uint16_t));
  const unsigned threads = 64u * (unsigned)((P.tile / kMT) * (P.tile / kMT));
  hipLaunchKernelGGL(k_degrid_mfma_bf16x3, dim3((unsigned)P.nkeys), dim3(threads), lds, s, a, P.d_tab_hi,
                     P.d_tab_lo);
  return hipGetLastError();
}

}  // namespace rts
