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
// queue of the tile's listing records whose window touches that subtile (ballot
// compaction), consuming it in chunks of sample slots.  A slot is 16 bytes in
// LDS: the window origin relative to the subtile and the two table-row bases as
// packed 16-bit pairs, then w*V (gridding) or the model index (degridding), so
// building the MFMA operands is branch-free: one slot read and two table reads
// per sample and lane.  Gridding accumulators stay in registers (no atomics);
// degridding reduces each sample's partial value over the subtile columns with
// DPP and adds it to the (zeroed) model with FP32 atomics, one atomic
// instruction per chunk.
#include "internal.h"

namespace rts {
namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
typedef unsigned u4_t __attribute__((ext_vector_type(4)));

constexpr int kMT = 16;          // subtile edge (one MFMA output block)
constexpr int kMaxWaves = (kMaxTile / kMT) * (kMaxTile / kMT);
constexpr int kQueue = 128;      // listing queue per wave (at most chunk - 1 + 64 entries)
constexpr int kFar = 0x4000;     // window offset of an empty slot: every row and column test fails

__device__ __forceinline__ uint32_t pack16(int lo, int hi) { return ((uint32_t)lo & 0xFFFFu) | ((uint32_t)hi << 16); }
__device__ __forceinline__ int lo16(uint32_t v) { return (int)(v << 16) >> 16; }
__device__ __forceinline__ int hi16(uint32_t v) { return (int)v >> 16; }

// Two products a0*k0, a1*k1 split into packed BF16 pairs: hi = bf16(p) (round to
// nearest even), lo = bf16(p - hi) with the residual taken by an FMA.
__device__ __forceinline__ void split_pair(float a0, float k0, float a1, float k1, uint32_t &hi, uint32_t &lo) {
  const f2v_t p = {a0 * k0, a1 * k1};
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(p, bf2_t));
  const f2v_t r = {__builtin_fmaf(a0, k0, -__uint_as_float(h << 16)),
                   __builtin_fmaf(a1, k1, -__uint_as_float(h & 0xFFFF0000u))};
  hi = h;
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf2_t));
}

// One float x split the same way; returns hi in the low and lo in the high half.
__device__ __forceinline__ uint32_t split_one(float x) {
  const uint32_t h = __builtin_bit_cast(uint16_t, (__bf16)x);
  const uint32_t l = __builtin_bit_cast(uint16_t, (__bf16)(x - __uint_as_float(h << 16)));
  return h | (l << 16);
}

// Table copy into LDS: the FP32 rows, then the BF16 hi and lo parts packed as
// one word per entry (hi in the low half).
__device__ __forceinline__ void load_tables(const TileArgs &a, const uint16_t *tab_hi, const uint16_t *tab_lo,
                                            float *&tabE, uint32_t *&thl) {
  extern __shared__ float4 smem4[];
  tabE = reinterpret_cast<float *>(smem4);
  thl = reinterpret_cast<uint32_t *>(tabE + a.OS2 * a.WNP);
  for (int i = threadIdx.x; i < a.OS2 * a.WNP; i += blockDim.x) {
    tabE[i] = a.tabE[i];
    thl[i] = (uint32_t)tab_hi[i] | ((uint32_t)tab_lo[i] << 16);
  }
  __syncthreads();
}

// Walk the tile's listings and call chunk(n) whenever the wave's queue holds
// `per_chunk` records whose window overlaps the subtile at (x0, y0) (and once
// more for the remainder).  q: the wave's queue of records; chunk reads q[0..n).
template <class Chunk>
__device__ __forceinline__ void for_subtile_chunks(const TileArgs &a, uint32_t beg, uint32_t end, int x0, int y0,
                                                   bool with_copies, uint2 *q, int per_chunk, Chunk chunk) {
  const int lane = threadIdx.x & 63;
  int qn = 0;                                        // wave-uniform
  for (uint32_t base = beg; base < end; base += 64) {
    const uint32_t k = base + (uint32_t)lane;
    bool ov = false;
    uint2 rec = make_uint2(0u, 0u);
    if (k < end) {
      rec = a.list[k];
      const bool any = (rec.y >> kRecAnyBit) & 1u;
      const bool copy = (rec.y >> kRecCopyBit) & 1u;
      const int X0 = (int)(rec.y & kRecXMask), Y0 = (int)((rec.y >> kRecYShift) & kRecXMask);
      ov = any && (with_copies || !copy) && X0 < x0 + kMT && X0 + a.WN > x0 && Y0 < y0 + kMT && Y0 + a.WN > y0;
    }
    const unsigned long long m = __ballot(ov);
    const int pos = qn + __popcll(m & ((1ull << lane) - 1ull));
    if (ov) q[pos] = rec;
    qn += __popcll(m);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
    while (qn >= per_chunk) {
      chunk(per_chunk);
      const int rest = qn - per_chunk;               // < 64
      const uint2 t = lane < rest ? q[per_chunk + lane] : make_uint2(0u, 0u);
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

// Slot of sample j of a queued record for the subtile at (x0, y0): .x = window
// origin (dy, dx) relative to the subtile, .y = table indices minus that origin
// (sy*WNP - dy, sx*WNP - dx), so that row y of the subtile reads entry .y.lo + y
// when 0 <= y - dy < WN.  An empty slot has the origin at kFar.
__device__ __forceinline__ void slot_geometry(const TileArgs &a, uint32_t recy, uint16_t cw, int x0, int y0,
                                              uint32_t &sx_word, uint32_t &sy_word) {
  const int dx = (int)(recy & kRecXMask) - x0;
  const int dy = (int)((recy >> kRecYShift) & kRecXMask) - y0;
  const int sx = cw & 0x7F, sy = (cw >> 7) & 0x7F;
  sx_word = pack16(dy, dx);
  sy_word = pack16(sy * a.WNP - dy, sx * a.WNP - dx);
}

__global__ __launch_bounds__(64 * kMaxWaves) void k_grid_mfma_bf16x3(TileArgs a, const uint16_t *tab_hi,
                                                                     const uint16_t *tab_lo) {
  constexpr int kChunk = 32;                         // sample slots per MFMA K step
  __shared__ uint4 slots[kMaxWaves][kChunk];
  __shared__ uint2 queue[kMaxWaves][kQueue];
  float *tabE;
  uint32_t *thl;
  load_tables(a, tab_hi, tab_lo, tabE, thl);

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
  const unsigned WN = (unsigned)a.WN;

  f4_t acc_re = {0.0f, 0.0f, 0.0f, 0.0f}, acc_im = {0.0f, 0.0f, 0.0f, 0.0f};
  const int i16 = lane & 15, g = lane >> 4;        // MFMA operand row/column and K group
  uint4 *ss = slots[wave];
  uint2 *q = queue[wave];
  // seg_max (2, 4 or 8) sample slots per listing, kChunk / seg_max listings per chunk
  const int lg = __builtin_ctz((unsigned)a.seg_max);

  for_subtile_chunks(a, beg, end, x0, y0, true, q, kChunk >> lg, [&](int n) {
    // Stage the chunk: slot lane holds sample (lane mod seg_max) of queued record lane / seg_max.
    if (lane < kChunk) {
      uint4 sl = make_uint4(pack16(kFar, kFar), 0u, 0u, 0u);
      const int li = lane >> lg;
      const int j = lane & (a.seg_max - 1);
      if (li < n) {
        const uint2 rec = q[li];
        const int nt = (int)((rec.y >> kRecNtShift) & 7u) + 1;
        if (j < nt) {
          const int copy = (int)((rec.y >> kRecCopyBit) & 1u);
          const size_t vi = rec.x + j;
          const size_t ci = vi + (size_t)(c * (a.ncopy - 1) + copy) * copy_stride;
          const uint16_t cw = a.coords[ci];
          const float2 v = a.vis[vi];
          const float wt = a.w[vi];
          uint32_t gx, gy;
          slot_geometry(a, rec.y, cw, x0, y0, gx, gy);
          const bool ok = (cw & kCoordValid) != 0;
          sl.x = ok ? gx : sl.x;
          sl.y = ok ? gy : 0u;
          sl.z = ok ? __float_as_uint(wt * v.x) : 0u;
          sl.w = ok ? __float_as_uint(copy ? -(wt * v.y) : wt * v.y) : 0u;
        }
      }
      ss[lane] = sl;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the slot writes are visible to the wave

    // Operands.  A[y][s] = ky_s(y0 + y), row y = i16, samples s = 8g + e.
    // B[s][x] = a_s kx_s(x0 + x), column x = i16, the same samples.
    u4_t ah, al, brh, brl, bih, bil;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      uint32_t av[2];
      float kx[2], ar[2], ai[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint4 sl = ss[8 * g + 2 * p + h];
        const int ry = i16 - lo16(sl.x), rx = i16 - hi16(sl.x);
        const bool iny = (unsigned)ry < WN, inx = (unsigned)rx < WN;
        const uint32_t t = thl[iny ? lo16(sl.y) + i16 : 0];
        const float k = tabE[inx ? hi16(sl.y) + i16 : 0];
        av[h] = iny ? t : 0u;
        kx[h] = inx ? k : 0.0f;
        ar[h] = __uint_as_float(sl.z);
        ai[h] = __uint_as_float(sl.w);
      }
      ah[p] = __builtin_amdgcn_perm(av[1], av[0], 0x05040100u);
      al[p] = __builtin_amdgcn_perm(av[1], av[0], 0x07060302u);
      uint32_t hh, ll;
      split_pair(ar[0], kx[0], ar[1], kx[1], hh, ll);
      brh[p] = hh;
      brl[p] = ll;
      split_pair(ai[0], kx[0], ai[1], kx[1], hh, ll);
      bih[p] = hh;
      bil[p] = ll;
    }
    const bf8_t Ah = __builtin_bit_cast(bf8_t, ah), Al = __builtin_bit_cast(bf8_t, al);
    const bf8_t Brh = __builtin_bit_cast(bf8_t, brh), Brl = __builtin_bit_cast(bf8_t, brl);
    const bf8_t Bih = __builtin_bit_cast(bf8_t, bih), Bil = __builtin_bit_cast(bf8_t, bil);
    acc_re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Brh, acc_re, 0, 0, 0);
    acc_re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Brl, acc_re, 0, 0, 0);
    acc_re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Brh, acc_re, 0, 0, 0);
    acc_im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bih, acc_im, 0, 0, 0);
    acc_im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bil, acc_im, 0, 0, 0);
    acc_im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bih, acc_im, 0, 0, 0);
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

// DPP moves within a row of 16 lanes: mirror (lane i <-> 15 - i), half mirror
// (i <-> 7 - i in each half), and quad swaps (xor 2, xor 1).
__device__ __forceinline__ float dpp_row_mirror(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_row_half_mirror(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
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
  __shared__ uint4 dslots[kMaxWaves][kChunk];
  __shared__ uint2 queue[kMaxWaves][kQueue];
  float *tabE;
  uint32_t *thl;
  load_tables(a, tab_hi, tab_lo, tabE, thl);

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
  const unsigned WN = (unsigned)a.WN;

  // B operand, loaded once: lane (x = i16, g) holds rows 8(g & 1) + e of Re G
  // (g < 2) or Im G (g >= 2) at subtile column x.
  bf8_t bh, bl;
  {
    const float2 *gt = a.gin + ((size_t)c * a.N + y0) * a.N + x0 + i16;
    u4_t h4, l4;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const float2 v0 = gt[(size_t)(8 * (g & 1) + 2 * p) * a.N];
      const float2 v1 = gt[(size_t)(8 * (g & 1) + 2 * p + 1) * a.N];
      const uint32_t s0 = split_one(g < 2 ? v0.x : v0.y), s1 = split_one(g < 2 ? v1.x : v1.y);
      h4[p] = __builtin_amdgcn_perm(s1, s0, 0x05040100u);
      l4[p] = __builtin_amdgcn_perm(s1, s0, 0x07060302u);
    }
    bh = __builtin_bit_cast(bf8_t, h4);
    bl = __builtin_bit_cast(bf8_t, l4);
  }
  uint4 *ds = dslots[wave];
  uint2 *q = queue[wave];
  const int lg = __builtin_ctz((unsigned)a.seg_max);
  const int b3 = (i16 >> 3) & 1, b2 = (i16 >> 2) & 1, b1 = (i16 >> 1) & 1;
  const uint32_t re_mask = g < 2 ? 0xFFFFFFFFu : 0u;   // K half of this lane: real (g < 2) or imaginary

  for_subtile_chunks(a, beg, end, x0, y0, false, q, kChunk >> lg, [&](int n) {
    // Stage 16 sample slots: slot j holds sample (j mod seg_max) of queued record j / seg_max.
    if (lane < kChunk) {
      uint4 sl = make_uint4(pack16(kFar, kFar), 0u, 0xFFFFFFFFu, 0u);
      const int li = lane >> lg;
      const int j = lane & (a.seg_max - 1);
      if (li < n) {
        const uint2 rec = q[li];
        const int nt = (int)((rec.y >> kRecNtShift) & 7u) + 1;
        if (j < nt) {
          const size_t vi = rec.x + j;
          const uint16_t cw = a.coords[vi + (size_t)(c * (a.ncopy - 1)) * ((size_t)a.B * a.T)];
          uint32_t gx, gy;
          slot_geometry(a, rec.y, cw, x0, y0, gx, gy);
          const bool ok = (cw & kCoordValid) != 0;
          sl.x = ok ? gx : sl.x;
          sl.y = ok ? gy : 0u;
          sl.z = ok ? (uint32_t)vi : 0xFFFFFFFFu;
        }
      }
      ds[lane] = sl;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the slot writes are visible to the wave

    // A operand: lane (s = i16, g) holds k_y of sample s at subtile rows 8(g & 1) + e,
    // in the real half (g < 2) or the imaginary half (g >= 2) of K.
    u4_t rh, rl, ih, il;
    {
      const uint4 sl = ds[i16];
      const int dy = lo16(sl.x), yb = lo16(sl.y);
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        uint32_t av[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int y = 8 * (g & 1) + 2 * p + h;
          const bool in = (unsigned)(y - dy) < WN;
          const uint32_t t = thl[in ? yb + y : 0];
          av[h] = in ? t : 0u;
        }
        const uint32_t hp = __builtin_amdgcn_perm(av[1], av[0], 0x05040100u);
        const uint32_t lp = __builtin_amdgcn_perm(av[1], av[0], 0x07060302u);
        rh[p] = hp & re_mask;
        rl[p] = lp & re_mask;
        ih[p] = hp & ~re_mask;
        il[p] = lp & ~re_mask;
      }
    }
    const bf8_t arh = __builtin_bit_cast(bf8_t, rh), arl = __builtin_bit_cast(bf8_t, rl);
    const bf8_t aih = __builtin_bit_cast(bf8_t, ih), ail = __builtin_bit_cast(bf8_t, il);
    f4_t hr = {0.0f, 0.0f, 0.0f, 0.0f}, hi = {0.0f, 0.0f, 0.0f, 0.0f};
    hr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bh, hr, 0, 0, 0);
    hr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bl, hr, 0, 0, 0);
    hr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, bh, hr, 0, 0, 0);
    hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bh, hi, 0, 0, 0);
    hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bl, hi, 0, 0, 0);
    hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, bh, hi, 0, 0, 0);

    // H[s][x] sits in lane x + 16 (s / 4), register s % 4.  Weight by k_x, then
    // sum the 8 values v[2r + part] over the 16 columns of a lane row by halving
    // exchanges (mirror, half mirror, xor 2, xor 1): afterwards lane x holds the
    // sum of value 4 b3 + 2 b2 + b1 (bits of x), i.e. sample 4g + 2 b3 + b2, part b1.
    float v[8];
    uint32_t vis_r[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint4 sl = ds[4 * g + r];
      const int rx = i16 - hi16(sl.x);
      const bool in = (unsigned)rx < WN;
      const float k = tabE[in ? hi16(sl.y) + i16 : 0];
      const float kx = in ? k : 0.0f;
      v[2 * r] = hr[r] * kx;
      v[2 * r + 1] = hi[r] * kx;
      vis_r[r] = sl.z;
    }
    float u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float keep = b3 ? v[4 + k] : v[k], send = b3 ? v[k] : v[4 + k];
      u[k] = keep + dpp_row_mirror(send);
    }
    float w2[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const float keep = b2 ? u[2 + k] : u[k], send = b2 ? u[k] : u[2 + k];
      w2[k] = keep + dpp_row_half_mirror(send);
    }
    float z = (b1 ? w2[1] : w2[0]) + dpp_xor2(b1 ? w2[0] : w2[1]);
    z += dpp_xor1(z);
    const uint32_t vi = b3 ? (b2 ? vis_r[3] : vis_r[2]) : (b2 ? vis_r[1] : vis_r[0]);
    if (!(i16 & 1) && vi != 0xFFFFFFFFu) atomicAdd(reinterpret_cast<float *>(a.model) + 2 * (size_t)vi + b1, z);
    __builtin_amdgcn_wave_barrier();   // the next chunk's slot writes follow these reads
  });
}

}  // namespace

hipError_t launch_grid_mfma(const Plan &P, const TileArgs &a, hipStream_t s) {
  const size_t lds = (size_t)a.OS2 * a.WNP * (sizeof(float) + sizeof(uint32_t));
  const unsigned threads = 64u * (unsigned)((P.tile / kMT) * (P.tile / kMT));
  hipLaunchKernelGGL(k_grid_mfma_bf16x3, dim3((unsigned)P.nkeys), dim3(threads), lds, s, a, P.d_tab_hi,
                     P.d_tab_lo);
  return hipGetLastError();
}

hipError_t launch_degrid_mfma(const Plan &P, const TileArgs &a, hipStream_t s) {
  // the model is the sum of per-subtile partial values: start from zero
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(a.model), (int64_t)2 * P.C * P.B * P.T, 0u, s);
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)a.OS2 * a.WNP * (sizeof(float) + sizeof(uint32_t));
  const unsigned threads = 64u * (unsigned)((P.tile / kMT) * (P.tile / kMT));
  hipLaunchKernelGGL(k_degrid_mfma_bf16x3, dim3((unsigned)P.nkeys), dim3(threads), lds, s, a, P.d_tab_hi,
                     P.d_tab_lo);
  return hipGetLastError();
}

}  // namespace rts
