// Gridding and degridding as dense per-tile contractions on the matrix cores,
// with BF16 hi+lo split operands (or FP32 operands) and FP32 accumulation.  The
// kernel names keep the bf16x3 suffix for both operand types.
//
// For one 16x16-cell subtile of one channel, Eq. (1) restricted to the subtile is
//     G_re = Av^T diag(w Re V) Au,   G_im = Av^T diag(w Im V) Au,
// where Av[s][y] (Au[s][x]) is the kernel weight of sample s on subtile row y
// (column x), zero outside its support; degridding is its adjoint, H = Av G
// followed by the sum over columns weighted by Au.  Every operand x is split as
// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), and each product is taken
// as hi*hi + hi*lo + lo*hi (three MFMAs per block, FP32 accumulation): about 16
// significant bits per operand, relative error of a few 1e-6.  The F32 variants
// (precision fp32_mfma) take FP32 operands with v_mfma_f32_16x16x4_f32 instead,
// four samples (gridding) or four rows (degridding) per instruction: FP32
// products and accumulation, relative error ~1e-7.
//
// A workgroup owns one tile of the plan (16 to 64 cells, sorted by the plan's
// counting sort); each of its waves owns a region of one or two 16x16 subtiles
// and keeps a queue of the tile's listing records whose window touches that
// region (ballot compaction), consuming it in chunks of sample slots.
//
// The kernel tables sit in LDS as zero-padded rows: row r (one phase) holds its
// WN weights followed by R - 1 zeros, after R leading zeros, where R is the
// region edge along that axis.  A sample's slot stores the LDS byte address of
// its table entry for region row (column) 0, so the weight at row y is a plain
// read at that address + 4y: offsets outside the support land on zeros, and an
// empty slot points at the leading zeros.  Building the MFMA operands is then
// reads, packing and (for gridding) the split of w V times the column weight.
//
// With a kernel per baseline (rts_plan_set_baseline_kernels) the same padded
// rows are built per baseline in device memory (every region edge padded to 32)
// and read from there; the slot then holds word offsets into those tables.
//
// Gridding accumulators stay in registers (no atomics); degridding reduces each
// sample's partial value over the region columns with DPP and adds it to the
// (zeroed) model with FP32 atomics, one atomic instruction per chunk.
#include "internal.h"

namespace rts {
namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef unsigned u4_t __attribute__((ext_vector_type(4)));
typedef unsigned u2_t __attribute__((ext_vector_type(2)));
typedef unsigned u4w_t __attribute__((ext_vector_type(4), aligned(4)));   // 16 bytes, word-aligned

constexpr int kMT = 16;          // subtile edge (one MFMA output block)
// Listing queue per wave: at most per_chunk - 1 + 64 entries, per_chunk = staged
// slots / seg_max <= 64 / 2 (seg_max is 2, 4 or 8).
constexpr int kQueue = 96;
// Sample slots staged at once (one per lane, feeding several MFMA steps): 64 with
// regions of two subtiles (8 waves), 32 with one (up to 16 waves), which keeps
// the widest padded tables within 64 KiB of LDS.
template <int NR>
constexpr int stage_slots() { return NR == 2 ? 64 : 32; }

// Waves per workgroup: one per region; regions of two subtiles when the tile
// edge is a multiple of 32 (at most 64 / 32 * 64 / 16 = 8), else one subtile
// (at most (48 / 16)^2 = 9, for tile 48; 16 bounds it).
template <int NR>
constexpr int max_waves() { return NR == 2 ? 8 : 16; }

// Padded table geometry for region rows RH and columns RW, in words: FP32
// weights (the column weights of gridding and degridding) then packed hi|lo
// BF16 words (the row operand).
struct PadGeom {
  int SX, SA;   // row strides: WN + RW - 1 and WN + RH - 1
  int TX, TA;   // table sizes: RW + OS2 * SX and RH + OS2 * SA
};
__host__ __device__ __forceinline__ PadGeom pad_geom(int WN, int OS2, int RH, int RW) {
  PadGeom p;
  p.SX = WN + RW - 1;
  p.SA = WN + RH - 1;
  p.TX = RW + OS2 * p.SX;
  p.TA = RH + OS2 * p.SA;
  return p;
}

// Per-baseline padded tables in device memory: for baseline b, FP32 weights at
// tab[b*TX + 32 + s*SX + i] and packed hi|lo words at thl[b*TA + 32 + s*SA + i]
// (extended row s, window column i), zero elsewhere; both strides WN + 31, so
// any region edge up to 32 reads zeros off the support.
struct PbTables {
  uint32_t *thl;
  float *tab;
  int TA, TX, SA, SX;
};
constexpr int kPbPad = 32;

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

// Low halves (hi parts) and high halves (lo parts) of two packed words, as one word.
__device__ __forceinline__ uint32_t lows(uint32_t w0, uint32_t w1) { return __builtin_amdgcn_perm(w1, w0, 0x05040100u); }
__device__ __forceinline__ uint32_t highs(uint32_t w0, uint32_t w1) { return __builtin_amdgcn_perm(w1, w0, 0x07060302u); }

// Padded tables into LDS (layout above); returns the LDS base.  Zero the whole
// area (16-byte stores; the launch rounds it up to whole 16-byte words), then
// place the WN weights of each phase row, 32 threads per row.
__device__ __forceinline__ const char *load_padded_tables(const TileArgs &a, const uint16_t *tab_hi,
                                                          const uint16_t *tab_lo, const PadGeom &pg, int RH,
                                                          int RW, bool f32) {
  extern __shared__ float4 smem4[];
  const int n4 = (pg.TX + pg.TA + 3) >> 2;
  for (int i = threadIdx.x; i < n4; i += blockDim.x) smem4[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  __syncthreads();
  float *tab = reinterpret_cast<float *>(smem4);
  uint32_t *thl = reinterpret_cast<uint32_t *>(tab + pg.TX);
  for (int i = threadIdx.x; i < a.OS2 * 32; i += blockDim.x) {
    const int r = i >> 5, t = i & 31;
    if (t < a.WN) {
      const int src = r * a.WNP + t;
      tab[RW + r * pg.SX + t] = a.tabE[src];
      thl[RH + r * pg.SA + t] = f32 ? __float_as_uint(a.tabE[src])
                                    : (uint32_t)tab_hi[src] | ((uint32_t)tab_lo[src] << 16);
    }
  }
  __syncthreads();
  return reinterpret_cast<const char *>(smem4);
}

__device__ __forceinline__ uint32_t lds_u32(const char *lds, uint32_t byte) {
  return *reinterpret_cast<const uint32_t *>(lds + byte);
}
__device__ __forceinline__ float lds_f32(const char *lds, uint32_t byte) {
  return *reinterpret_cast<const float *>(lds + byte);
}

// Walk the tile's listings and call chunk(n) whenever the wave's queue holds
// `per_chunk` records whose window overlaps the rw x rh region at (x0, y0) (and
// once more for the remainder).  q: the wave's queue of records; chunk reads
// q[0..n).  The next 64 records are loaded while the current ones are used.
template <class Chunk>
__device__ __forceinline__ void for_subtile_chunks(const TileArgs &a, uint32_t beg, uint32_t end, int x0, int y0,
                                                   int rw, int rh, bool with_copies, uint2 *q, int per_chunk,
                                                   Chunk chunk) {
  const int lane = threadIdx.x & 63;
  int qn = 0;                                        // wave-uniform
  uint2 nrec = make_uint2(0u, 0u);
  if (beg + (uint32_t)lane < end) nrec = a.list[beg + lane];
  for (uint32_t base = beg; base < end; base += 64) {
    const uint32_t k = base + (uint32_t)lane;
    bool ov = false;
    const uint2 rec = nrec;
    if (k + 64 < end) nrec = a.list[k + 64];
    if (k < end) {
      const bool any = (rec.y >> kRecAnyBit) & 1u;
      const bool copy = (rec.y >> kRecCopyBit) & 1u;
      const int X0 = (int)(rec.y & kRecXMask), Y0 = (int)((rec.y >> kRecYShift) & kRecXMask);
      ov = any && (with_copies || !copy) && X0 < x0 + rw && X0 + a.WN > x0 && Y0 < y0 + rh && Y0 + a.WN > y0;
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

// The (channel, tile) key of this workgroup, or -1 for a workgroup with none.
// With a longest-first order (a.order), workgroup b takes position b / 8 of
// eighth b mod 8 of the tile range: each XCD (workgroups go to the eight XCDs in
// turn) walks one contiguous eighth, its heaviest tiles first, which shortens
// the tail where a few dense uv tiles would otherwise run last.  Without it,
// xcd_remap gives each XCD its eighth in key order.
__device__ __forceinline__ int tile_key(const TileArgs &a) {
  if (!a.order) return xcd_remap(blockIdx.x, gridDim.x);
  const int per = (a.nkeys + 7) / 8;
  const int g = blockIdx.x & 7, i = blockIdx.x >> 3;
  if (i >= min(per, a.nkeys - g * per)) return -1;
  return (int)a.order[g * per + i];
}

// LDS byte addresses of a sample's table entries for region row 0 (packed hi|lo
// row weights) and region column 0 (FP32 column weights).  The queue filter
// keeps dy in [-(WN-1), RH-1] and dx in [-(WN-1), RW-1], so every read at
// + 4y (y < RH) or + 4x (x < RW) stays inside the sample's padded row.
__device__ __forceinline__ void slot_addresses(const TileArgs &a, const PadGeom &pg, int RH, int RW, uint32_t recy,
                                               uint16_t cw, int x0, int y0, uint32_t &ya, uint32_t &xa) {
  const int dx = (int)(recy & kRecXMask) - x0;
  const int dy = (int)((recy >> kRecYShift) & kRecXMask) - y0;
  const int sx = cw & 0x7F, sy = (cw >> 7) & 0x7F;
  ya = 4u * (uint32_t)(pg.TX + RH + sy * pg.SA - dy);
  xa = 4u * (uint32_t)(RW + sx * pg.SX - dx);
}

// Word offsets of a sample's per-baseline table entries for region row and
// column 0 (the per-baseline form of slot_addresses); vi is the visibility index
// (c*B + b)*T + t.
__device__ __forceinline__ void slot_offsets_pb(const TileArgs &a, const PbTables &pb, uint32_t vi, uint32_t recy,
                                                uint16_t cw, int x0, int y0, uint32_t &ya, uint32_t &xa) {
  const int dx = (int)(recy & kRecXMask) - x0;
  const int dy = (int)((recy >> kRecYShift) & kRecXMask) - y0;
  const int sx = cw & 0x7F, sy = (cw >> 7) & 0x7F;
  const uint32_t bl = (vi / (uint32_t)a.T) % (uint32_t)a.B;
  ya = bl * (uint32_t)pb.TA + (uint32_t)(kPbPad + sy * pb.SA - dy);
  xa = bl * (uint32_t)pb.TX + (uint32_t)(kPbPad + sx * pb.SX - dx);
}

// Gridding of a region of GR x 1 subtiles (16 GR rows, 16 columns): the B
// operand (w V times the column weights, the costlier one to build) is shared
// by the GR row blocks.  One v_mfma_f32_16x16x32_bf16 per term and block: K
// runs over 32 sample slots.  Registers are capped at 80 so that three
// workgroups of 8 waves share a CU.
template <int GR, bool PB, bool F32, bool RES>
__global__ __launch_bounds__(64 * max_waves<GR>()) __attribute__((amdgpu_waves_per_eu(6)))
void k_grid_mfma_bf16x3(TileArgs a, const uint16_t *tab_hi, const uint16_t *tab_lo, PbTables pb) {
  constexpr int kChunk = 32;                         // sample slots per MFMA K step
  constexpr int RH = GR * kMT, RW = kMT;
  constexpr int kStage = stage_slots<GR>();
  __shared__ uint4 slots[max_waves<GR>()][kStage];
  __shared__ uint2 queue[max_waves<GR>()][kQueue];
  const int key = tile_key(a);
  if (key < 0) return;
  const PadGeom pg = pad_geom(a.WN, a.OS2, RH, RW);
  const char *lds = PB ? nullptr : load_padded_tables(a, tab_hi, tab_lo, pg, RH, RW, F32);

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int nwx = a.tile / RW;                      // regions per tile row
  const int c = key / a.nT2;
  const int rem = key - c * a.nT2;
  const int ty = rem / a.nT, tx = rem - ty * a.nT;
  const int x0 = tx * a.tile + RW * (wave % nwx), y0 = ty * a.tile + RH * (wave / nwx);
  const uint32_t cap = (uint32_t)a.list_cap;
  const uint32_t beg = min(a.tile_off[key], cap), end = min(a.tile_off[key + 1], cap);
  const size_t copy_stride = (size_t)a.B * a.T;
  const uint32_t empty_ya = PB ? 0u : 4u * (uint32_t)pg.TX, empty_xa = 0u;

  f4_t acc_re[GR], acc_im[GR];
#pragma unroll
  for (int rb = 0; rb < GR; ++rb) {
    acc_re[rb] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
    acc_im[rb] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
  }
  const int i16 = lane & 15, g = lane >> 4;        // MFMA operand row/column and K group
  uint4 *ss = slots[wave];
  uint2 *q = queue[wave];
  // seg_max (2, 4 or 8) sample slots per listing, kChunk / seg_max listings per chunk
  const int lg = __builtin_ctz((unsigned)a.seg_max);
  // Residual form: this wave's share of chi2 = sum w |V - M|^2, each sample
  // counted once, by the wave whose region holds its window origin in the home
  // listing of its segment.
  double chi2 = 0.0;

  // Contraction of nsteps K steps of staged slots.
  auto contract = [&](const uint4 *sb, int nsteps) {
    for (int ks = 0; ks < nsteps; ++ks) {
    const uint4 *sk = sb + kChunk * ks;
    if constexpr (F32) {
      // FP32 operands, one v_mfma_f32_16x16x4_f32 per term, row block and step of
      // 4 samples s = 4 st + g: A_rb[y][g] = ky_s(y0 + 16 rb + y) in lane y + 16g,
      // B[g][x] = a_s kx_s(x0 + x) in lane x + 16g.
#pragma unroll
      for (int st = 0; st < kChunk / 4; ++st) {
        const uint4 sl = sk[4 * st + g];
        float av[GR], kx;
        if (PB) {
#pragma unroll
          for (int rb = 0; rb < GR; ++rb) av[rb] = __uint_as_float(pb.thl[sl.x + i16 + kMT * rb]);
          kx = pb.tab[sl.y + i16];
        } else {
#pragma unroll
          for (int rb = 0; rb < GR; ++rb) av[rb] = lds_f32(lds, sl.x + 4u * i16 + 4u * kMT * rb);
          kx = lds_f32(lds, sl.y + 4u * i16);
        }
        const float br = __uint_as_float(sl.z) * kx, bi = __uint_as_float(sl.w) * kx;
#pragma unroll
        for (int rb = 0; rb < GR; ++rb) {
          acc_re[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb], br, acc_re[rb], 0, 0, 0);
          acc_im[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb], bi, acc_im[rb], 0, 0, 0);
        }
      }
    } else {
      // Operands.  A_rb[y][s] = ky_s(y0 + 16 rb + y), row y = i16, samples s = 8g + e.
      // B[s][x] = a_s kx_s(x0 + x), column x = i16, the same samples.
      u4_t ah[GR], al[GR], brh, brl, bih, bil;
  #pragma unroll
      for (int p = 0; p < 4; ++p) {
        uint32_t av[GR][2];
        float kx[2], ar[2], ai[2];
  #pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint4 sl = sk[8 * g + 2 * p + h];
          if (PB) {
            const uint32_t ya = sl.x + i16, xa = sl.y + i16;
  #pragma unroll
            for (int rb = 0; rb < GR; ++rb) av[rb][h] = pb.thl[ya + kMT * rb];
            kx[h] = pb.tab[xa];
          } else {
            const uint32_t ya = sl.x + 4u * i16, xa = sl.y + 4u * i16;
  #pragma unroll
            for (int rb = 0; rb < GR; ++rb) av[rb][h] = lds_u32(lds, ya + 4u * kMT * rb);
            kx[h] = lds_f32(lds, xa);
          }
          ar[h] = __uint_as_float(sl.z);
          ai[h] = __uint_as_float(sl.w);
        }
  #pragma unroll
        for (int rb = 0; rb < GR; ++rb) {
          ah[rb][p] = lows(av[rb][0], av[rb][1]);
          al[rb][p] = highs(av[rb][0], av[rb][1]);
        }
        uint32_t hh, ll;
        split_pair(ar[0], kx[0], ar[1], kx[1], hh, ll);
        brh[p] = hh;
        brl[p] = ll;
        split_pair(ai[0], kx[0], ai[1], kx[1], hh, ll);
        bih[p] = hh;
        bil[p] = ll;
      }
      const bf8_t Brh = __builtin_bit_cast(bf8_t, brh), Brl = __builtin_bit_cast(bf8_t, brl);
      const bf8_t Bih = __builtin_bit_cast(bf8_t, bih), Bil = __builtin_bit_cast(bf8_t, bil);
  #pragma unroll
      for (int rb = 0; rb < GR; ++rb) {
        const bf8_t Ah = __builtin_bit_cast(bf8_t, ah[rb]), Al = __builtin_bit_cast(bf8_t, al[rb]);
        acc_re[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Brh, acc_re[rb], 0, 0, 0);
        acc_re[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Brl, acc_re[rb], 0, 0, 0);
        acc_re[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Brh, acc_re[rb], 0, 0, 0);
        acc_im[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bih, acc_im[rb], 0, 0, 0);
        acc_im[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bil, acc_im[rb], 0, 0, 0);
        acc_im[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bih, acc_im[rb], 0, 0, 0);
      }
    }
    }
  };
  for_subtile_chunks(a, beg, end, x0, y0, RW, RH, true, q, kStage >> lg, [&](int n) {
    // Stage kStage slots, one per lane: slot lane holds sample (lane mod seg_max)
    // of queued record lane / seg_max.  They feed up to kStage / 32 K steps.
    if (kStage == 64 || lane < kStage) {
      uint4 sl = make_uint4(empty_ya, empty_xa, 0u, 0u);
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
          float2 v = a.vis[vi];
          const float wt = a.w[vi];
          if (RES) {                                 // the fused step grids w (V - M)
            const float2 m = a.model[vi];
            v.x -= m.x;
            v.y -= m.y;
            const int dx0 = (int)(rec.y & kRecXMask) - x0;
            const int dy0 = (int)((rec.y >> kRecYShift) & kRecXMask) - y0;
            const bool mine = ((rec.y >> kRecHomeBit) & 1u) && copy == 0 && (unsigned)dx0 < (unsigned)RW &&
                              (unsigned)dy0 < (unsigned)RH && (cw & kCoordValid);
            if (mine) chi2 += (double)(wt * fmaf(v.x, v.x, v.y * v.y));
          }
          uint32_t ya, xa;
          if (PB)
            slot_offsets_pb(a, pb, (uint32_t)vi, rec.y, cw, x0, y0, ya, xa);
          else
            slot_addresses(a, pg, RH, RW, rec.y, cw, x0, y0, ya, xa);
          const bool ok = (cw & kCoordValid) != 0;
          sl.x = ok ? ya : empty_ya;
          sl.y = ok ? xa : empty_xa;
          sl.z = ok ? __float_as_uint(wt * v.x) : 0u;
          sl.w = ok ? __float_as_uint(copy ? -(wt * v.y) : wt * v.y) : 0u;
        }
      }
      ss[lane] = sl;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the slot writes are visible to the wave
    contract(ss, (n << lg) > kChunk ? 2 : 1);   // the second K step only when its slots hold samples
    __builtin_amdgcn_wave_barrier();   // the next chunk's slot writes follow these reads
  });

  if constexpr (RES) {
    // one partial chi2 per workgroup (every key has exactly one workgroup)
    __shared__ double red[max_waves<GR>()];
    for (int o = 32; o > 0; o >>= 1) chi2 += __shfl_down(chi2, o, 64);
    if (lane == 0) red[wave] = chi2;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
      a.chi2_part[key] = t;
    }
  }

  // D[y][x] of row block rb sits in lane x + 16 * (y / 4), register y % 4.
  float2 *out = a.gout + ((size_t)c * a.N + y0) * a.N + x0;
#pragma unroll
  for (int rb = 0; rb < GR; ++rb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int y = kMT * rb + 4 * g + r;
      out[(size_t)y * a.N + i16] = make_float2(acc_re[rb][r], acc_im[rb][r]);
    }
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

// Degridding of a region of 1 x DC subtiles (16 rows, 16 DC columns): for the
// queued samples (16 at a time, rows of the MFMA), H = Av G holds, per sample
// and region column x, the sum over the region's rows of k_y * G, formed with
// v_mfma_f32_16x16x16_bf16 (K = the 16 rows) separately for Re G and Im G; the
// A operand (k_y) is shared by the DC column blocks.  The sample's partial
// model value over the region is sum_x H[s][x] k_x(x).  A window crossing
// region edges is covered by every region it touches, so the partial values are
// added to the (zeroed) model with FP32 atomics.
template <int DC, bool PB, bool F32>
__global__ __launch_bounds__(64 * max_waves<DC>()) void k_degrid_mfma_bf16x3(TileArgs a, const uint16_t *tab_hi,
                                                                             const uint16_t *tab_lo, PbTables pb) {
  constexpr int kChunk = 16;                         // samples per MFMA step (its rows)
  constexpr int RH = kMT, RW = DC * kMT;
  constexpr int kStage = stage_slots<DC>();
  __shared__ uint4 dslots[max_waves<DC>()][kStage];
  __shared__ uint2 queue[max_waves<DC>()][kQueue];
  const int key = tile_key(a);
  if (key < 0) return;
  const PadGeom pg = pad_geom(a.WN, a.OS2, RH, RW);
  const char *lds = PB ? nullptr : load_padded_tables(a, tab_hi, tab_lo, pg, RH, RW, F32);

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nwx = a.tile / RW;                      // regions per tile row
  const int c = key / a.nT2;
  const int rem = key - c * a.nT2;
  const int ty = rem / a.nT, tx = rem - ty * a.nT;
  const int x0 = tx * a.tile + RW * (wave % nwx), y0 = ty * a.tile + RH * (wave / nwx);
  const uint32_t cap = (uint32_t)a.list_cap;
  const uint32_t beg = min(a.tile_off[key], cap), end = min(a.tile_off[key + 1], cap);
  const int i16 = lane & 15, g = lane >> 4;
  const uint32_t empty_ya = PB ? 0u : 4u * (uint32_t)pg.TX, empty_xa = 0u;

  // B operands, loaded once.  BF16x3: lane (x = i16, g) of block cb holds rows
  // 4g + e of Re G and Im G at region column 16 cb + x, split into hi and lo
  // parts.  FP32: lane (x, g) holds row 4t + g of K step t (gre, gim).
  s4_t brh[DC], brl[DC], bih[DC], bil[DC];
  float gre[DC][4], gim[DC][4];
  if (F32) {
#pragma unroll
    for (int cb = 0; cb < DC; ++cb) {
      const float2 *gt = a.gin + ((size_t)c * a.N + y0 + g) * a.N + x0 + kMT * cb + i16;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float2 v = gt[(size_t)(4 * t) * a.N];
        gre[cb][t] = v.x;
        gim[cb][t] = v.y;
      }
    }
  }
#pragma unroll
  for (int cb = 0; cb < (F32 ? 0 : DC); ++cb) {
    const float2 *gt = a.gin + ((size_t)c * a.N + y0 + 4 * g) * a.N + x0 + kMT * cb + i16;
    uint32_t sr[4], si[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float2 v = gt[(size_t)e * a.N];
      sr[e] = split_one(v.x);
      si[e] = split_one(v.y);
    }
    brh[cb] = __builtin_bit_cast(s4_t, u2_t{lows(sr[0], sr[1]), lows(sr[2], sr[3])});
    brl[cb] = __builtin_bit_cast(s4_t, u2_t{highs(sr[0], sr[1]), highs(sr[2], sr[3])});
    bih[cb] = __builtin_bit_cast(s4_t, u2_t{lows(si[0], si[1]), lows(si[2], si[3])});
    bil[cb] = __builtin_bit_cast(s4_t, u2_t{highs(si[0], si[1]), highs(si[2], si[3])});
  }
  uint4 *ds = dslots[wave];
  uint2 *q = queue[wave];
  const int lg = __builtin_ctz((unsigned)a.seg_max);
  const int b3 = (i16 >> 3) & 1, b2 = (i16 >> 2) & 1, b1 = (i16 >> 1) & 1;

  for_subtile_chunks(a, beg, end, x0, y0, RW, RH, false, q, kStage >> lg, [&](int n) {
    // Stage kStage sample slots, one per lane: slot j holds sample (j mod seg_max)
    // of queued record j / seg_max.  They feed up to kStage / 16 steps of 16 samples.
    if (kStage == 64 || lane < kStage) {
      uint4 sl = make_uint4(empty_ya, empty_xa, 0xFFFFFFFFu, 0u);
      const int li = lane >> lg;
      const int j = lane & (a.seg_max - 1);
      if (li < n) {
        const uint2 rec = q[li];
        const int nt = (int)((rec.y >> kRecNtShift) & 7u) + 1;
        if (j < nt) {
          const size_t vi = rec.x + j;
          const uint16_t cw = a.coords[vi + (size_t)(c * (a.ncopy - 1)) * ((size_t)a.B * a.T)];
          uint32_t ya, xa;
          if (PB)
            slot_offsets_pb(a, pb, (uint32_t)vi, rec.y, cw, x0, y0, ya, xa);
          else
            slot_addresses(a, pg, RH, RW, rec.y, cw, x0, y0, ya, xa);
          const bool ok = (cw & kCoordValid) != 0;
          sl.x = ok ? ya : empty_ya;
          sl.y = ok ? xa : empty_xa;
          sl.z = ok ? (uint32_t)vi : 0xFFFFFFFFu;
        }
      }
      ds[lane] = sl;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the slot writes are visible to the wave

    const int nsteps = ((n << lg) + kChunk - 1) / kChunk;   // steps holding samples (wave-uniform)
    for (int ks = 0; ks < nsteps; ++ks) {
    const uint4 *dk = ds + kChunk * ks;
    // Column weights of the samples 4g + r whose H rows this lane receives.  From
    // device memory (per-baseline tables), or ahead of the longer FP32-operand
    // contraction, they are read before it so that the reads overlap it; for the
    // BF16x3 contraction from LDS, after it (fewer live registers).
    float kxv[4][DC];
    uint32_t vis_r[4];
    auto column_weights = [&]() {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint4 sl = dk[4 * g + r];
#pragma unroll
        for (int cb = 0; cb < DC; ++cb)
          kxv[r][cb] = PB ? pb.tab[sl.y + i16 + kMT * cb] : lds_f32(lds, sl.y + 4u * i16 + 4u * kMT * cb);
        vis_r[r] = sl.z;
      }
    };
    if (PB || F32) column_weights();
    f4_t hr[DC], hi[DC];
    if constexpr (F32) {
      // FP32: K step t covers region rows 4t + g; A[s][g] = k_y of sample s = i16.
      const uint32_t ya = dk[i16].x;
#pragma unroll
      for (int cb = 0; cb < DC; ++cb) hr[cb] = hi[cb] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float av = PB ? __uint_as_float(pb.thl[ya + 4u * t + g]) : lds_f32(lds, ya + 4u * (4u * t + g));
#pragma unroll
        for (int cb = 0; cb < DC; ++cb) {
          hr[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, gre[cb][t], hr[cb], 0, 0, 0);
          hi[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, gim[cb][t], hi[cb], 0, 0, 0);
        }
      }
    } else {
      // A operand: lane (s = i16, g) holds k_y of sample s at region rows 4g + e.
      s4_t ah, al;
      {
        uint32_t t0, t1, t2, t3;
        if (PB) {
          // four consecutive words at any word offset: a 16-byte load with 4-byte alignment
          const u4w_t t = *reinterpret_cast<const u4w_t *>(pb.thl + dk[i16].x + 4u * g);
          t0 = t[0];
          t1 = t[1];
          t2 = t[2];
          t3 = t[3];
        } else {
          const uint32_t ya = dk[i16].x + 16u * g;
          t0 = lds_u32(lds, ya);
          t1 = lds_u32(lds, ya + 4u);
          t2 = lds_u32(lds, ya + 8u);
          t3 = lds_u32(lds, ya + 12u);
        }
        ah = __builtin_bit_cast(s4_t, u2_t{lows(t0, t1), lows(t2, t3)});
        al = __builtin_bit_cast(s4_t, u2_t{highs(t0, t1), highs(t2, t3)});
      }
  #pragma unroll
      for (int cb = 0; cb < DC; ++cb) {
        const f4_t z = {0.0f, 0.0f, 0.0f, 0.0f};
        hr[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, brh[cb], z, 0, 0, 0);
        hr[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, brl[cb], hr[cb], 0, 0, 0);
        hr[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, brh[cb], hr[cb], 0, 0, 0);
        hi[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bih[cb], z, 0, 0, 0);
        hi[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bil[cb], hi[cb], 0, 0, 0);
        hi[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bih[cb], hi[cb], 0, 0, 0);
      }
    }

    // H_cb[s][x] sits in lane x + 16 (s / 4), register s % 4.  Weight by k_x and
    // add the column blocks, then sum the 8 values v[2r + part] over the 16
    // columns of a lane row by halving exchanges (mirror, half mirror, xor 2,
    // xor 1): afterwards lane x holds the sum of value 4 b3 + 2 b2 + b1 (bits of
    // x), i.e. sample 4g + 2 b3 + b2, part b1.
    if (!PB && !F32) column_weights();
    float v[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v[2 * r] = v[2 * r + 1] = 0.0f;
#pragma unroll
      for (int cb = 0; cb < DC; ++cb) {
        v[2 * r] += hr[cb][r] * kxv[r][cb];
        v[2 * r + 1] += hi[cb][r] * kxv[r][cb];
      }
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
    }
    __builtin_amdgcn_wave_barrier();   // the next chunk's slot writes follow these reads
  });
}

size_t padded_lds_bytes(const TileArgs &a, int RH, int RW) {
  const PadGeom pg = pad_geom(a.WN, a.OS2, RH, RW);
  return (size_t)16 * (size_t)((pg.TX + pg.TA + 3) / 4);
}

PbTables pb_tables(const Plan &P) {
  PbTables pb{};
  pb.thl = P.d_pb_thl;
  pb.tab = P.d_pb_tab;
  pb.SA = pb.SX = P.WN + kPbPad - 1;
  pb.TA = pb.TX = kPbPad + 2 * P.OS * pb.SA;
  return pb;
}

// Per-baseline padded rows from the caller's [B][OS][W] table (layout above).
__global__ void k_build_pb_tables(const float *__restrict__ tab, int64_t total, int OS, int W, int WN, PbTables pb,
                                  int f32) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int per = 2 * OS * WN;
  const int64_t b = idx / per;
  const int rem = (int)(idx - b * per);
  const int srow = rem / WN, i = rem - srow * WN;
  const int d = srow / OS, p = srow - d * OS, j = i - d;
  const float v = (j >= 0 && j < W) ? tab[(b * OS + p) * W + j] : 0.0f;
  pb.tab[b * pb.TX + kPbPad + srow * pb.SX + i] = v;
  const __bf16 h = (__bf16)v;
  const __bf16 l = (__bf16)(v - (float)h);
  const uint32_t w = f32 ? __float_as_uint(v)
                         : (uint32_t)__builtin_bit_cast(uint16_t, h) | ((uint32_t)__builtin_bit_cast(uint16_t, l) << 16);
  pb.thl[b * pb.TA + kPbPad + srow * pb.SA + i] = w;
}

}  // namespace

size_t mfma_lds_bytes(int WN, int OS2, int tile) {
  const int pair = tile % (2 * kMT) == 0 ? 2 : 1;
  const size_t waves = (size_t)max_waves<1>();
  const size_t grid_static = pair == 2 ? (size_t)max_waves<2>() * (stage_slots<2>() * 16 + kQueue * 8)
                                       : waves * (stage_slots<1>() * 16 + kQueue * 8);
  const size_t degrid_static = grid_static;
  const PadGeom g = pad_geom(WN, OS2, pair * kMT, kMT), d = pad_geom(WN, OS2, kMT, pair * kMT);
  const size_t gl = grid_static + (size_t)16 * ((g.TX + g.TA + 3) / 4);
  const size_t dl = degrid_static + (size_t)16 * ((d.TX + d.TA + 3) / 4);
  return std::max(gl, dl);
}

int64_t pb_table_words(const Plan &P) {
  return (int64_t)P.B * (kPbPad + 2 * P.OS * (P.WN + kPbPad - 1));
}

hipError_t build_baseline_tables(const Plan &P, const float *tab, hipStream_t s) {
  const PbTables pb = pb_tables(P);
  const int64_t words = pb_table_words(P);
  hipError_t e = launch_fill_u32(P.d_pb_thl, words, 0u, s);
  if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t *>(P.d_pb_tab), words, 0u, s);
  if (e != hipSuccess) return e;
  const int64_t total = (int64_t)P.B * 2 * P.OS * P.WN;
  hipLaunchKernelGGL(k_build_pb_tables, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, tab, total, P.OS,
                     P.W, P.WN, pb, (int)(P.precision == RTS_PREC_FP32_MFMA));
  return hipGetLastError();
}

// Workgroups to launch: one per key, or 8 * ceil(nkeys / 8) with the
// longest-first order (see tile_key).
static unsigned mfma_grid_size(const Plan &P, const TileArgs &a) {
  return a.order ? (unsigned)(8 * ((P.nkeys + 7) / 8)) : (unsigned)P.nkeys;
}

template <int NR, bool PB, bool F32>
void launch_grid_variant(const Plan &P, const TileArgs &a, hipStream_t s, const PbTables &pb, unsigned threads,
                         size_t lds) {
  hipLaunchKernelGGL((k_grid_mfma_bf16x3<NR, PB, F32, false>), dim3(mfma_grid_size(P, a)), dim3(threads), lds,
                     s, a, P.d_tab_hi, P.d_tab_lo, pb);
}

template <int NR, bool PB, bool F32>
void launch_resid_variant(const Plan &P, const TileArgs &a, hipStream_t s, const PbTables &pb, unsigned threads,
                          size_t lds) {
  hipLaunchKernelGGL((k_grid_mfma_bf16x3<NR, PB, F32, true>), dim3(mfma_grid_size(P, a)), dim3(threads), lds,
                     s, a, P.d_tab_hi, P.d_tab_lo, pb);
}

template <int NR, bool PB, bool F32>
void launch_degrid_variant(const Plan &P, const TileArgs &a, hipStream_t s, const PbTables &pb, unsigned threads,
                           size_t lds) {
  hipLaunchKernelGGL((k_degrid_mfma_bf16x3<NR, PB, F32>), dim3(mfma_grid_size(P, a)), dim3(threads), lds, s, a,
                     P.d_tab_hi, P.d_tab_lo, pb);
}

// The kernel variant for (regions of two subtiles when the tile edge is a
// multiple of 32, per-baseline tables, FP32 operands).
#define RTS_MFMA_PICK(fn)                                                                                       \
  do {                                                                                                         \
    const int code = (pair == 2 ? 4 : 0) | (pbk ? 2 : 0) | (f32 ? 1 : 0);                                      \
    switch (code) {                                                                                            \
      case 0: fn<1, false, false>(P, a, s, pb, threads, lds); break;                                          \
      case 1: fn<1, false, true>(P, a, s, pb, threads, lds); break;                                           \
      case 2: fn<1, true, false>(P, a, s, pb, threads, lds); break;                                           \
      case 3: fn<1, true, true>(P, a, s, pb, threads, lds); break;                                            \
      case 4: fn<2, false, false>(P, a, s, pb, threads, lds); break;                                          \
      case 5: fn<2, false, true>(P, a, s, pb, threads, lds); break;                                           \
      case 6: fn<2, true, false>(P, a, s, pb, threads, lds); break;                                           \
      default: fn<2, true, true>(P, a, s, pb, threads, lds); break;                                           \
    }                                                                                                          \
  } while (0)

hipError_t launch_grid_mfma(const Plan &P, const TileArgs &a, hipStream_t s) {
  const int pair = P.tile % (2 * kMT) == 0 ? 2 : 1;
  const unsigned threads = 64u * (unsigned)((P.tile / kMT) * (P.tile / kMT) / pair);
  const bool pbk = P.d_pb_thl != nullptr, f32 = P.precision == RTS_PREC_FP32_MFMA;
  const size_t lds = pbk ? 0 : padded_lds_bytes(a, pair * kMT, kMT);
  const PbTables pb = pb_tables(P);
  RTS_MFMA_PICK(launch_grid_variant);
  return hipGetLastError();
}

hipError_t launch_degrid_mfma(const Plan &P, const TileArgs &a, hipStream_t s) {
  // the model is the sum of per-region partial values: start from zero
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(a.model), (int64_t)2 * P.C * P.B * P.T, 0u, s);
  if (e != hipSuccess) return e;
  const int pair = P.tile % (2 * kMT) == 0 ? 2 : 1;
  const unsigned threads = 64u * (unsigned)((P.tile / kMT) * (P.tile / kMT) / pair);
  const bool pbk = P.d_pb_thl != nullptr, f32 = P.precision == RTS_PREC_FP32_MFMA;
  const size_t lds = pbk ? 0 : padded_lds_bytes(a, kMT, pair * kMT);
  const PbTables pb = pb_tables(P);
  RTS_MFMA_PICK(launch_degrid_variant);
  return hipGetLastError();
}

// The fused step's gridding pass: w (V - M) over the valid samples, M the model
// written by launch_degrid_mfma into a.model; it also leaves one partial sum of
// chi2 per key in a.chi2_part.
hipError_t launch_grid_resid_mfma(const Plan &P, const TileArgs &a, hipStream_t s) {
  const int pair = P.tile % (2 * kMT) == 0 ? 2 : 1;
  const unsigned threads = 64u * (unsigned)((P.tile / kMT) * (P.tile / kMT) / pair);
  const bool pbk = P.d_pb_thl != nullptr, f32 = P.precision == RTS_PREC_FP32_MFMA;
  const size_t lds = pbk ? 0 : padded_lds_bytes(a, pair * kMT, kMT);
  const PbTables pb = pb_tables(P);
  RTS_MFMA_PICK(launch_resid_variant);
  return hipGetLastError();
}


}  // namespace rts
