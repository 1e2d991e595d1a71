// Tile kernels: one workgroup owns one (channel, uv tile) of the output grid.
//
// Section 5.2 of the paper gives each block of pixels to one thread block and lets
// it read only the visibilities binned near it, staging them in shared memory.
// Here a workgroup owns a tile x tile square of one channel's grid in LDS
// (FP64 accumulator, no global atomics on grid data) and walks the work
// list of segments whose (W+1)x(W+1) window touches the tile.  A quad of lanes
// handles one segment: up to SMAX consecutive samples of one baseline that share
// the window, so the G_in window and the accumulated update stay in registers
// across the samples and reach LDS once per segment.  Consecutive samples that
// snap to the same oversampled position (most of them, since a baseline moves by
// a small fraction of a cell per time step) share their kernel rows, so the quad
// computes one degridded value and one outer-product update per run of such
// samples rather than per sample.  A segment whose window crosses a tile edge is
// listed in every tile it touches; each copy adds only the cells of its own tile,
// so every output cell has exactly one writer.
//
// Modes:
//   kGrid:   G_out = sum_s w_s V_s k_y k_x                    (Eq. (1))
//   kDegrid: M_s = sum k_y k_x G_in, written by the home listing  (adjoint)
//   kFused:  M = degrid(G_in); r = V - M; G_out = grid(r, w); chi2 partials
#pragma once

#include "internal.h"

namespace rts {

// Outputs (grid tiles, model values) are written once and not read again by the
// kernel: non-temporal stores keep them from displacing G_in windows and sample
// data in L2.
typedef float rts_nt_v4f __attribute__((ext_vector_type(4)));
typedef float rts_nt_v2f __attribute__((ext_vector_type(2)));
typedef float rts_v4f_a8 __attribute__((ext_vector_type(4), aligned(8)));   // 16 bytes at an 8-byte boundary


// Lanes per segment and window columns per lane.  A group of GROUP adjacent
// lanes shares one segment; lane q of the group owns window columns q*CPL ..
// q*CPL+CPL-1, holds those columns of the G_in window and of the accumulated
// update in registers, and the degridded value of each run of samples is the sum
// of the group's partial sums (butterfly steps inside the group of lanes).
// Minimum waves per SIMD the register allocation of the tile kernel targets for
// 128- and 512-thread workgroups (128 registers).  64-cell tiles hold a 66 KiB
// FP64 accumulator, so at most two of their workgroups share a CU; with windows
// wider than 8 cells they run 256-thread workgroups (two waves per SIMD) that
// may use up to 256 registers.
#ifndef RTS_TILE_WAVES
#define RTS_TILE_WAVES 4
#endif

// Butterfly partners inside a quad of lanes through DPP quad permutations (no LDS
// traffic, unlike a generic lane shuffle).
__device__ __forceinline__ float quad_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float quad_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}
// Sum over the quad; every lane gets the same bits ((a+b)+(c+d) in each lane's
// order, and FP addition commutes).
__device__ __forceinline__ float quad_sum(float v) {
  v += quad_xor1(v);
  return v + quad_xor2(v);
}
__device__ __forceinline__ uint32_t quad_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true));
  return max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true));
}

// Element i of a per-channel array: a uniform base and a 32-bit byte offset, so
// the loads take the scalar-base addressing form (no 64-bit address arithmetic
// per lane).  Per-channel arrays stay below 4 GiB (n_base * n_time < 2^29).
template <class T>
__device__ __forceinline__ const T *elem(const T *base, uint32_t i) {
  return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ T *elem(T *base, uint32_t i) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + i * (uint32_t)sizeof(T));
}

// One (channel, tile) of the work: zero the accumulator, walk the tile's work
// list, write the tile.  tabE must already hold the extended kernel table.
// 512-thread workgroups (64-cell tiles) take the tile's listings in batches of
// kSortBatch and visit each batch sorted by the block of tile/sort_side cells
// on a side that holds the window centre (a counting sort in LDS), so that the
// quads of a wave read overlapping G_in windows and share their cache lines.
// Bins per tile edge: 8 (8 x 8-cell blocks at tile 64) for segments of up to 4
// samples, 4 for longer segments (the sizes that measured fastest for each).
constexpr int kSortBatch = 1024;
constexpr int kSortBinsMax = 64;
template <int SMAX>
constexpr int sort_side() { return SMAX >= 8 ? 4 : 8; }
template <int BLOCK>
constexpr bool tile_sorts() { return BLOCK == 512; }

template <int WN, int SMAX, int MODE, int BLOCK, int GROUP>
__device__ __forceinline__ void tile_body(const TileArgs &a, const int key, const float *tabE, double *acc,
                                          uint2 *sorted) {
  // GROUP (= 4) lanes share a segment; each owns CPL window columns.
  static_assert(GROUP == 4, "the DPP reductions and the quad layout assume four lanes per segment");
  constexpr int kGroup = GROUP;
  constexpr int CPL = (WN + kGroup - 1) / kGroup;
  constexpr bool kFullCols = (WN % kGroup) == 0;   // every lane's columns lie in the window
  const int c = key / a.nT2;
  const int rem = key - c * a.nT2;
  const int ty = rem / a.nT, tx = rem - ty * a.nT;
  const int T = a.tile;
  const int x0 = tx * T, y0 = ty * T;
  const int TT = T * T;
  const int AS = T + kAccPad;            // accumulator row stride (cells)
  const int PL = T * AS;                 // offset of the imaginary plane

  if (MODE != kDegrid) {
    for (int i = threadIdx.x; i < 2 * PL; i += BLOCK) acc[i] = 0.0;
    __syncthreads();
  }

  const uint32_t cap = (uint32_t)a.list_cap;
  const uint32_t beg = min(a.tile_off[key], cap), end = min(a.tile_off[key + 1], cap);
  // This channel's visibilities, weights, model and packed coordinates ([C][ncopy]
  // [B][T]), and its G_in plane: listings index them with 32-bit offsets.
  const uint32_t BT = (uint32_t)a.B * (uint32_t)a.T;
  const uint32_t vbase = (uint32_t)c * BT;
  const float2 *vis_c = a.vis + vbase;
  const float *w_c = a.w + vbase;
  float2 *model_c = a.model + vbase;
  const uint16_t *coords_c = a.coords + (size_t)c * a.ncopy * BT;
  const float2 *gin_c = a.gin + (size_t)c * a.N * a.N;
  const int q = threadIdx.x & (kGroup - 1);       // lane within the group
  const int col0 = q * CPL;                       // first window column of this lane
  double chi2 = 0.0;

  constexpr uint32_t kStride = BLOCK / kGroup;
  constexpr bool kSort = tile_sorts<BLOCK>();
  constexpr int kSortSide = sort_side<SMAX>();
  constexpr int kSortBins = kSortSide * kSortSide;
  static_assert(kSortBins <= kSortBinsMax, "sort bins");
  __shared__ uint32_t sort_cnt[kSortBinsMax];
  for (uint32_t bb = beg;; bb += kSortBatch) {
  uint32_t lo = beg, hi = end;
  if constexpr (kSort) {
    if (bb >= end) break;
    const int nb = (int)min((uint32_t)kSortBatch, end - bb);
    if (threadIdx.x < kSortBins) sort_cnt[threadIdx.x] = 0u;
    __syncthreads();
    constexpr int kPer = kSortBatch / BLOCK;
    uint2 r[kPer];
    int bin[kPer];
    uint32_t pos[kPer];
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int j = (int)threadIdx.x + m * BLOCK;
      bin[m] = -1;
      if (j < nb) {
        r[m] = a.list[bb + j];
        const int cx = (int)(r[m].y & kRecXMask) - x0 + WN / 2;
        const int cy = (int)((r[m].y >> kRecYShift) & kRecXMask) - y0 + WN / 2;
        const int bx = min(max(cx, 0) * kSortSide / T, kSortSide - 1);
        const int by = min(max(cy, 0) * kSortSide / T, kSortSide - 1);
        bin[m] = by * kSortSide + bx;
        pos[m] = atomicAdd(&sort_cnt[bin[m]], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      // exclusive scan of the bin counts by one wave (a lane per bin)
      const int l = threadIdx.x;
      const uint32_t n = l < kSortBins ? sort_cnt[l] : 0u;
      uint32_t incl = n;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (l >= o) incl += t;
      }
      if (l < kSortBins) sort_cnt[l] = incl - n;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kPer; ++m)
      if (bin[m] >= 0) sorted[sort_cnt[bin[m]] + pos[m]] = r[m];
    __syncthreads();
    lo = 0;
    hi = (uint32_t)nb;
  }
  uint32_t k = lo + threadIdx.x / kGroup;
  uint2 rec_next = make_uint2(0u, 0u);
  if (k < hi) rec_next = kSort ? sorted[k] : a.list[k];
  for (; k < hi; k += kStride) {
    const uint2 rec = rec_next;
    if (k + kStride < hi) rec_next = kSort ? sorted[k + kStride] : a.list[k + kStride];   // prefetch the next record
    const bool home = (rec.y >> kRecHomeBit) & 1u;
    if (MODE == kDegrid && !home) continue;
    const int X0 = (int)(rec.y & kRecXMask);
    const int Y0 = (int)((rec.y >> kRecYShift) & kRecXMask);
    const int nt = (int)((rec.y >> kRecNtShift) & 7u) + 1;
    const int copy = (int)((rec.y >> kRecCopyBit) & 1u);
    const bool any = (rec.y >> kRecAnyBit) & 1u;
    const uint32_t vi = rec.x - vbase;          // first sample, within the channel
    const bool put_model = home && copy == 0 && (MODE == kDegrid || (MODE == kFused && a.write_model));
    if (!any) {
      if (put_model)
        for (int s = q; s < nt; s += kGroup) *elem(model_c, vi + s) = make_float2(0.0f, 0.0f);
      continue;
    }
    const uint32_t ci = vi + (uint32_t)copy * BT;

    // Issue every global load of the segment before any arithmetic: this lane's
    // columns of the G_in window first (their addresses need only the listing
    // record), then the packed coordinates of the segment's samples and the
    // visibilities and weights of this lane's own samples, so that the segment
    // waits for one memory round trip.
    // The wave issues them at raised priority, so that its round trip starts
    // before the other waves' arithmetic.
    float2 gw[WN][CPL];
    __builtin_amdgcn_s_setprio(2);
    if (MODE != kGrid) {
      const uint32_t g0 = (uint32_t)(Y0 * a.N + X0 + col0);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const uint32_t gj = g0 + (uint32_t)(j * a.N);
        if (CPL == 2 && kFullCols) {
          // the lane's two columns as one 16-byte load (8-byte aligned)
          const rts_v4f_a8 t = *reinterpret_cast<const rts_v4f_a8 *>(elem(gin_c, gj));
          gw[j][0] = make_float2(t.x, t.y);
          gw[j][CPL - 1] = make_float2(t.z, t.w);
        } else {
#pragma unroll
          for (int i = 0; i < CPL; ++i)
            gw[j][i] = (kFullCols || col0 + i < WN) ? *elem(gin_c, gj + (uint32_t)i) : make_float2(0.0f, 0.0f);
        }
      }
    }
    // Packed coordinates of all of the segment's samples (every lane finds the
    // runs below from them), and the visibilities and weights of this lane's own
    // samples q, q+4, ...
    constexpr int kMine = (SMAX + kGroup - 1) / kGroup;
    uint32_t cws[SMAX];
    // A whole track that is one segment starts SMAX-aligned: its coordinates are
    // loaded with one 16-byte (or 8-byte) vector load.
    if (a.vec && nt == SMAX) {
      if (SMAX == 8) {
        const uint4 c4 = *reinterpret_cast<const uint4 *>(elem(coords_c, ci));
        cws[0] = c4.x & 0xFFFFu; cws[1 % SMAX] = c4.x >> 16;
        cws[2 % SMAX] = c4.y & 0xFFFFu; cws[3 % SMAX] = c4.y >> 16;
        cws[4 % SMAX] = c4.z & 0xFFFFu; cws[5 % SMAX] = c4.z >> 16;
        cws[6 % SMAX] = c4.w & 0xFFFFu; cws[7 % SMAX] = c4.w >> 16;
      } else {
        const uint2 c2 = *reinterpret_cast<const uint2 *>(elem(coords_c, ci));
        cws[0] = c2.x & 0xFFFFu; cws[1 % SMAX] = c2.x >> 16;
        cws[2 % SMAX] = c2.y & 0xFFFFu; cws[3 % SMAX] = c2.y >> 16;
      }
    } else {
#pragma unroll
      for (int s = 0; s < SMAX; ++s) cws[s] = s < nt ? (uint32_t)*elem(coords_c, ci + s) : 0u;
    }
    float2 vo[kMine];
    float wo[kMine];
#pragma unroll
    for (int h = 0; h < kMine; ++h) {
      vo[h] = make_float2(0.0f, 0.0f);
      wo[h] = 0.0f;
      const int s = kGroup * h + q;
      if (MODE != kDegrid && s < nt) {
        vo[h] = *elem(vis_c, vi + s);
        wo[h] = *elem(w_c, vi + s);
      }
    }
    __builtin_amdgcn_s_setprio(0);

    // Runs.  Samples that snap to the same oversampled position have the same
    // kernel rows: they share one degridded value, and their gridding terms add up
    // before the outer product, sum_s w_s r_s k_y k_x = (sum_s w_s r_s) k_y k_x
    // (Eq. (1) regrouped).  A run is a maximal stretch of consecutive valid
    // samples with one packed coordinate; an invalid sample belongs to no run and
    // does not break one.  nrun counts the segment's runs; ko[h] is the run of own
    // sample h (-1 when it is invalid) and co[h] its packed coordinate.
    // (With SMAX < kGroup, lanes q >= SMAX own no sample.)
    int nrun = 0;
    int ko[kMine];
    uint32_t co[kMine];
#pragma unroll
    for (int h = 0; h < kMine; ++h) {
      ko[h] = -1;
      co[h] = 0u;
    }
    {
      uint32_t last = 0u;
#pragma unroll
      for (int s = 0; s < SMAX; ++s) {
        const bool ok = (cws[s] & kCoordValid) != 0;
        nrun += (ok && cws[s] != last) ? 1 : 0;
        last = ok ? cws[s] : last;
#pragma unroll
        for (int h = 0; h < kMine; ++h) {
          if (s - kGroup * h >= 0 && s - kGroup * h < kGroup && q == s - kGroup * h) {
            ko[h] = ok ? nrun - 1 : -1;
            co[h] = cws[s];
          }
        }
      }
    }
    // The accumulated update; run slot 0 (every listed segment has a valid sample)
    // initialises it.
    float2 up[WN][CPL];
    float2 mo[kMine];       // degridded values of the own samples
#pragma unroll
    for (int h = 0; h < kMine; ++h) mo[h] = make_float2(0.0f, 0.0f);
    constexpr int KYN = (WN + 3) & ~3;
    auto read_rows = [&](const uint32_t cw, float (&ky)[KYN], float (&kx)[CPL]) {
      const int sx = cw & 0x7F, sy = (cw >> 7) & 0x7F;
      const float4 *ry = reinterpret_cast<const float4 *>(tabE + sy * KYN);   // KYN == WNP, the row stride
#pragma unroll
      for (int j4 = 0; j4 < KYN / 4; ++j4) {
        const float4 t4 = ry[j4];
        ky[4 * j4] = t4.x;
        ky[4 * j4 + 1] = t4.y;
        ky[4 * j4 + 2] = t4.z;
        ky[4 * j4 + 3] = t4.w;
      }
      const float *rx = tabE + sx * KYN + col0;
      if (CPL == 2 && kFullCols) {
        const float2 t2 = *reinterpret_cast<const float2 *>(rx);
        kx[0] = t2.x;
        kx[CPL - 1] = t2.y;
      } else if (CPL == 4 && kFullCols) {
        const float4 t4 = *reinterpret_cast<const float4 *>(rx);
        kx[0] = t4.x;
        kx[1 % CPL] = t4.y;
        kx[2 % CPL] = t4.z;
        kx[3 % CPL] = t4.w;
      } else {
#pragma unroll
        for (int i = 0; i < CPL; ++i) kx[i] = (kFullCols || col0 + i < WN) ? rx[i] : 0.0f;
      }
    };
    // One slot per run; a wave runs as many slots as its segment with the most
    // runs (a slot past a segment's last run has no members and adds zeros).
    // Windows wider than 8 cells with segments of at most 4 samples run every
    // slot: without the exit between slots the compiler degrids the next slot
    // before adding this one's outer product, so the G_in window is dead before
    // the window update is live and both fit in the registers.
    constexpr bool kSkipSlots = WN <= 8 || SMAX >= 8;
    // reachx / reachy: whether any run's cell is the second one on that axis
    // (extended-table rows OS..2*OS-1); if none is, the window's last column / row
    // holds only zero taps and the flush skips it.
    const int OSh = a.OS2 >> 1;
    bool reachx = false, reachy = false;
#pragma unroll
    for (int r = 0; r < SMAX; ++r) {
      if (kSkipSlots && r > 0 && !__any(r < nrun)) break;
      // The run's coordinate (all of its members have it; the other lanes offer 0)
      // and, for gridding, its summed weight and weighted visibility, each summed
      // over the quad.
      bool mem[kMine];
      uint32_t cw = 0u;
      float sw = 0.0f, sx = 0.0f, sy = 0.0f;
#pragma unroll
      for (int h = 0; h < kMine; ++h) {
        mem[h] = ko[h] == r;
        cw = mem[h] ? co[h] : cw;
        if (MODE != kDegrid) {
          sw += mem[h] ? wo[h] : 0.0f;
          sx += mem[h] ? wo[h] * vo[h].x : 0.0f;
          sy += mem[h] ? wo[h] * vo[h].y : 0.0f;
        }
      }
      cw = quad_max_u32(cw);
      reachx = reachx || (int)(cw & 0x7F) >= OSh;
      reachy = reachy || (int)((cw >> 7) & 0x7F) >= OSh;
      if (MODE != kDegrid) {
        sw = quad_sum(sw);
        sx = quad_sum(sx);
        sy = quad_sum(sy);
      }
      float ky[KYN], kx[CPL];
      read_rows(cw, ky, kx);

      float2 m = make_float2(0.0f, 0.0f);
      if (MODE != kGrid) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
          float hr = 0.0f, hi = 0.0f;
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            hr = fmaf(ky[j], gw[j][i].x, hr);
            hi = fmaf(ky[j], gw[j][i].y, hi);
          }
          m.x = fmaf(kx[i], hr, m.x);
          m.y = fmaf(kx[i], hi, m.y);
        }
        m.x = quad_sum(m.x);
        m.y = quad_sum(m.y);
#pragma unroll
        for (int h = 0; h < kMine; ++h) mo[h] = mem[h] ? m : mo[h];
      }
      if (MODE != kDegrid) {
        // The run's gridding weight: sum of w (conj(V) for the -uv copy) less
        // the degridded value times the summed weight (the summed weighted residual).
        if (copy) sy = -sy;
        float ar = sx, ai = sy;
        if (MODE == kFused) {
          ar = fmaf(-m.x, sw, sx);
          ai = fmaf(-m.y, sw, sy);
          const bool has = r < nrun;
          ar = has ? ar : 0.0f;
          ai = has ? ai : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
          const float br = ar * kx[i], bi = ai * kx[i];
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            if (r == 0) {
              up[j][i] = make_float2(br * ky[j], bi * ky[j]);
            } else {
              up[j][i].x = fmaf(br, ky[j], up[j][i].x);
              up[j][i].y = fmaf(bi, ky[j], up[j][i].y);
            }
          }
        }
      }
    }

    if (MODE == kFused) {
      // Chi-squared of the own samples (FP32 per lane, FP64 across listings).
      float c2 = 0.0f;
#pragma unroll
      for (int h = 0; h < kMine; ++h) {
        const float rr = vo[h].x - mo[h].x;
        const float ri = (copy ? -vo[h].y : vo[h].y) - mo[h].y;
        c2 += ko[h] >= 0 ? wo[h] * fmaf(rr, rr, ri * ri) : 0.0f;
      }
      if (home) chi2 += (double)c2;
    }
    // The quad writes the model values of the segment, four consecutive samples
    // per store instruction.
    if (MODE != kGrid && put_model) {
#pragma unroll
      for (int h = 0; h < kMine; ++h)
        if (kGroup * h + q < nt) {
          const rts_nt_v2f t2 = {mo[h].x, mo[h].y};
          __builtin_nontemporal_store(t2, reinterpret_cast<rts_nt_v2f *>(elem(model_c, vi + kGroup * h + q)));
        }
    }
    if (MODE != kDegrid) {
      // Add this lane's window columns to the tile accumulator.  A wave whose
      // windows all lie inside the tile (most waves) skips the per-cell bounds
      // checks; a wave with any window across a tile edge takes the checked form
      // for all of its segments (one path per wave instead of both).
      const int lx = X0 + col0 - x0, ly = Y0 - y0;
      const bool inside = T >= WN && (unsigned)(X0 - x0) <= (unsigned)(T - WN) && (unsigned)ly <= (unsigned)(T - WN);
      double *row = acc + ly * AS + lx;           // real plane; dereferenced only inside the tile
      // Cells of the window's last column or row that no run reaches hold exact
      // zeros and are not added.
      if (__all(inside)) {
#pragma unroll
        for (int j = 0; j < WN; ++j) {
#pragma unroll
          for (int i = 0; i < CPL; ++i) {
            const bool on = (j < WN - 1 || reachy) && (col0 + i < WN - 1 || reachx);
            if ((kFullCols || col0 + i < WN) && on) {
              atomicAdd(row + i, (double)up[j][i].x);
              atomicAdd(row + PL + i, (double)up[j][i].y);
            }
          }
          row += AS;
        }
      } else {
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          if ((unsigned)(ly + j) < (unsigned)T && (j < WN - 1 || reachy)) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) {
              if ((kFullCols || col0 + i < WN) && (col0 + i < WN - 1 || reachx) && (unsigned)(lx + i) < (unsigned)T) {
                atomicAdd(row + i, (double)up[j][i].x);
                atomicAdd(row + PL + i, (double)up[j][i].y);
              }
            }
          }
          row += AS;
        }
      }
    }
  }

  if constexpr (!kSort) break;
  __syncthreads();   // the next batch overwrites the sorted listings
  }

  if (MODE == kFused) {
    __shared__ double red[BLOCK / 64];
    for (int o = 32; o > 0; o >>= 1) chi2 += __shfl_down(chi2, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = chi2;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < BLOCK / 64; ++i) t += red[i];
      a.chi2_part[key] = t;
    }
  }
  if (MODE != kDegrid) {
    __syncthreads();
    float4 *out = reinterpret_cast<float4 *>(a.gout);
    const int half = T / 2;
    for (int i = threadIdx.x; i < TT / 2; i += BLOCK) {
      const int yy = i / half, xx = i - yy * half;
      const double2 re = *reinterpret_cast<const double2 *>(acc + yy * AS + 2 * xx);
      const double2 im = *reinterpret_cast<const double2 *>(acc + PL + yy * AS + 2 * xx);
      rts_nt_v4f t4 = {(float)re.x, (float)im.x, (float)re.y, (float)im.y};
      __builtin_nontemporal_store(t4, reinterpret_cast<rts_nt_v4f *>(&out[(((size_t)c * a.N + y0 + yy) * a.N + x0) / 2 + xx]));
    }
  }
  __syncthreads();   // the accumulator and the reduction slots are reused by the next tile
}

#define RTS_TILE_ATTRS(BLOCK, GROUP) \
  __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(BLOCK != 256 ? RTS_TILE_WAVES : 2)))

// Shared-memory layout of both launches: the extended kernel table, then the FP64
// accumulator [2][tile][tile + kAccPad] (kGrid, kFused), then (512-thread
// workgroups) the sorted batch of listings.  LDS float atomics are an order of
// magnitude slower than FP64 ones on this GPU; FP64 also keeps the tile sums
// nearly independent of the order the work list is visited in.
template <int BLOCK, int MODE>
__device__ __forceinline__ float *load_table(const TileArgs &a, double *&acc, uint2 *&sorted) {
  extern __shared__ float4 smem4[];
  float *tabE = reinterpret_cast<float *>(smem4);     // [2*OS][WNP], rows 16-byte aligned
  acc = reinterpret_cast<double *>(tabE + a.OS2 * a.WNP);
  sorted = reinterpret_cast<uint2 *>(acc + (MODE != kDegrid ? 2 * a.tile * (a.tile + kAccPad) : 0));
  for (int i = threadIdx.x; i < a.OS2 * a.WNP; i += BLOCK) tabE[i] = a.tabE[i];
  __syncthreads();
  return tabE;
}

// One workgroup per (channel, tile), XCD-remapped.
template <int WN, int SMAX, int MODE, int BLOCK, int GROUP>
__global__ RTS_TILE_ATTRS(BLOCK, GROUP) void k_tile(TileArgs a) {
  double *acc;
  uint2 *sorted;
  const float *tabE = load_table<BLOCK, MODE>(a, acc, sorted);
  tile_body<WN, SMAX, MODE, BLOCK, GROUP>(a, xcd_remap(blockIdx.x, gridDim.x), tabE, acc, sorted);
}

// Persistent launch: a few workgroups per CU pull tiles from eight queues, one
// per XCD range of tiles, each holding its range in longest-first order (the
// plan's LPT order); a workgroup drains the queue of its own XCD first, then
// the others.  Every pop advances a counter, so every workgroup ends.
template <int WN, int SMAX, int MODE, int BLOCK, int GROUP>
__global__ RTS_TILE_ATTRS(BLOCK, GROUP) void k_tile_persistent(TileArgs a) {
  double *acc;
  uint2 *sorted;
  const float *tabE = load_table<BLOCK, MODE>(a, acc, sorted);
  __shared__ int item;
  const int per = (a.nkeys + 7) / 8;
  for (int k = 0; k < 8; ++k) {
    const int qi = (blockIdx.x + k) & 7;
    const int qlen = min(per, a.nkeys - qi * per);
    for (;;) {
      if (threadIdx.x == 0) item = (int)atomicAdd(&a.queue[qi], 1u);
      __syncthreads();
      const int it = item;
      __syncthreads();
      if (it >= qlen) break;
      tile_body<WN, SMAX, MODE, BLOCK, GROUP>(a, (int)a.order[qi * per + it], tabE, acc, sorted);
    }
  }
}

}  // namespace rts
