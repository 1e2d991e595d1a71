// Plan kernels: FP64 uv -> grid coordinates, segmentation of each baseline's
// track, and the counting sort of (segment, tile) listings by (channel, tile).
//
// Section 5.2 of the paper bins visibilities by uv bin and sorts them so that a
// workgroup reads only the visibilities near its pixels.  Here the sort key is the
// owning (channel, tile) of every tile a segment's window touches, and the sort is
// a counting sort (histogram -> exclusive scan -> scatter), O(v) instead of the
// O(v log v) comparison sort the paper used.
#include "internal.h"

namespace rts {
namespace {

// x = u*s + N/2 and xs = floor(x*OS + 1/2), each step rounded once, so that the
// result is bit-identical to a plain IEEE evaluation.  The compiler would fuse
// u*s + N/2 into one FMA (one rounding instead of two) and could then snap a
// sample that lies within an ulp of a phase boundary to the neighbouring phase;
// contraction is off in this function.
__device__ __forceinline__ bool snap(double u, double v, double s, int N, int OS, int &xs,
                                     int &ys) {
#pragma clang fp contract(off)
  const double half = (double)(N / 2);
  const double x = u * s + half;
  const double y = v * s + half;
  const double xo = floor(x * (double)OS + 0.5);
  const double yo = floor(y * (double)OS + 0.5);
  if (!(fabs(xo) < 1073741824.0) || !(fabs(yo) < 1073741824.0)) {  // false for NaN too
    xs = ys = 0;
    return false;
  }
  xs = (int)xo;
  ys = (int)yo;
  return true;
}

// Split an oversampled coordinate into cell and phase r in [r0, r0 + OS)
// (floor division; an arithmetic shift when OS is a power of two).
__device__ __forceinline__ void split(int xs, int r0, int OS, int log2os, int &cell, int &r) {
  const int q = xs - r0;
  if (log2os >= 0)
    cell = q >> log2os;
  else
    cell = (q >= 0) ? q / OS : -((-q + OS - 1) / OS);
  r = xs - cell * OS;
}

struct Sample {
  int cx, cy, rx, ry;
  bool valid;
  bool flagged;
};

__device__ __forceinline__ Sample sample(const PlanArgs &a, double u, double v, double s,
                                         float w) {
  Sample o;
  int xs, ys;
  const bool fin = snap(u, v, s, a.N, a.OS, xs, ys);
  split(xs, a.r0, a.OS, a.log2os, o.cx, o.rx);
  split(ys, a.r0, a.OS, a.log2os, o.cy, o.ry);
  const bool on = fin && o.cx - a.h_lo >= 0 && o.cx - a.h_lo + a.W - 1 <= a.N - 1 &&
                  o.cy - a.h_lo >= 0 && o.cy - a.h_lo + a.W - 1 <= a.N - 1;
  o.flagged = (w == 0.0f);
  o.valid = on && !o.flagged;
  return o;
}

struct Seg {
  int t0, nt;
  bool any;
  int X0, Y0;
  int fx, fy;   // 1: no sample's taps reach the window's last column (row)
};

// 1 when no valid sample of a segment reaches the last column (row) of its
// (W+1)-cell window: its samples sit in one cell column (row) and the window was
// not shifted at the grid edge, so that column holds zero weights.  A window that
// crosses a tile edge with that column only is not listed in the next tile,
// where it would add nothing.
__device__ __forceinline__ int last_free(const PlanArgs &a, bool any, int X0, int mx) {
  return (any && mx - a.h_lo + a.W - 1 < X0 + a.WN - 1) ? 1 : 0;
}

// Walk one baseline track of channel c and emit its segments in time order.  A
// segment is a run of at most seg_max consecutive samples whose valid samples'
// cells span at most 2x2 cells, so a (W+1)x(W+1) window holds all their taps.
// Segments partition the track: invalid samples ride along (or form a segment
// with any == false), so every sample belongs to exactly one segment.
template <class F>
__device__ __forceinline__ void walk_track(const PlanArgs &a, int c, int b, int copy, F &&emit) {
  const double s = a.scale[c];
  const double sg = copy ? -1.0 : 1.0;
  const double *uv = a.uvw + (size_t)b * a.T * 3;
  const float *w = a.w + ((size_t)c * a.B + b) * a.T;
  int t0 = 0;
  bool any = false;
  int mnx = 0, mxx = 0, mny = 0, mxy = 0;
  auto close = [&](int t1) {
    Seg sgm;
    sgm.t0 = t0;
    sgm.nt = t1 - t0;
    sgm.any = any;
    sgm.X0 = any ? min(mnx - a.h_lo, a.N - a.WN) : 0;
    sgm.Y0 = any ? min(mny - a.h_lo, a.N - a.WN) : 0;
    sgm.fx = last_free(a, any, sgm.X0, mxx);
    sgm.fy = last_free(a, any, sgm.Y0, mxy);
    emit(sgm);
  };
  for (int t = 0; t < a.T; ++t) {
    const Sample sm = sample(a, sg * uv[t * 3], sg * uv[t * 3 + 1], s, w[t]);
    if (sm.valid) {
      if (any) {
        const int nx0 = min(mnx, sm.cx), nx1 = max(mxx, sm.cx);
        const int ny0 = min(mny, sm.cy), ny1 = max(mxy, sm.cy);
        if (nx1 - nx0 > 1 || ny1 - ny0 > 1 || t - t0 >= a.seg_max) {
          close(t);
          t0 = t;
          mnx = mxx = sm.cx;
          mny = mxy = sm.cy;
        } else {
          mnx = nx0; mxx = nx1; mny = ny0; mxy = ny1;
        }
      } else {
        if (t - t0 >= a.seg_max) {
          close(t);
          t0 = t;
        }
        any = true;
        mnx = mxx = sm.cx;
        mny = mxy = sm.cy;
      }
    } else if (t - t0 >= a.seg_max) {
      close(t);
      t0 = t;
      any = false;
    }
  }
  close(a.T);
}

// Listings of a segment: every tile its window overlaps (at most 2 per axis since
// tile >= W+1).  A segment without valid samples of the +uv copy is listed once,
// in tile (0,0), so that its home listing writes its zero model.
template <class G>
__device__ __forceinline__ void for_listings(const PlanArgs &a, int c, int copy, const Seg &sg,
                                             G &&fn) {
  if (!sg.any) {
    if (copy == 0) fn((int64_t)c * a.nT2, 0, 0, true);
    return;
  }
  int tx0, tx1, ty0, ty1;
  if (a.log2tile >= 0) {
    tx0 = sg.X0 >> a.log2tile; tx1 = (sg.X0 + a.WN - 1 - sg.fx) >> a.log2tile;
    ty0 = sg.Y0 >> a.log2tile; ty1 = (sg.Y0 + a.WN - 1 - sg.fy) >> a.log2tile;
  } else {
    tx0 = sg.X0 / a.tile; tx1 = (sg.X0 + a.WN - 1 - sg.fx) / a.tile;
    ty0 = sg.Y0 / a.tile; ty1 = (sg.Y0 + a.WN - 1 - sg.fy) / a.tile;
  }
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx)
      fn((int64_t)c * a.nT2 + ty * a.nT + tx, tx, ty, tx == tx0 && ty == ty0);
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v) {
  __shared__ unsigned long long red[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  unsigned long long t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) t += red[i];
  return t;
}

__device__ __forceinline__ uint2 make_rec(const PlanArgs &a, int c, int b, int copy,
                                          const Seg &sg, bool home) {
  uint2 r;
  r.x = (uint32_t)((((size_t)c * a.B + b) * a.T) + sg.t0);
  r.y = (uint32_t)sg.X0 | ((uint32_t)sg.Y0 << kRecYShift) | ((uint32_t)(sg.nt - 1) << kRecNtShift) |
        ((uint32_t)home << kRecHomeBit) | ((uint32_t)copy << kRecCopyBit) |
        ((uint32_t)sg.any << kRecAnyBit);
  return r;
}

// Pass 1: packed per-sample coordinates, sample statistics and listing counts.
__global__ __launch_bounds__(kBlock) void k_plan_count(PlanArgs a) {
  extern __shared__ uint32_t hist[];
  const int c0 = blockIdx.y * a.cg;
  const int c1 = min(a.C, c0 + a.cg);
  const int nloc = (c1 - c0) * a.nT2;
  if (a.use_lds) {
    for (int i = threadIdx.x; i < nloc; i += blockDim.x) hist[i] = 0;
    __syncthreads();
  }
  unsigned long long nvalid = 0, nflag = 0, noff = 0, nseg = 0, nlist = 0;
  const int b2 = blockIdx.x * blockDim.x + threadIdx.x;
  if (b2 < a.B * a.ncopy) {
    const int copy = b2 / a.B, b = b2 - copy * a.B;
    const double sg = copy ? -1.0 : 1.0;
    const double *uv = a.uvw + (size_t)b * a.T * 3;
    for (int c = c0; c < c1; ++c) {
      const double s = a.scale[c];
      const float *w = a.w + ((size_t)c * a.B + b) * a.T;
      uint16_t *co = a.coords + (((size_t)c * a.ncopy + copy) * a.B + b) * a.T;
      walk_track(a, c, b, copy, [&](const Seg &sgm) {
        ++nseg;
        for (int t = sgm.t0; t < sgm.t0 + sgm.nt; ++t) {
          const Sample sm = sample(a, sg * uv[t * 3], sg * uv[t * 3 + 1], s, w[t]);
          uint16_t code = 0;
          if (sm.valid) {
            const int dx = sm.cx - (sgm.X0 + a.h_lo), dy = sm.cy - (sgm.Y0 + a.h_lo);
            const int sx = dx * a.OS + (sm.rx - a.r0), sy = dy * a.OS + (sm.ry - a.r0);
            code = (uint16_t)(kCoordValid | (sy << 7) | sx);
          }
          co[t] = code;
          if (copy == 0) {
            nvalid += sm.valid;
            nflag += sm.flagged;
            noff += !sm.valid && !sm.flagged;
          }
        }
        for_listings(a, c, copy, sgm, [&](int64_t key, int, int, bool) {
          ++nlist;
          if (a.use_lds)
            atomicAdd(&hist[key - (int64_t)c0 * a.nT2], 1u);
          else
            atomicAdd(&a.counts[key], 1u);
        });
      });
    }
  }
  if (a.use_lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < nloc; i += blockDim.x)
      if (hist[i]) atomicAdd(&a.counts[(int64_t)c0 * a.nT2 + i], hist[i]);
  }
  const unsigned long long v0 = block_sum_u64(nvalid);
  const unsigned long long v1 = block_sum_u64(nflag);
  const unsigned long long v2 = block_sum_u64(noff);
  const unsigned long long v3 = block_sum_u64(nseg);
  const unsigned long long v4 = block_sum_u64(nlist);
  if (threadIdx.x == 0) {
    if (v0) atomicAdd(&a.stats[0], v0);
    if (v1) atomicAdd(&a.stats[1], v1);
    if (v2) atomicAdd(&a.stats[2], v2);
    if (v3) atomicAdd(&a.stats[3], v3);
    if (v4) atomicAdd(&a.stats[4], v4);
  }
}


// Pass 2: every listing claims its slot.  With the LDS histogram, a workgroup
// reserves one contiguous range per key with a single global atomic and hands
// out slots from LDS.
__global__ __launch_bounds__(kBlock) void k_plan_scatter(PlanArgs a) {
  extern __shared__ uint32_t base[];
  const int c0 = blockIdx.y * a.cg;
  const int c1 = min(a.C, c0 + a.cg);
  const int nloc = (c1 - c0) * a.nT2;
  const int b2 = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = b2 < a.B * a.ncopy;
  const int copy = active ? b2 / a.B : 0, b = active ? b2 - copy * a.B : 0;
  if (a.use_lds) {
    for (int i = threadIdx.x; i < nloc; i += blockDim.x) base[i] = 0;
    __syncthreads();
    if (active)
      for (int c = c0; c < c1; ++c)
        walk_track(a, c, b, copy, [&](const Seg &sgm) {
          for_listings(a, c, copy, sgm, [&](int64_t key, int, int, bool) {
            atomicAdd(&base[key - (int64_t)c0 * a.nT2], 1u);
          });
        });
    __syncthreads();
    for (int i = threadIdx.x; i < nloc; i += blockDim.x)
      if (base[i]) base[i] = atomicAdd(&a.counts[(int64_t)c0 * a.nT2 + i], base[i]);
    __syncthreads();
  }
  if (!active) return;
  for (int c = c0; c < c1; ++c)
    walk_track(a, c, b, copy, [&](const Seg &sgm) {
      for_listings(a, c, copy, sgm, [&](int64_t key, int, int, bool home) {
        const uint32_t pos = a.use_lds ? atomicAdd(&base[key - (int64_t)c0 * a.nT2], 1u)
                                       : atomicAdd(&a.counts[key], 1u);
        if ((int64_t)pos < a.list_cap)
          a.list[pos] = make_rec(a, c, b, copy, sgm, home);
        else
          atomicAdd(&a.stats[5], 1ull);
      });
    });
}

// ------------------------------------------------- lane-per-sample plan (T <= 64)
// The samples of one track sit in adjacent lanes (a group of `tgroup` lanes, the
// power of two >= T), so uvw and weight loads are coalesced and every sample's
// FP64 coordinates are computed once per pass.  Every lane of a group then runs
// the same greedy segmentation over the group's samples (read with lane
// shuffles), so each lane learns the segment it belongs to without a leader; the
// first lane of each segment emits its listings with global atomics.
struct LaneSeg {
  int t0, nt, X0, Y0, fx, fy;
  bool any;
  bool single;   // the whole track is this one segment
};

__device__ __forceinline__ LaneSeg lane_segment(const PlanArgs &a, const Sample &sm, int t, int G) {
  LaneSeg mine{0, 0, 0, 0, 0, 0, false, false};
  int t0 = 0;
  bool any = false;
  int mnx = 0, mxx = 0, mny = 0, mxy = 0;
  auto close = [&](int t1) {
    if (t >= t0 && t < t1) {
      mine.t0 = t0;
      mine.nt = t1 - t0;
      mine.any = any;
      mine.X0 = any ? min(mnx - a.h_lo, a.N - a.WN) : 0;
      mine.Y0 = any ? min(mny - a.h_lo, a.N - a.WN) : 0;
      mine.fx = last_free(a, any, mine.X0, mxx);
      mine.fy = last_free(a, any, mine.Y0, mxy);
    }
  };
  for (int tt = 0; tt < a.T; ++tt) {
    const int vv = __shfl((int)sm.valid, tt, G);
    const int cx = __shfl(sm.cx, tt, G);
    const int cy = __shfl(sm.cy, tt, G);
    if (vv) {
      if (any) {
        const int nx0 = min(mnx, cx), nx1 = max(mxx, cx);
        const int ny0 = min(mny, cy), ny1 = max(mxy, cy);
        if (nx1 - nx0 > 1 || ny1 - ny0 > 1 || tt - t0 >= a.seg_max) {
          close(tt);
          t0 = tt;
          mnx = mxx = cx;
          mny = mxy = cy;
        } else {
          mnx = nx0; mxx = nx1; mny = ny0; mxy = ny1;
        }
      } else {
        if (tt - t0 >= a.seg_max) {
          close(tt);
          t0 = tt;
        }
        any = true;
        mnx = mxx = cx;
        mny = mxy = cy;
      }
    } else if (tt - t0 >= a.seg_max) {
      close(tt);
      t0 = tt;
      any = false;
    }
  }
  close(a.T);
  return mine;
}

// Min / max over an aligned group of G lanes (G a power of two <= 64), result in
// every lane of the group.  DPP quad permutations and row mirrors for G <= 16.
__device__ __forceinline__ int dpp_ctrl_xor(int v, int level) {
  switch (level) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // quad [1,0,3,2]
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);   // quad [2,3,0,1]
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    default: return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true); // row_mirror
  }
}

template <bool MAX>
__device__ __forceinline__ int group_reduce(int v, int G) {
  int lvl = 0;
  for (int w = 2; w <= G && w <= 16; w <<= 1, ++lvl) {
    const int o = dpp_ctrl_xor(v, lvl);
    v = MAX ? max(v, o) : min(v, o);
  }
  for (int w = 32; w <= G; w <<= 1) {
    const int o = __shfl_xor(v, w >> 1, 64);
    v = MAX ? max(v, o) : min(v, o);
  }
  return v;
}

// Segment of lane t: when the whole track fits one segment (at most seg_max
// samples and its valid samples span at most 2x2 cells), which the greedy walk
// would also produce, it is found with four group reductions; otherwise the walk
// runs.  All lanes of the wave must call this (it uses cross-lane operations).
__device__ __forceinline__ LaneSeg track_segment(const PlanArgs &a, const Sample &sm, int t, int G) {
  const int big = 1 << 30;
  const int mnx = group_reduce<false>(sm.valid ? sm.cx : big, G);
  const int mxx = group_reduce<true>(sm.valid ? sm.cx : -big, G);
  const int mny = group_reduce<false>(sm.valid ? sm.cy : big, G);
  const int mxy = group_reduce<true>(sm.valid ? sm.cy : -big, G);
  const bool any = mxx >= mnx;
  if (a.T <= a.seg_max && (!any || (mxx - mnx <= 1 && mxy - mny <= 1))) {
    LaneSeg sg;
    sg.t0 = 0;
    sg.nt = a.T;
    sg.any = any;
    sg.X0 = any ? min(mnx - a.h_lo, a.N - a.WN) : 0;
    sg.Y0 = any ? min(mny - a.h_lo, a.N - a.WN) : 0;
    sg.fx = last_free(a, any, sg.X0, mxx);
    sg.fy = last_free(a, any, sg.Y0, mxy);
    sg.single = true;
    return sg;
  }
  return lane_segment(a, sm, t, G);
}

template <bool SCATTER>
__global__ __launch_bounds__(kBlock) void k_plan_lanes(PlanArgs a) {
  const int G = a.tgroup;
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int t = (int)(gid & (G - 1));
  const int64_t tr = gid / G;                         // track over ncopy * B
  const bool active = tr < (int64_t)a.ncopy * a.B && t < a.T;
  const int copy = active ? (int)(tr / a.B) : 0;
  const int b = active ? (int)(tr - (int64_t)copy * a.B) : 0;
  double u = 0.0, v = 0.0;
  if (active) {
    const double sg = copy ? -1.0 : 1.0;
    const double *p = a.uvw + ((size_t)b * a.T + t) * 3;
    u = sg * p[0];
    v = sg * p[1];
  }
  unsigned long long nvalid = 0, nflag = 0, noff = 0, nseg = 0, nlist = 0;
  const int c0 = blockIdx.y * a.cg;
  const int c1 = min(a.C, c0 + a.cg);
  for (int c = c0; c < c1; ++c) {
    const size_t si = ((size_t)c * a.B + b) * a.T + t;
    Sample sm;
    if (active) {
      sm = sample(a, u, v, a.scale[c], a.w[si]);
    } else {
      sm.cx = sm.cy = sm.rx = sm.ry = 0;
      sm.valid = sm.flagged = false;
    }
    const LaneSeg sg = track_segment(a, sm, t, G);
    if (!active) continue;
    if (!SCATTER) {
      uint16_t code = 0;
      if (sm.valid) {
        const int dx = sm.cx - (sg.X0 + a.h_lo), dy = sm.cy - (sg.Y0 + a.h_lo);
        const int sx = dx * a.OS + (sm.rx - a.r0), sy = dy * a.OS + (sm.ry - a.r0);
        code = (uint16_t)(kCoordValid | (sy << 7) | sx);
      }
      a.coords[(((size_t)c * a.ncopy + copy) * a.B + b) * a.T + t] = code;
      if (copy == 0) {
        nvalid += sm.valid;
        nflag += sm.flagged;
        noff += !sm.valid && !sm.flagged;
      }
    }
    if (t != sg.t0) continue;
    Seg seg;
    seg.t0 = sg.t0; seg.nt = sg.nt; seg.any = sg.any; seg.X0 = sg.X0; seg.Y0 = sg.Y0;
    seg.fx = sg.fx; seg.fy = sg.fy;
    if (!SCATTER) ++nseg;
    for_listings(a, c, copy, seg, [&](int64_t key, int, int, bool home) {
      if (!SCATTER) {
        ++nlist;
        atomicAdd(&a.counts[key], 1u);
      } else {
        const uint32_t pos = atomicAdd(&a.counts[key], 1u);
        if ((int64_t)pos < a.list_cap)
          a.list[pos] = make_rec(a, c, b, copy, seg, home);
        else
          atomicAdd(&a.stats[5], 1ull);
      }
    });
  }
  if (!SCATTER) {
    const unsigned long long v0 = block_sum_u64(nvalid);
    const unsigned long long v1 = block_sum_u64(nflag);
    const unsigned long long v2 = block_sum_u64(noff);
    const unsigned long long v3 = block_sum_u64(nseg);
    const unsigned long long v4 = block_sum_u64(nlist);
    if (threadIdx.x == 0) {
      if (v0) atomicAdd(&a.stats[0], v0);
      if (v1) atomicAdd(&a.stats[1], v1);
      if (v2) atomicAdd(&a.stats[2], v2);
      if (v3) atomicAdd(&a.stats[3], v3);
      if (v4) atomicAdd(&a.stats[4], v4);
    }
  }
}

// ------------------------------------------- chunked counting sort (T <= 64)
// Workgroup (bx, by) owns a contiguous chunk of tracks and a group of cg
// channels.  Pass 1 counts its listings per (channel, tile) key in an LDS
// histogram and writes the whole histogram to hist[key][bx] (key-major, no
// atomics).  One exclusive scan over hist in (key, bx) order gives every
// workgroup the first slot of each key in the sorted list; pass 2 recomputes the
// same listings and claims slots from LDS copies of those offsets.
template <bool SCATTER>
__global__ __launch_bounds__(kBlock) void k_plan_chunk(PlanArgs a) {
  extern __shared__ uint32_t bins[];                 // [cg][nT2]
  const int G = a.tgroup;
  const int c0 = blockIdx.y * a.cg;
  const int c1 = min(a.C, c0 + a.cg);
  const int nloc = (c1 - c0) * a.nT2;
  const int bx = blockIdx.x;
  if (!SCATTER) {
    for (int i = threadIdx.x; i < nloc; i += kBlock) bins[i] = 0u;
  } else {
    for (int i = threadIdx.x; i < nloc; i += kBlock)
      bins[i] = a.offs[(size_t)bx * a.nkeys + (size_t)c0 * a.nT2 + i] + a.tile_off[(size_t)c0 * a.nT2 + i];
  }
  __syncthreads();
  const int64_t ntr = (int64_t)a.ncopy * a.B;
  const int64_t tr_beg = (int64_t)bx * a.chunk;
  const int64_t tr_end = min(ntr, tr_beg + a.chunk);
  const int per_iter = kBlock / G;
  const int t = threadIdx.x & (G - 1);
  unsigned long long nvalid = 0, nflag = 0, noff = 0, nseg = 0, nlist = 0;
  for (int64_t base = tr_beg; base < tr_end; base += per_iter) {
    const int64_t tr = base + threadIdx.x / G;
    const bool active = tr < tr_end && t < a.T;
    const int copy = active ? (int)(tr / a.B) : 0;
    const int b = active ? (int)(tr - (int64_t)copy * a.B) : 0;
    double u = 0.0, v = 0.0;
    if (active) {
      const double sg = copy ? -1.0 : 1.0;
      const double *p = a.uvw + ((size_t)b * a.T + t) * 3;
      u = sg * p[0];
      v = sg * p[1];
    }
#pragma unroll 1
    for (int c = c0; c < c1; ++c) {
      const float wt = active ? a.w[((size_t)c * a.B + b) * a.T + t] : 0.0f;
      Sample sm;
      if (active) {
        sm = sample(a, u, v, a.scale[c], wt);
      } else {
        sm.cx = sm.cy = sm.rx = sm.ry = 0;
        sm.valid = sm.flagged = false;
      }
      const LaneSeg sg = track_segment(a, sm, t, G);
      if (!active) continue;
      if (!SCATTER) {
        uint16_t code = 0;
        if (sm.valid) {
          const int dx = sm.cx - (sg.X0 + a.h_lo), dy = sm.cy - (sg.Y0 + a.h_lo);
          const int sx = dx * a.OS + (sm.rx - a.r0), sy = dy * a.OS + (sm.ry - a.r0);
          code = (uint16_t)(kCoordValid | (sy << 7) | sx);
        }
        a.coords[(((size_t)c * a.ncopy + copy) * a.B + b) * a.T + t] = code;
        if (copy == 0) {
          nvalid += sm.valid;
          nflag += sm.flagged;
          noff += !sm.valid && !sm.flagged;
        }
      }
      if (!SCATTER && t == 0)
        a.desc[((size_t)c * a.ncopy + copy) * a.B + b] =
            sg.single ? ((uint32_t)sg.any << kDescAnyBit) | ((uint32_t)sg.fx << kDescFxBit) |
                            ((uint32_t)sg.fy << kDescFyBit) | ((uint32_t)sg.Y0 << kRecYShift) | (uint32_t)sg.X0
                      : kDescMulti;
      if (t != sg.t0) continue;
      Seg seg;
      seg.t0 = sg.t0; seg.nt = sg.nt; seg.any = sg.any; seg.X0 = sg.X0; seg.Y0 = sg.Y0;
      seg.fx = sg.fx; seg.fy = sg.fy;
      if (!SCATTER) ++nseg;
      for_listings(a, c, copy, seg, [&](int64_t key, int, int, bool home) {
        const int bin = (int)(key - (int64_t)c0 * a.nT2);
        if (!SCATTER) {
          ++nlist;
          atomicAdd(&bins[bin], 1u);
        } else {
          const uint32_t pos = atomicAdd(&bins[bin], 1u);
          if ((int64_t)pos < a.list_cap)
            a.list[pos] = make_rec(a, c, b, copy, seg, home);
          else
            atomicAdd(&a.stats[5], 1ull);
        }
      });
    }
  }
  if (!SCATTER) {
    __syncthreads();
    for (int i = threadIdx.x; i < nloc; i += kBlock)
      a.hist[(size_t)bx * a.nkeys + (size_t)c0 * a.nT2 + i] = bins[i];
    const unsigned long long v0 = block_sum_u64(nvalid);
    const unsigned long long v1 = block_sum_u64(nflag);
    const unsigned long long v2 = block_sum_u64(noff);
    const unsigned long long v3 = block_sum_u64(nseg);
    const unsigned long long v4 = block_sum_u64(nlist);
    if (threadIdx.x == 0) {
      if (v0) atomicAdd(&a.stats[0], v0);
      if (v1) atomicAdd(&a.stats[1], v1);
      if (v2) atomicAdd(&a.stats[2], v2);
      if (v3) atomicAdd(&a.stats[3], v3);
      if (v4) atomicAdd(&a.stats[4], v4);
    }
  }
}

// Pass 1 of the chunked sort for tracks of at most kTrackRegs samples: one thread
// per track keeps the track's coordinates in registers (no cross-lane work), so
// each sample's FP64 coordinates are computed once and the listing bookkeeping
// is done once per track.  Tracks that split into several segments (rare) are
// walked again from memory with the same greedy rule.  The kernel is built for
// tracks of up to 4 and up to 8 samples (TR), so short tracks hold half the
// registers.
constexpr int kTrackRegs = 8;

typedef double rts_d2_a8 __attribute__((ext_vector_type(2), aligned(8)));

// The T (<= kTrackRegs) weights of track b in channel c (vector loads when T is 4
// or 8 and the weights are 16-byte aligned; a track then starts 16-byte aligned).
template <int TR>
__device__ __forceinline__ void load_track_weights(const PlanArgs &a, int c, int b, float (&w)[TR]) {
  const float *p = a.w + ((size_t)c * a.B + b) * a.T;
  float4 x = make_float4(0.0f, 0.0f, 0.0f, 0.0f), y = x;
  if (a.vec_t) {
    x = reinterpret_cast<const float4 *>(p)[0];
    if (TR == 8 && a.T == 8) y = reinterpret_cast<const float4 *>(p)[1];
  } else {
    if (a.T > 0) x.x = p[0];
    if (a.T > 1) x.y = p[1];
    if (a.T > 2) x.z = p[2];
    if (a.T > 3) x.w = p[3];
    if (TR == 8 && a.T > 4) y.x = p[4];
    if (TR == 8 && a.T > 5) y.y = p[5];
    if (TR == 8 && a.T > 6) y.z = p[6];
    if (TR == 8 && a.T > 7) y.w = p[7];
  }
  w[0] = x.x; w[1 % TR] = x.y; w[2 % TR] = x.z; w[3 % TR] = x.w;
  if (TR == 8) {
    w[4 % TR] = y.x; w[5 % TR] = y.y; w[6 % TR] = y.z; w[7 % TR] = y.w;
  }
}

template <int TR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_plan_track_count(PlanArgs a) {
  extern __shared__ uint32_t bins[];                 // [cg][nT2]
  const int c0 = blockIdx.y * a.cg;
  const int c1 = min(a.C, c0 + a.cg);
  const int nloc = (c1 - c0) * a.nT2;
  const int bx = blockIdx.x;
  for (int i = threadIdx.x; i < nloc; i += kBlock) bins[i] = 0u;
  __syncthreads();
  const int64_t ntr = (int64_t)a.ncopy * a.B;
  const int64_t tr_end = min(ntr, (int64_t)bx * a.chunk + a.chunk);
  // per-thread sample counts stay below the plan's 2^31 samples: 32-bit adds
  uint32_t nvalid = 0, nflag = 0, noff = 0;
  unsigned long long nseg = 0, nlist = 0;
  for (int64_t tr = (int64_t)bx * a.chunk + threadIdx.x; tr < tr_end; tr += kBlock) {
    const int copy = (int)(tr / a.B);
    const int b = (int)(tr - (int64_t)copy * a.B);
    const double sgn = copy ? -1.0 : 1.0;
    double u[TR], v[TR];
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      u[t] = v[t] = 0.0;
      if (t < a.T) {
        // (u, v) of one sample in one 16-byte load (8-byte aligned address)
        const rts_d2_a8 uv = *reinterpret_cast<const rts_d2_a8 *>(a.uvw + ((size_t)b * a.T + t) * 3);
        u[t] = sgn * uv.x;
        v[t] = sgn * uv.y;
      }
    }
    // The weights of the next channel are loaded while this one is processed.
    float wn[TR];
    load_track_weights(a, c0, b, wn);
#pragma unroll 1
    for (int c = c0; c < c1; ++c) {
      float wv[TR];
#pragma unroll
      for (int t = 0; t < TR; ++t) wv[t] = wn[t];
      if (c + 1 < c1) load_track_weights(a, c + 1, b, wn);
      const double sc = a.scale[c];
      Sample sm[TR];
      int mnx = 1 << 30, mxx = -(1 << 30), mny = 1 << 30, mxy = -(1 << 30);
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        sm[t].valid = sm[t].flagged = false;
        sm[t].cx = sm[t].cy = sm[t].rx = sm[t].ry = 0;
        if (t < a.T) {
          sm[t] = sample(a, u[t], v[t], sc, wv[t]);
          if (copy == 0) {
            nvalid += sm[t].valid;
            nflag += sm[t].flagged;
            noff += !sm[t].valid && !sm[t].flagged;
          }
          if (sm[t].valid) {
            mnx = min(mnx, sm[t].cx); mxx = max(mxx, sm[t].cx);
            mny = min(mny, sm[t].cy); mxy = max(mxy, sm[t].cy);
          }
        }
      }
      const bool any = mxx >= mnx;
      uint16_t *co = a.coords + (((size_t)c * a.ncopy + copy) * a.B + b) * a.T;
      const size_t di = ((size_t)c * a.ncopy + copy) * a.B + b;
      auto count = [&](const Seg &seg) {
        ++nseg;
        for_listings(a, c, copy, seg, [&](int64_t key, int, int, bool) {
          ++nlist;
          atomicAdd(&bins[(int)(key - (int64_t)c0 * a.nT2)], 1u);
        });
      };
      if (a.T <= a.seg_max && (!any || (mxx - mnx <= 1 && mxy - mny <= 1))) {
        Seg seg;
        seg.t0 = 0;
        seg.nt = a.T;
        seg.any = any;
        seg.X0 = any ? min(mnx - a.h_lo, a.N - a.WN) : 0;
        seg.Y0 = any ? min(mny - a.h_lo, a.N - a.WN) : 0;
        seg.fx = last_free(a, any, seg.X0, mxx);
        seg.fy = last_free(a, any, seg.Y0, mxy);
        uint32_t code[TR];
#pragma unroll
        for (int t = 0; t < TR; ++t) {
          code[t] = 0u;
          if (t < a.T && sm[t].valid) {
            const int sx = (sm[t].cx - (seg.X0 + a.h_lo)) * a.OS + (sm[t].rx - a.r0);
            const int sy = (sm[t].cy - (seg.Y0 + a.h_lo)) * a.OS + (sm[t].ry - a.r0);
            code[t] = kCoordValid | (uint32_t)(sy << 7) | (uint32_t)sx;
          }
        }
        if (TR == 8 && a.vec_t && a.T == 8) {
          *reinterpret_cast<uint4 *>(co) = make_uint4(code[0] | code[1 % TR] << 16,
                                                      code[2 % TR] | code[3 % TR] << 16,
                                                      code[4 % TR] | code[5 % TR] << 16,
                                                      code[6 % TR] | code[7 % TR] << 16);
        } else if (a.vec_t && a.T == 4) {
          *reinterpret_cast<uint2 *>(co) = make_uint2(code[0] | code[1 % TR] << 16,
                                                      code[2 % TR] | code[3 % TR] << 16);
        } else {
#pragma unroll
          for (int t = 0; t < TR; ++t)
            if (t < a.T) co[t] = (uint16_t)code[t];
        }
        a.desc[di] = ((uint32_t)any << kDescAnyBit) | ((uint32_t)seg.fx << kDescFxBit) |
                     ((uint32_t)seg.fy << kDescFyBit) | ((uint32_t)seg.Y0 << kRecYShift) | (uint32_t)seg.X0;
        count(seg);
      } else {
        a.desc[di] = kDescMulti;
        const double sg2 = sgn;
        const double *uv = a.uvw + (size_t)b * a.T * 3;
        const float *wrow = a.w + ((size_t)c * a.B + b) * a.T;
        walk_track(a, c, b, copy, [&](const Seg &seg) {
          for (int t = seg.t0; t < seg.t0 + seg.nt; ++t) {
            const Sample s2 = sample(a, sg2 * uv[t * 3], sg2 * uv[t * 3 + 1], sc, wrow[t]);
            uint16_t code = 0;
            if (s2.valid) {
              const int sx = (s2.cx - (seg.X0 + a.h_lo)) * a.OS + (s2.rx - a.r0);
              const int sy = (s2.cy - (seg.Y0 + a.h_lo)) * a.OS + (s2.ry - a.r0);
              code = (uint16_t)(kCoordValid | (sy << 7) | sx);
            }
            co[t] = code;
          }
          count(seg);
        });
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nloc; i += kBlock)
    a.hist[(size_t)bx * a.nkeys + (size_t)c0 * a.nT2 + i] = bins[i];
  const unsigned long long v0 = block_sum_u64(nvalid);
  const unsigned long long v1 = block_sum_u64(nflag);
  const unsigned long long v2 = block_sum_u64(noff);
  const unsigned long long v3 = block_sum_u64(nseg);
  const unsigned long long v4 = block_sum_u64(nlist);
  if (threadIdx.x == 0) {
    if (v0) atomicAdd(&a.stats[0], v0);
    if (v1) atomicAdd(&a.stats[1], v1);
    if (v2) atomicAdd(&a.stats[2], v2);
    if (v3) atomicAdd(&a.stats[3], v3);
    if (v4) atomicAdd(&a.stats[4], v4);
  }
}

// Pass 2 of the chunked sort, one thread per track: a single-segment track is
// emitted from the descriptor written by pass 1; a track that pass 1 split into
// several segments is walked again from uvw and the weights (same greedy rule).
__global__ __launch_bounds__(kBlock) void k_plan_scatter_tracks(PlanArgs a) {
  extern __shared__ uint32_t bins[];
  const int bx = blockIdx.x;
  const int c0 = blockIdx.y * a.cg;
  const int c1 = min(a.C, c0 + a.cg);
  const int nloc = (c1 - c0) * a.nT2;
  for (int i = threadIdx.x; i < nloc; i += kBlock)
    bins[i] = a.offs[(size_t)bx * a.nkeys + (size_t)c0 * a.nT2 + i] + a.tile_off[(size_t)c0 * a.nT2 + i];
  __syncthreads();
  const int64_t ntr = (int64_t)a.ncopy * a.B;
  const int64_t tr_end = min(ntr, (int64_t)bx * a.chunk + a.chunk);
  // Channels outermost: the records one workgroup writes for a key form one
  // contiguous run of the work list, and visiting one channel's keys at a time
  // writes each run within a short interval (whole cache lines in L2).
  // Each thread takes eight tracks per pass and loads their descriptors together,
  // so that the loads overlap instead of each track waiting for its own.
  constexpr int kUnroll = 8;
  for (int c = c0; c < c1; ++c) {
    const uint32_t *desc_c = a.desc + (size_t)c * a.ncopy * a.B;   // [ncopy][B]: index tr
    for (int64_t tr0 = (int64_t)bx * a.chunk + threadIdx.x; tr0 < tr_end; tr0 += kUnroll * kBlock) {
    uint32_t dd[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t tr = tr0 + (int64_t)u * kBlock;
      dd[u] = tr < tr_end ? desc_c[tr] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t tr = tr0 + (int64_t)u * kBlock;
      if (tr >= tr_end) break;
      const int copy = (int)(tr / a.B);
      const int b = (int)(tr - (int64_t)copy * a.B);
      auto emit = [&](const Seg &seg) {
        for_listings(a, c, copy, seg, [&](int64_t key, int, int, bool home) {
          const uint32_t pos = atomicAdd(&bins[(int)(key - (int64_t)c0 * a.nT2)], 1u);
          if ((int64_t)pos < a.list_cap)
            a.list[pos] = make_rec(a, c, b, copy, seg, home);
          else
            atomicAdd(&a.stats[5], 1ull);
        });
      };
      const uint32_t d = dd[u];
      if (d != kDescMulti) {
        Seg seg;
        seg.t0 = 0;
        seg.nt = a.T;
        seg.any = (d >> kDescAnyBit) & 1u;
        seg.X0 = (int)(d & kRecXMask);
        seg.Y0 = (int)((d >> kRecYShift) & kRecXMask);
        seg.fx = (int)((d >> kDescFxBit) & 1u);
        seg.fy = (int)((d >> kDescFyBit) & 1u);
        emit(seg);
      } else {
        walk_track(a, c, b, copy, emit);
      }
    }
    }
  }
}

// Longest-first tile order per XCD range (persistent launch): tiles are bucketed by
// their work-list length (clamped to kLptBins-1), longest bucket first, within the
// eighth of the tile range each XCD owns.
// Bucket of a tile with n listings, heaviest first: an increasing map of n with
// 16 buckets per octave (exponent and the next four bits of n + 1), reversed.
__device__ __forceinline__ int lpt_bin(uint32_t n) {
  const uint32_t m = n + 1u;
  const int e = 31 - __clz((int)m);
  const int f = e >= 4 ? (int)((m >> (e - 4)) & 15u) : (int)((m << (4 - e)) & 15u);
  return kLptBins - 1 - min(e * 16 + f, kLptBins - 1);
}

__global__ __launch_bounds__(kBlock) void k_lpt_count(const uint32_t *tile_off, int64_t nkeys, uint32_t *cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nkeys) return;
  const int64_t per = (nkeys + 7) / 8;
  const int bin = lpt_bin(tile_off[k + 1] - tile_off[k]);
  atomicAdd(&cnt[(k / per) * kLptBins + bin], 1u);
}

__global__ __launch_bounds__(kBlock) void k_lpt_scatter(const uint32_t *tile_off, int64_t nkeys, uint32_t *cursor,
                                                        uint32_t *order) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nkeys) return;
  const int64_t per = (nkeys + 7) / 8;
  const int bin = lpt_bin(tile_off[k + 1] - tile_off[k]);
  const uint32_t pos = atomicAdd(&cursor[(k / per) * kLptBins + bin], 1u);
  order[pos] = (uint32_t)k;
}

// Chunked sort, between the passes: in place, hist[bx][k] becomes the number of
// listings of key k in the chunks before bx, and totals[k] the count of key k.
// A workgroup owns 32 keys; each of its 8 groups of 32 lanes sums one eighth of
// the chunks (coalesced rows), then writes running offsets from its base.
__global__ __launch_bounds__(kBlock) void k_hist_colscan(uint32_t *hist, int nbx, int64_t nkeys,
                                                         uint32_t *totals) {
  __shared__ uint32_t part[kBlock / 32][32];
  const int lane = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const int64_t k = (int64_t)blockIdx.x * 32 + lane;
  const int per = (nbx + kBlock / 32 - 1) / (kBlock / 32);
  const int b0 = min(nbx, grp * per), b1 = min(nbx, b0 + per);
  uint32_t sum = 0;
  if (k < nkeys) {
#pragma unroll 4
    for (int bx = b0; bx < b1; ++bx) sum += hist[(size_t)bx * nkeys + k];
  }
  part[grp][lane] = sum;
  __syncthreads();
  uint32_t base = 0, total = 0;
  for (int g = 0; g < kBlock / 32; ++g) {
    const uint32_t p = part[g][lane];
    if (g < grp) base += p;
    total += p;
  }
  if (k < nkeys) {
    for (int bx = b0; bx < b1; ++bx) {
      const size_t i = (size_t)bx * nkeys + k;
      const uint32_t v = hist[i];
      hist[i] = base;
      base += v;
    }
    if (grp == 0) totals[k] = total;
  }
}

// ---------------------------------------------------------------- exclusive scan
constexpr int kScanPerThread = 16;
constexpr int kScanPerBlock = kBlock * kScanPerThread;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t &total) {
  __shared__ uint32_t ws[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t n = __shfl_up(x, o, 64);
    if (lane >= o) x += n;
  }
  __syncthreads();
  if (lane == 63) ws[wid] = x;
  __syncthreads();
  uint32_t pre = 0;
  total = 0;
  for (int i = 0; i < kBlock / 64; ++i) {
    if (i < wid) pre += ws[i];
    total += ws[i];
  }
  return pre + x - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_local(const uint32_t *in, uint32_t *out,
                                                       uint32_t *bsum, int64_t n) {
  // Each thread owns 16 consecutive counts, read and written as four 16-byte
  // vectors when the block is full (the tail block falls back to scalars).
  const int64_t base = (int64_t)blockIdx.x * kScanPerBlock + (int64_t)threadIdx.x * kScanPerThread;
  uint32_t v[kScanPerThread];
  const bool full = (int64_t)(blockIdx.x + 1) * kScanPerBlock <= n;
  if (full) {
    const uint4 *p = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
    for (int h = 0; h < kScanPerThread / 4; ++h) {
      const uint4 x = p[h];
      v[4 * h] = x.x; v[4 * h + 1] = x.y; v[4 * h + 2] = x.z; v[4 * h + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) v[i] = (base + i < n) ? in[base + i] : 0u;
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPerThread; ++i) s += v[i];
  uint32_t total;
  uint32_t pre = block_excl_scan(s, total);
#pragma unroll
  for (int i = 0; i < kScanPerThread; ++i) {
    const uint32_t x = v[i];
    v[i] = pre;
    pre += x;
  }
  if (full) {
    uint4 *q = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
    for (int h = 0; h < kScanPerThread / 4; ++h) q[h] = make_uint4(v[4 * h], v[4 * h + 1], v[4 * h + 2], v[4 * h + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i)
      if (base + i < n) out[base + i] = v[i];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the block sums in place; bsum[nb] = total.
__global__ __launch_bounds__(kBlock) void k_scan_bsum(uint32_t *bsum, int64_t nb) {
  uint32_t carry = 0;
  for (int64_t start = 0; start < nb; start += kBlock) {
    const int64_t i = start + threadIdx.x;
    const uint32_t v = (i < nb) ? bsum[i] : 0u;
    uint32_t total;
    const uint32_t pre = block_excl_scan(v, total);
    if (i < nb) bsum[i] = carry + pre;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t *tile_off, uint32_t *cursor,
                                                     const uint32_t *bsum, int64_t n, int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const uint32_t v = tile_off[i] + bsum[i / kScanPerBlock];
    tile_off[i] = v;
    if (cursor) cursor[i] = v;
  }
  if (i == 0) tile_off[n] = bsum[nb];
}

// ------------------------------------------------------------ coordinates (a1)
__global__ __launch_bounds__(kBlock) void k_coords(const double *uvw, const double *scale,
                                                   const float *w, int32_t *out, int N, int W,
                                                   int OS, int C, int B, int T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)C * B * T;
  if (i >= n) return;
  const int64_t bt = i % ((int64_t)B * T);
  const int c = (int)(i / ((int64_t)B * T));
  PlanArgs a{};
  a.N = N; a.W = W; a.OS = OS;
  a.r0 = (W & 1) ? -(OS / 2) : 0;
  a.h_lo = (W & 1) ? (W - 1) / 2 : W / 2 - 1;
  a.log2os = -1;
  int xs, ys;
  const bool fin = snap(uvw[bt * 3], uvw[bt * 3 + 1], scale[c], N, OS, xs, ys);
  const Sample sm = sample(a, uvw[bt * 3], uvw[bt * 3 + 1], scale[c], w[i]);
  out[i * 3] = fin ? xs : 0;
  out[i * 3 + 1] = fin ? ys : 0;
  out[i * 3 + 2] = sm.valid ? 1 : 0;
}

// mask[c][b][t] = 1 for valid samples of the +uv copy (from the packed coordinates).
__global__ __launch_bounds__(kBlock) void k_valid_mask(const uint16_t *coords, uint8_t *mask, int B, int T,
                                                       int ncopy, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t bt = (int64_t)B * T;
  const int64_t c = i / bt;
  mask[i] = (coords[i + c * (ncopy - 1) * bt] & kCoordValid) ? 1 : 0;
}

__global__ __launch_bounds__(1024) void k_chi2_reduce(const double *part, int64_t n, double *out) {
  __shared__ double red[16];
  // eight independent partial sums per thread keep eight loads in flight
  double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t step = (int64_t)blockDim.x * 8;
  int64_t i0 = threadIdx.x;
  for (; i0 + 7 * (int64_t)blockDim.x < n; i0 += step) {
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] += part[i0 + k * (int64_t)blockDim.x];
  }
  for (int64_t i = i0; i < n; i += blockDim.x) p[0] += part[i];
  double s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    *out = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_plan_count(const PlanArgs &a, hipStream_t s) {
  if (a.nbx > 0) {
    dim3 g3((unsigned)a.nbx, (a.C + a.cg - 1) / a.cg);
    const size_t lds = (size_t)a.cg * a.nT2 * sizeof(uint32_t);
    if (a.T <= 4)
      hipLaunchKernelGGL(k_plan_track_count<4>, g3, dim3(kBlock), lds, s, a);
    else if (a.T <= kTrackRegs)
      hipLaunchKernelGGL(k_plan_track_count<kTrackRegs>, g3, dim3(kBlock), lds, s, a);
    else
      hipLaunchKernelGGL(k_plan_chunk<false>, g3, dim3(kBlock), lds, s, a);
    return hipGetLastError();
  }
  if (a.tgroup > 0) {
    const int64_t lanes = (int64_t)a.ncopy * a.B * a.tgroup;
    dim3 g2((unsigned)((lanes + kBlock - 1) / kBlock), (a.C + a.cg - 1) / a.cg);
    hipLaunchKernelGGL(k_plan_lanes<false>, g2, dim3(kBlock), 0, s, a);
    return hipGetLastError();
  }
  dim3 grid((a.B * a.ncopy + kBlock - 1) / kBlock, (a.C + a.cg - 1) / a.cg);
  const size_t lds = a.use_lds ? (size_t)a.cg * a.nT2 * sizeof(uint32_t) : 0;
  hipLaunchKernelGGL(k_plan_count, grid, dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_plan_scatter(const PlanArgs &a, hipStream_t s) {
  if (a.nbx > 0) {
    dim3 g3((unsigned)a.nbx, (a.C + a.cg - 1) / a.cg);
    hipLaunchKernelGGL(k_plan_scatter_tracks, g3, dim3(kBlock), (size_t)a.cg * a.nT2 * sizeof(uint32_t), s, a);
    return hipGetLastError();
  }
  if (a.tgroup > 0) {
    const int64_t lanes = (int64_t)a.ncopy * a.B * a.tgroup;
    dim3 g2((unsigned)((lanes + kBlock - 1) / kBlock), (a.C + a.cg - 1) / a.cg);
    hipLaunchKernelGGL(k_plan_lanes<true>, g2, dim3(kBlock), 0, s, a);
    return hipGetLastError();
  }
  dim3 grid((a.B * a.ncopy + kBlock - 1) / kBlock, (a.C + a.cg - 1) / a.cg);
  const size_t lds = a.use_lds ? (size_t)a.cg * a.nT2 * sizeof(uint32_t) : 0;
  hipLaunchKernelGGL(k_plan_scatter, grid, dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *counts, uint32_t *tile_off, uint32_t *cursor,
                       uint32_t *tmp, int64_t n, hipStream_t s) {
  const int64_t nb = (n + kScanPerBlock - 1) / kScanPerBlock;
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kBlock), 0, s, counts, tile_off, tmp, n);
  hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(kBlock), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     tile_off, cursor, (const uint32_t *)tmp, n, nb);
  return hipGetLastError();
}

hipError_t launch_hist_scan(uint32_t *hist, int nbx, int64_t nkeys, uint32_t *totals, uint32_t *tile_off,
                            uint32_t *tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_hist_colscan, dim3((unsigned)((nkeys + 31) / 32)), dim3(kBlock), 0, s, hist, nbx, nkeys,
                     totals);
  return launch_scan(totals, tile_off, nullptr, tmp, nkeys, s);
}

hipError_t launch_lpt_order(const uint32_t *tile_off, int64_t nkeys, uint32_t *lpt, uint32_t *order,
                            hipStream_t s) {
  uint32_t *cnt = lpt, *off = lpt + kLptOff, *tmp = lpt + kLptTmp;
  hipError_t e = launch_fill_u32(cnt, 8 * kLptBins, 0u, s);
  if (e != hipSuccess) return e;
  const unsigned nb = (unsigned)((nkeys + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_lpt_count, dim3(nb), dim3(kBlock), 0, s, tile_off, nkeys, cnt);
  e = launch_scan(cnt, off, cnt, tmp, 8 * kLptBins, s);   // cnt becomes the cursors
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lpt_scatter, dim3(nb), dim3(kBlock), 0, s, tile_off, nkeys, cnt, order);
  return hipGetLastError();
}

hipError_t launch_coords(const double *uvw, const double *scale, const float *w, int32_t *out,
                         int N, int W, int OS, int C, int B, int T, hipStream_t s) {
  const int64_t n = (int64_t)C * B * T;
  hipLaunchKernelGGL(k_coords, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, uvw,
                     scale, w, out, N, W, OS, C, B, T);
  return hipGetLastError();
}

hipError_t launch_valid_mask(const uint16_t *coords, uint8_t *mask, int B, int T, int ncopy, int64_t n,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_valid_mask, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, coords, mask,
                     B, T, ncopy, n);
  return hipGetLastError();
}

hipError_t launch_chi2_reduce(const double *part, int64_t n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_chi2_reduce, dim3(1), dim3(1024), 0, s, part, n, out);
  return hipGetLastError();
}

}  // namespace rts
