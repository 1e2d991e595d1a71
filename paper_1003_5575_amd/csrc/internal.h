// Internal declarations shared by the host ABI and the HIP kernels of librtsgrid.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "rtsgrid.h"

namespace rts {

constexpr int kMaxW = 16;
constexpr int kMaxWMfma = 24;   // supports up to this on the matrix-core path (BF16x3 plans)
constexpr int kMaxOS = 64;
constexpr int kMaxN = 8192;
constexpr int kMaxTile = 64;     // FP64 tile accumulator: 16*64*66 B = 66 KiB of LDS
// The FP64 tile accumulator holds the real and the imaginary parts in two planes of
// tile rows of tile + kAccPad cells (66 KiB at tile 64).  With the pad, cell (x, y)
// of a plane lies in LDS bank pair (x + kAccPad*y) mod 32, so the adds of windows
// in neighbouring rows (a wave's windows are sorted by position) spread over the
// banks instead of sharing the banks of their columns.
constexpr int kAccPad = 2;
constexpr double kCLight = 299792458.0;
constexpr int kBlock = 256;          // threads per workgroup of every kernel here
constexpr int kMaxCg = 8;            // most channels one plan workgroup handles

enum Mode { kGrid = 0, kDegrid = 1, kFused = 2 };

// Work-list record (8 bytes) for one (segment, tile) pair.
//   x: index of the segment's first sample in the [C][B][T] visibility arrays
//   y: X0 | Y0 << 13 | (nt-1) << 26 | home << 29 | copy << 30 | any_valid << 31
// (X0, Y0) is the origin cell of the segment's (W+1)x(W+1) window, nt its sample
// count, home marks the listing in the tile that holds the window origin (the one
// that writes the model), copy marks the conjugate (-u,-v) copy.
constexpr uint32_t kRecXMask = 0x1FFFu;
constexpr int kRecYShift = 13;
constexpr int kRecNtShift = 26;
constexpr int kRecHomeBit = 29;
constexpr int kRecCopyBit = 30;
constexpr int kRecAnyBit = 31;

// Per-sample packed window coordinates (16 bits):
//   bit 15 valid | sy << 7 | sx, with s = d*OS + (r - r0) in [0, 2*OS): d in {0,1} is
//   the sample's cell offset from the window origin + h_lo, r its kernel phase.
constexpr uint16_t kCoordValid = 0x8000u;

// Per-track segment descriptor written by the first plan pass (chunked sort):
// X0 | Y0 << 13 | fx << 26 | fy << 27 | any << 30 for a track that is one segment
// (fx, fy: the window's last column / row holds no taps), kDescMulti otherwise.
constexpr int kDescFxBit = 26;
constexpr int kDescFyBit = 27;
constexpr int kDescAnyBit = 30;
constexpr uint32_t kDescMulti = 0x80000000u;

struct PlanArgs {
  const double *uvw;      // [B][T][3]
  const double *scale;    // [C]  f_c / (c du)
  const float *w;         // [C][B][T]
  uint16_t *coords;       // [C][ncopy][B][T]
  uint2 *list;            // [capacity]
  uint32_t *counts;       // [nkeys] counts (count pass) / cursors (scatter pass)
  unsigned long long *stats;  // [6]: valid, flagged, offgrid, segments, listings, dropped
  int64_t list_cap;       // capacity of list; listings beyond it are dropped and counted
  int N, W, OS, WN, r0, h_lo;
  int log2os;             // log2(OS) when OS is a power of two, else -1
  int tile, nT, nT2;
  int log2tile;           // log2(tile) when tile is a power of two, else -1
  int C, B, T, ncopy, seg_max;
  int cg, use_lds;
  int tgroup;             // lanes per track (power of two >= T) for the lane path, 0 = per-track path
  int nbx;                // chunked sort: track chunks (0 = not used)
  int64_t chunk;          // chunked sort: tracks per chunk
  uint32_t *hist;         // chunked sort: [nbx][nkeys] counts (chunk-major: coalesced rows)
  const uint32_t *offs;   // chunked sort: [nbx][nkeys] offsets of each chunk within its key
  const uint32_t *tile_off;  // chunked sort: [nkeys + 1] first slot of each key
  int64_t nkeys;          // C * nT2
  int vec_t;              // T is 4 or 8 and the weights are 16-byte aligned: vector loads
  uint32_t *desc;         // chunked sort: per-track segment descriptors [C][ncopy][B]
};

struct TileArgs {
  const uint2 *list;
  const uint32_t *tile_off;  // [nkeys+1]
  const uint16_t *coords;
  const float *tabE;         // [2*OS][WNP]
  const float2 *vis;
  const float *w;
  const float2 *gin;
  float2 *model;
  float2 *gout;
  double *chi2_part;         // [nkeys]
  int64_t list_cap;          // listings at or beyond this index are ignored
  int N, tile, nT, nT2, nkeys;
  int B, T, ncopy;
  int OS2, WNP, WN;
  int write_model;
  int vec;                   // whole-track segments may use 16-byte vector loads and stores
  int seg_max;               // most samples per segment (a power of two)
  const uint32_t *order;     // tiles in per-XCD longest-first order (persistent launch, matrix-core kernels)
  uint32_t *queue;           // persistent launch: 8 queue counters (zeroed before launch)
};

}  // namespace rts

namespace rts {
// Consecutive workgroups are dispatched round-robin over the 8 XCDs, each with its
// own L2.  Remap so that every XCD walks one contiguous range of tiles: a tile's
// neighbours (whose windows overlap it) then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n >> 3, r = n & 7, xcd = bid & 7, slot = bid >> 3;
  return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}
}  // namespace rts

// Plan state behind the opaque rts_plan_t handle.
struct rts_plan_s {
  rts_params p{};
  int N = 0, W = 0, OS = 0, WN = 0, WNP = 0, tile = 0, nT = 0, nT2 = 0;
  int C = 0, B = 0, T = 0, ncopy = 1, r0 = 0, h_lo = 0, seg_max = 0;
  double beta = 0.0;
  int64_t nkeys = 0;
  int device = 0;
  int n_cu = 256;                  // compute units of the plan's device
  void *fft = nullptr;             // imager: batched 2-D inverse FFT plan (created on first use)
  float *d_rcorr = nullptr;        // imager: 1 / khat((i - N/2) / N), i < N
  std::vector<float> tab;    // [OS][W]
  std::vector<float> tabE;   // [2*OS][WNP]
  std::vector<uint16_t> tab_hi, tab_lo;   // [2*OS][WNP] bf16 bits: hi = bf16(k), lo = bf16(k - hi)
  int precision = 0;
  float *d_tabE = nullptr;
  uint16_t *d_tab_hi = nullptr;
  uint16_t *d_tab_lo = nullptr;
  uint32_t *d_pb_thl = nullptr;   // per-baseline padded kernel rows (packed hi|lo), NULL = shared kernel
  float *d_pb_tab = nullptr;      // per-baseline padded kernel rows (FP32)
  double *d_scale = nullptr;
  uint16_t *d_coords = nullptr;
  uint2 *d_list = nullptr;
  uint32_t *d_tile_off = nullptr;
  uint32_t *d_cursor = nullptr;
  uint32_t *d_scan_tmp = nullptr;
  uint32_t *d_hist = nullptr;     // chunked sort counts, then in-chunk offsets [nbx][nkeys]
  uint32_t *d_desc = nullptr;     // chunked sort per-track descriptors [C][ncopy][B]
  uint32_t *d_order = nullptr;    // tiles in per-XCD longest-first order [nkeys]
  uint32_t *d_lpt = nullptr;      // LPT bucket counts, offsets, scan scratch, queues
  int schedule = 0;               // rts_schedule in effect
  int nbx = 0;
  int64_t chunk = 0;
  int cg = 1;                     // chunked sort: channels per workgroup
  unsigned long long *d_stats = nullptr;
  double *d_chi2_part = nullptr;
  int64_t list_cap = 0;
  int64_t scan_blocks = 0;
  bool stats_pending = false;   // an update ran since the statistics were read back
  rts_plan_info info{};
};

namespace rts {

using Plan = ::rts_plan_s;

// error state (abi.cpp)
void set_error(const char *fmt, ...);

// kernel launchers (plan.hip)
hipError_t launch_plan_count(const PlanArgs &a, hipStream_t s);
hipError_t launch_plan_scatter(const PlanArgs &a, hipStream_t s);
hipError_t launch_scan(const uint32_t *counts, uint32_t *tile_off, uint32_t *cursor,
                       uint32_t *tmp, int64_t n, hipStream_t s);
hipError_t launch_hist_scan(uint32_t *hist, int nbx, int64_t nkeys, uint32_t *totals, uint32_t *tile_off,
                            uint32_t *tmp, hipStream_t s);
hipError_t launch_coords(const double *uvw, const double *scale, const float *w, int32_t *out,
                         int N, int W, int OS, int C, int B, int T, hipStream_t s);
hipError_t launch_chi2_reduce(const double *part, int64_t n, double *out, hipStream_t s);
hipError_t launch_valid_mask(const uint16_t *coords, uint8_t *mask, int B, int T, int ncopy, int64_t n,
                             hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, int n_cu, hipStream_t s);
// gradient terms (backward.hip)
hipError_t launch_grid_backward(const float2 *vis, const float *w, float2 *d, float *gw, int64_t n, hipStream_t s);
hipError_t launch_chi2_backward(const Plan &P, const float2 *vis, const float *w, const float2 *model,
                                const double *gchi2, float2 *gv, float *gw, const float2 *gres, float2 *gg,
                                hipStream_t s);
// Matrix-core path: largest LDS need of its kernels for this geometry (bytes),
// per-baseline table size (words per table) and its construction.
size_t mfma_lds_bytes(int WN, int OS2, int tile);
int64_t pb_table_words(const Plan &P);
hipError_t build_baseline_tables(const Plan &P, const float *tab, hipStream_t s);

// tile kernels (tile_*.hip)
template <int MODE>
hipError_t launch_tile_mode(const Plan &P, const TileArgs &a, hipStream_t s, bool prepare);
hipError_t launch_tile(int mode, const Plan &P, const TileArgs &a, hipStream_t s);
hipError_t prepare_tile_kernels(const Plan &P);
hipError_t launch_grid_mfma(const Plan &P, const TileArgs &a, hipStream_t s);
double bessel_i0(double x);
void destroy_imager(Plan *P);
hipError_t launch_degrid_mfma(const Plan &P, const TileArgs &a, hipStream_t s);
hipError_t launch_lpt_order(const uint32_t *tile_off, int64_t nkeys, uint32_t *lpt, uint32_t *order, hipStream_t s);
// Longest-first tile order (persistent launch, matrix-core kernels): tiles are
// bucketed by their work-list length (16 buckets per octave) within each eighth
// of the tile range.
// Workspace layout (uint32 words): bucket counts, then their exclusive scan
// (8*kLptBins+1 words), scan block sums, and the eight queue counters.
constexpr int kLptBins = 1024;
constexpr int64_t kLptOff = 8 * kLptBins;
constexpr int64_t kLptTmp = 16 * kLptBins + 8;
constexpr int64_t kLptQueue = kLptTmp + 8;
constexpr int64_t kLptWords = kLptQueue + 8;
bool tile_supported(int W, int seg_max);

}  // namespace rts
