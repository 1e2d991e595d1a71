// Instantiation of the tile kernel for every supported (W+1, samples-per-segment)
// pair of one mode.  Included once per mode so the three modes compile in parallel.
#pragma once

#include "tile_kernel.h"

namespace rts {

// With prepare set, only raise the kernel's dynamic-LDS limit (done once, when a
// plan is built, so that launches stay capturable); otherwise launch.
#define RTS_TILE_LAUNCH(WNV, SM, BLK, GRP)                                                     \
  {                                                                                            \
    if (prepare) {                                                                             \
      if (lds > 65536) {                                                                       \
        hipError_t e = hipFuncSetAttribute((const void *)k_tile<WNV, SM, MODE, BLK, GRP>,      \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        if (e != hipSuccess) return e;                                                         \
        return hipFuncSetAttribute((const void *)k_tile_persistent<WNV, SM, MODE, BLK, GRP>,   \
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);      \
      }                                                                                        \
      return hipSuccess;                                                                       \
    }                                                                                          \
    if (persistent) {                                                                          \
      hipError_t e = launch_fill_u32(a.queue, 8, 0u, s);                                       \
      if (e != hipSuccess) return e;                                                           \
      hipLaunchKernelGGL((k_tile_persistent<WNV, SM, MODE, BLK, GRP>), dim3(npers), dim3(BLK), lds, s, a); \
    } else {                                                                                   \
      hipLaunchKernelGGL((k_tile<WNV, SM, MODE, BLK, GRP>), dim3(nblk), dim3(BLK), lds, s, a);  \
    }                                                                                          \
  }
// Windows up to 8 cells run with 128 registers and four waves per SIMD: small
// tiles in 128-thread workgroups, larger tiles in 512-thread workgroups (two per
// compute unit, which is what the LDS of the FP64 accumulator allows, so eight
// waves per CU instead of four: the batched workload's four-sample segments are
// latency-bound).  Wider windows use 256-thread workgroups with the 256-register
// budget (they would spill with 128).
#define RTS_TILE_CASE(WNV, SM)                                                        \
  case (WNV)*16 + (SM):                                                               \
    if ((WNV) <= 8 && P.tile <= 32) RTS_TILE_LAUNCH(WNV, SM, 128, 4)                  \
    else if ((WNV) <= 8) RTS_TILE_LAUNCH(WNV, SM, 512, 4)                             \
    else RTS_TILE_LAUNCH(WNV, SM, 256, 4)                                             \
    break;

template <int MODE>
hipError_t launch_tile_mode(const Plan &P, const TileArgs &a, hipStream_t s, bool prepare) {
  const unsigned nblk = (unsigned)P.nkeys;
  // Persistent launch: as many workgroups as fit on the GPU at once (LDS decides
  // for large tiles), never more than there are tiles.
  const bool persistent = P.schedule == RTS_SCHEDULE_PERSISTENT && a.order && a.queue;
  const int per_cu = (P.tile >= 64) ? 2 : 6;
  const unsigned npers = (unsigned)std::min<int64_t>(P.nkeys, (int64_t)P.n_cu * per_cu);
  size_t lds0 = (size_t)a.OS2 * a.WNP * sizeof(float);
  if (MODE != kDegrid) lds0 += (size_t)2 * P.tile * (P.tile + kAccPad) * sizeof(double);
  // 512-thread workgroups also hold a sorted batch of listings
  const size_t lds = lds0 + ((P.WN <= 8 && P.tile > 32) ? (size_t)kSortBatch * sizeof(uint2) : 0);
  switch (P.WN * 16 + P.seg_max) {
    RTS_TILE_CASE(3, 4) RTS_TILE_CASE(3, 8)
    RTS_TILE_CASE(4, 4) RTS_TILE_CASE(4, 8)
    RTS_TILE_CASE(5, 4) RTS_TILE_CASE(5, 8)
    RTS_TILE_CASE(6, 4) RTS_TILE_CASE(6, 8)
    RTS_TILE_CASE(7, 4) RTS_TILE_CASE(7, 8)
    RTS_TILE_CASE(8, 4) RTS_TILE_CASE(8, 8)
    RTS_TILE_CASE(9, 4) RTS_TILE_CASE(9, 8)
    RTS_TILE_CASE(10, 4) RTS_TILE_CASE(11, 4) RTS_TILE_CASE(12, 4) RTS_TILE_CASE(13, 4)
    RTS_TILE_CASE(14, 2) RTS_TILE_CASE(15, 2) RTS_TILE_CASE(16, 2) RTS_TILE_CASE(17, 2)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#undef RTS_TILE_CASE
#undef RTS_TILE_LAUNCH

}  // namespace rts
