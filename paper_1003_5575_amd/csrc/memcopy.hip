// Reference streaming copy: the attainable HBM bandwidth of this device, measured
// with the same kind of access the tile kernels make for their bulk traffic
// (16-byte vector loads, non-temporal 16-byte stores, grid-stride over the buffer).
#include "internal.h"

namespace rts {
namespace {

typedef unsigned int rts_u4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_stream_copy(const rts_u4 *__restrict__ src, rts_u4 *__restrict__ dst,
                                                        int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride) {
    const rts_u4 v = src[i];
    __builtin_nontemporal_store(v, &dst[i]);
  }
}

__global__ __launch_bounds__(kBlock) void k_copy_tail(const unsigned char *src, unsigned char *dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, int n_cu, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 > 0) {
    // eight resident workgroups per compute unit, each striding over the buffer
    const int64_t nblk = std::min<int64_t>((n16 + kBlock - 1) / kBlock, (int64_t)n_cu * 8);
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)nblk), dim3(kBlock), 0, s,
                       reinterpret_cast<const rts_u4 *>(src), reinterpret_cast<rts_u4 *>(dst), n16);
  }
  const int64_t tail = bytes - n16 * 16;
  if (tail > 0)
    hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(kBlock), 0, s,
                       static_cast<const unsigned char *>(src) + n16 * 16, static_cast<unsigned char *>(dst) + n16 * 16,
                       tail);
  return hipGetLastError();
}

}  // namespace rts
