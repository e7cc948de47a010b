// Measurement aid: a streaming device copy, the practical read+write ceiling of the memory system
// that the batched launch is compared with, and the calibration kernel of the HBM traffic
// counters (it reads and writes exactly the bytes it is given).
//
// One 16-byte vector per lane and one pass over the grid: every block copies 4 KB and exits, so
// the blocks in flight at any moment cover a contiguous window of the buffers that moves through
// them in order. On MI355X this one-pass shape copies large buffers at ~6.2 TB/s, where
// persistent grid-strided walks (each block looping over the whole buffer) reach 4.2-5.7 TB/s.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gmm.h"
#include "gmm_internal.hpp"

namespace rgbd {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kBlock) copy16_kernel(const v4u* __restrict__ src, v4u* __restrict__ dst,
                                                        uint64_t n16) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

__global__ void __launch_bounds__(kBlock) copy_tail_kernel(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst,
                                                           uint32_t n) {
  if (threadIdx.x < n) dst[threadIdx.x] = src[threadIdx.x];
}

}  // namespace rgbd

using namespace rgbd;

extern "C" gmm_status gmm_device_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes == 0) return GMM_OK;
  if (!dst || !src) return fail(GMM_ERR_INVALID_ARG, "NULL pointer");
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return fail(GMM_ERR_INVALID_ARG, "dst and src must be 16-byte aligned");
  const uintptr_t d = reinterpret_cast<uintptr_t>(dst), s = reinterpret_cast<uintptr_t>(src);
  if (d < s + bytes && s < d + bytes) return fail(GMM_ERR_INVALID_ARG, "dst and src overlap");
  const uint64_t n16 = bytes / 16;
  const uint64_t blocks = (n16 + kBlock - 1) / kBlock;
  if (blocks >= (1ull << 31)) return fail(GMM_ERR_INVALID_ARG, "copy larger than one launch's grid");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (n16) {
    copy16_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, hs>>>(static_cast<const v4u*>(src),
                                                                                static_cast<v4u*>(dst), n16);
    e = hipGetLastError();
  }
  const uint32_t tail = static_cast<uint32_t>(bytes % 16);
  if (e == hipSuccess && tail) {
    copy_tail_kernel<<<1, dim3(kBlock), 0, hs>>>(static_cast<const uint8_t*>(src) + 16 * n16,
                                                 static_cast<uint8_t*>(dst) + 16 * n16, tail);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(e, "copy kernel launch");
  return GMM_OK;
}
