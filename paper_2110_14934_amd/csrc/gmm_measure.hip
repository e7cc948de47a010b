// Measurement aid: a streaming device copy, the practical read+write ceiling of the memory system
// that the batched launch is compared with, and the calibration kernel of the HBM traffic
// counters (it reads and writes exactly the bytes it is given).
//
// Each lane moves 16-byte vectors in a grid-strided loop with four loads in flight before their
// stores, so a wave issues 4 KB of reads per round; the grid is a multiple of the CU count.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gmm.h"
#include "gmm_internal.hpp"

namespace rgbd {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kBlock) copy16_kernel(const v4u* __restrict__ src, v4u* __restrict__ dst,
                                                        uint64_t n16) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kBlock;
  uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const v4u a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n16; i += stride) dst[i] = src[i];
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
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const uint64_t n16 = bytes / 16;
  if (n16) {
    const uint64_t want = (n16 + 4ull * kBlock - 1) / (4ull * kBlock);
    const unsigned grid = static_cast<unsigned>(std::max<uint64_t>(1, std::min<uint64_t>(want, 16ull * cus)));
    copy16_kernel<<<dim3(grid), dim3(kBlock), 0, hs>>>(static_cast<const v4u*>(src), static_cast<v4u*>(dst), n16);
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
