// Confusion counts of two bit-packed masks (the quantities of Eqs. 1-3, Sec. V.A).
//
// One lane per mask word: popcounts of pred&truth, pred&~truth, ~pred&~truth, ~pred&truth over
// the valid bits, reduced across the wave with cross-lane adds, then one 64-bit atomic add per
// wave and counter into the 4-entry result (which a first tiny kernel clears).
#include <hip/hip_runtime.h>

#include "gmm.h"
#include "gmm_internal.hpp"

namespace rgbd {

__global__ void __launch_bounds__(4) clear_counts_kernel(unsigned long long* counts) {
  if (threadIdx.x < 4) counts[threadIdx.x] = 0ull;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__global__ void __launch_bounds__(kBlock) confusion_kernel(const uint64_t* __restrict__ pred,
                                                           const uint64_t* __restrict__ truth,
                                                           int64_t npix, int64_t nwords,
                                                           unsigned long long* counts) {
  unsigned long long tp = 0, fp = 0, tn = 0, fn = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t w = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; w < nwords; w += stride) {
    const uint64_t p = pred[w];
    const uint64_t t = truth[w];
    const int64_t rem = npix - w * 64;
    const uint64_t valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
    tp += __popcll(p & t & valid);
    fp += __popcll(p & ~t & valid);
    tn += __popcll(~p & ~t & valid);
    fn += __popcll(~p & t & valid);
  }
  tp = wave_sum(tp);
  fp = wave_sum(fp);
  tn = wave_sum(tn);
  fn = wave_sum(fn);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicAdd(&counts[0], tp);
    atomicAdd(&counts[1], fp);
    atomicAdd(&counts[2], tn);
    atomicAdd(&counts[3], fn);
  }
}

}  // namespace rgbd

using namespace rgbd;

extern "C" gmm_status gmm_mask_confusion(const uint64_t* pred, const uint64_t* truth, int64_t npix,
                                         uint64_t* counts, void* stream) {
  if (!pred || !truth || !counts) return fail(GMM_ERR_INVALID_ARG, "NULL mask or counts");
  if (npix <= 0) return fail(GMM_ERR_INVALID_ARG, "npix must be > 0");
  if ((reinterpret_cast<uintptr_t>(pred) | reinterpret_cast<uintptr_t>(truth) |
       reinterpret_cast<uintptr_t>(counts)) % 8)
    return fail(GMM_ERR_INVALID_ARG, "masks and counts must be 8-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t nwords = (npix + 63) / 64;
  const int64_t blocks = std::min<int64_t>((nwords + kBlock - 1) / kBlock, 1024);
  auto* c = reinterpret_cast<unsigned long long*>(counts);
  clear_counts_kernel<<<1, 4, 0, s>>>(c);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    confusion_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s>>>(pred, truth, npix, nwords, c);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(e, "confusion kernel launch");
  return GMM_OK;
}
