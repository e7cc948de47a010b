// Batched launch for callers that cannot allocate device memory: gmm_batch_apply_static.
//
// gmm_batch_apply keeps each batch's stream descriptors and tile map in device memory that
// gmm_batch_create allocates. This entry point takes the handles directly and keeps the same
// per-call tables in one file-scope device array instead (`scratch`, below): the descriptors of
// up to kStaticMaxStreams streams and each stream's first tile. They reach the device through
// small pack kernels whose arguments carry kPackPerLaunch descriptors each (kernel arguments are
// captured by value, so no host buffer has to outlive the call), and the persistent kernel finds
// a tile's stream by a binary search over the first tiles rather than through a tile map. The
// per-pixel body is the one every other kernel of the library runs, so results are bit-identical
// to gmm_batch_apply.
//
// The array is one per device and shared by every call on that device: calls that overlap on one
// device (different streams, or different host threads without ordering) race on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "gmm.h"
#include "gmm_frame.hpp"
#include "gmm_internal.hpp"

namespace rgbd {

constexpr int kStaticMaxStreams = GMM_STATIC_MAX_STREAMS;
constexpr int kPackPerLaunch = 8;
constexpr size_t kTableBytes = static_cast<size_t>(kStaticMaxStreams) * sizeof(FrameArgs);
constexpr size_t kScratchBytes = (kTableBytes + kStaticMaxStreams * sizeof(uint32_t) + 255) / 256 * 256;
static_assert(kTableBytes % 256 == 0, "the first-tile array starts 256-byte aligned");

// [descriptors: kStaticMaxStreams x FrameArgs][first tile of each stream: kStaticMaxStreams x u32]
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct PackArgs {
  FrameArgs a[kPackPerLaunch];
  uint32_t first[kPackPerLaunch];
  uint32_t base;   // index of a[0] in the tables
  uint32_t count;  // entries used
};

__global__ void __launch_bounds__(64) pack_kernel(PackArgs p, FrameArgs* __restrict__ table,
                                                  uint32_t* __restrict__ first) {
  const uint32_t i = threadIdx.x;
  if (i < p.count) {
    table[p.base + i] = p.a[i];
    first[p.base + i] = p.first[i];
  }
}

template <int M, typename S, int BLOCK, bool MEASURE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5))) batch_search_kernel(const FrameArgs* __restrict__ table,
                                                             const uint32_t* __restrict__ first,
                                                             uint32_t n_streams, uint32_t n_tiles,
                                                             uint32_t tile_px) {
  __shared__ uint32_t lds[BLOCK / kWave][48];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    // the last stream whose first tile is <= t (first[0] = 0, increasing)
    uint32_t lo = 0, hi = n_streams - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (first[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const FrameArgs a = table[lo];
    const uint32_t t0 = (t - first[lo]) * tile_px;
    process_tile<M, S, BLOCK, MEASURE>(a, t0, tile_px, lane, lds[wv]);
  }
}

template <int M, typename S, bool MEASURE>
static hipError_t launch_search_msm(int block, dim3 grid, const FrameArgs* table, const uint32_t* first,
                                    uint32_t n, uint32_t n_tiles, uint32_t tile_px, hipStream_t s) {
  if (block == 256)
    batch_search_kernel<M, S, 256, MEASURE><<<grid, dim3(256), 0, s>>>(table, first, n, n_tiles, tile_px);
  else if (block == 512)
    batch_search_kernel<M, S, 512, MEASURE><<<grid, dim3(512), 0, s>>>(table, first, n, n_tiles, tile_px);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int M, typename S>
static hipError_t launch_search_ms(int block, dim3 grid, const FrameArgs* table, const uint32_t* first,
                                   uint32_t n, uint32_t n_tiles, uint32_t tile_px, bool measure, hipStream_t s) {
  return measure ? launch_search_msm<M, S, true>(block, grid, table, first, n, n_tiles, tile_px, s)
                 : launch_search_msm<M, S, false>(block, grid, table, first, n, n_tiles, tile_px, s);
}

template <typename S>
static hipError_t launch_search_s(int M, int block, dim3 grid, const FrameArgs* table, const uint32_t* first,
                                  uint32_t n, uint32_t n_tiles, uint32_t tile_px, bool measure, hipStream_t s) {
  switch (M) {
    case 1: return launch_search_ms<1, S>(block, grid, table, first, n, n_tiles, tile_px, measure, s);
    case 2: return launch_search_ms<2, S>(block, grid, table, first, n, n_tiles, tile_px, measure, s);
    case 3: return launch_search_ms<3, S>(block, grid, table, first, n, n_tiles, tile_px, measure, s);
    case 4: return launch_search_ms<4, S>(block, grid, table, first, n, n_tiles, tile_px, measure, s);
    case 5: return launch_search_ms<5, S>(block, grid, table, first, n, n_tiles, tile_px, measure, s);
    default: return hipErrorInvalidValue;
  }
}

// `measure`: some descriptor has a traffic record (see launch_batch).
static hipError_t launch_search(int M, int dtype, int block, dim3 grid, const FrameArgs* table,
                                const uint32_t* first, uint32_t n, uint32_t n_tiles, uint32_t tile_px,
                                bool measure, hipStream_t s) {
  switch (dtype) {
    case GMM_F32: return launch_search_s<float>(M, block, grid, table, first, n, n_tiles, tile_px, measure, s);
    case GMM_F16: return launch_search_s<f16s>(M, block, grid, table, first, n, n_tiles, tile_px, measure, s);
    case GMM_BF16: return launch_search_s<bf16s>(M, block, grid, table, first, n, n_tiles, tile_px, measure, s);
    default: return hipErrorInvalidValue;
  }
}

// Per device: the device address of `scratch` (from hipGetSymbolAddress, taken once with the
// device current; the array's name in host code is not a device address) and the CU count.
constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;
static bool g_static_ready[kMaxDevices];
static uint8_t* g_scratch_ptr[kMaxDevices];
static int g_static_cus[kMaxDevices];

static gmm_status static_setup(int dev, uint8_t** ptr, int* cus) {
  if (dev < 0 || dev >= kMaxDevices) return fail(GMM_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ready[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static scratch array");
    if (p == nullptr) return fail(GMM_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
    int n = 0;
    e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "CU count");
    g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
    g_static_cus[dev] = n;
    g_static_ready[dev] = true;
  }
  *ptr = g_scratch_ptr[dev];
  *cus = g_static_cus[dev];
  return GMM_OK;
}

}  // namespace rgbd

using namespace rgbd;

extern "C" gmm_status gmm_batch_apply_static(gmm_handle* const* handles, int32_t n, const gmm_stream_io* io,
                                             const gmm_batch_tuning* tuning, void* stream) {
  if (n < 1 || n > kStaticMaxStreams)
    return fail(GMM_ERR_INVALID_ARG, "n must be in 1.." + std::to_string(kStaticMaxStreams) +
                                         " (the size of the static descriptor table)");
  if (!handles || !io) return fail(GMM_ERR_INVALID_ARG, "NULL handles or io");
  const gmm_batch_tuning t = tuning ? *tuning : gmm_batch_tuning{256, 1024, 8};
  if (t.block_threads != 256 && t.block_threads != 512)
    return fail(GMM_ERR_INVALID_ARG, "block_threads must be 256 or 512");
  if (t.tile_pixels < t.block_threads || t.tile_pixels % t.block_threads || t.tile_pixels > 64 * t.block_threads)
    return fail(GMM_ERR_INVALID_ARG, "tile_pixels must be a multiple of block_threads, at most 64x it");
  if (t.blocks_per_cu < 1 || t.blocks_per_cu > 32) return fail(GMM_ERR_INVALID_ARG, "blocks_per_cu must be in 1..32");
  // every handle once (a handle twice would race inside the launch): sorted copy on the stack
  const gmm_handle* sorted[kStaticMaxStreams];
  for (int32_t i = 0; i < n; ++i) {
    const gmm_handle* h = handles[i];
    if (!h) return fail(GMM_ERR_INVALID_ARG, "NULL handle");
    if (is_augmented(h)) return fail(GMM_ERR_UNSUPPORTED, "augmented handles run one at a time");
    if (h->cfg.device != handles[0]->cfg.device || h->cfg.M != handles[0]->cfg.M ||
        h->cfg.state_dtype != handles[0]->cfg.state_dtype)
      return fail(GMM_ERR_INVALID_ARG, "all handles need the same device, M and state dtype");
    sorted[i] = h;
  }
  std::sort(sorted, sorted + n);
  for (int32_t i = 1; i < n; ++i)
    if (sorted[i] == sorted[i - 1]) return fail(GMM_ERR_INVALID_ARG, "a handle appears twice");
  uint64_t total = 0;
  for (int32_t i = 0; i < n; ++i) {
    gmm_handle* h = handles[i];
    const gmm_stream_io& s = io[i];
    gmm_status st = check_frame_args(h, s.rgb, s.rgb_pitch_bytes, s.depth, s.depth_pitch_bytes, s.fg_rgb, s.fg_depth);
    if (st != GMM_OK) {
      set_error("stream " + std::to_string(i) + ": " + gmm_last_error());
      return st;
    }
    if (s.fused) {
      if (!has_both(h)) return fail(GMM_ERR_STATE, "stream " + std::to_string(i) + ": fusion needs both modalities");
      if (reinterpret_cast<uintptr_t>(s.fused) % 8)
        return fail(GMM_ERR_INVALID_ARG, "stream " + std::to_string(i) + ": fused mask not 8-byte aligned");
    }
    total += (static_cast<uint64_t>(h->npix) + t.tile_pixels - 1) / t.tile_pixels;
  }
  if (total >= (1ull << 31)) return fail(GMM_ERR_INVALID_ARG, "too many tiles in one launch");
  const int dev = handles[0]->cfg.device;
  DeviceGuard g(dev);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the handles' device");
  uint8_t* base = nullptr;
  int cus = 0;
  gmm_status st = static_setup(dev, &base, &cus);
  if (st != GMM_OK) return st;
  FrameArgs* table = reinterpret_cast<FrameArgs*>(base);
  uint32_t* first = reinterpret_cast<uint32_t*>(base + kTableBytes);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  uint32_t next_first = 0;
  bool measure = false;
  for (int32_t b = 0; b < n && e == hipSuccess; b += kPackPerLaunch) {
    PackArgs p{};
    p.base = static_cast<uint32_t>(b);
    p.count = static_cast<uint32_t>(std::min(kPackPerLaunch, n - b));
    for (uint32_t i = 0; i < p.count; ++i) {
      gmm_handle* h = handles[b + i];
      const gmm_stream_io& s = io[b + i];
      p.a[i] = frame_args(h, s.rgb, s.rgb_pitch_bytes, s.depth, s.depth_pitch_bytes, s.fg_rgb, s.fg_depth, s.fused);
      measure = measure || p.a[i].wave_bytes != nullptr;
      p.first[i] = next_first;
      next_first += static_cast<uint32_t>((h->npix + t.tile_pixels - 1) / t.tile_pixels);
    }
    pack_kernel<<<1, 64, 0, hs>>>(p, table, first);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(e, "descriptor pack kernel launch");
  const uint32_t n_tiles = static_cast<uint32_t>(total);
  const uint32_t want = static_cast<uint32_t>(t.blocks_per_cu) * static_cast<uint32_t>(cus);
  const dim3 grid(std::max(1u, std::min(want, n_tiles)));
  e = launch_search(handles[0]->cfg.M, handles[0]->cfg.state_dtype, t.block_threads, grid, table, first,
                    static_cast<uint32_t>(n), n_tiles, static_cast<uint32_t>(t.tile_pixels), measure, hs);
  if (e != hipSuccess) return hip_fail(e, "static batch kernel launch");
  for (int32_t i = 0; i < n; ++i) handles[i]->last_stream = hs;
  return GMM_OK;
}
