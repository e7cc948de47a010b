// Batched path: every stream of a batch advances one frame in ONE persistent launch.
//
// Work is cut into tiles of `tile_pixels` consecutive pixels of one stream (a multiple of the
// block size, so tiles start on mask-word boundaries). A device tile map gives each tile's
// stream; per-stream kernel arguments (frame and mask pointers, state blocks, constants) live in
// a device descriptor table with one slot per prepared frame-set. The grid is a multiple of the
// CU count and each block walks tiles b, b+G, b+2G, ... so every block samples every stream and
// uneven resolutions balance without atomics. The per-pixel body is the one the single-stream
// kernel uses (process_pixel), so results are bit-identical to one launch per stream.
//
// A launch reads only device memory prepared earlier (descriptor slot, tile map): it allocates
// nothing and synchronises nothing, so it can be captured into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "gmm.h"
#include "gmm_frame.hpp"
#include "gmm_internal.hpp"

namespace rgbd {

// Five waves per SIMD: the body fits them without spilling (checked at build time by the tests).
// MEASURE: the body that adds each wave's state bytes to the streams' traffic records; the launch
// takes it only when a stream of the batch has one, so the common body never forms the counts.
template <int M, typename S, int BLOCK, bool MEASURE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5))) batch_kernel(const FrameArgs* __restrict__ table,
                                                      const uint32_t* __restrict__ tile_map,
                                                      const uint32_t* __restrict__ first_tile,
                                                      uint32_t n_tiles, uint32_t tile_px) {
  __shared__ uint32_t lds[BLOCK / kWave][48];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const uint32_t s = tile_map[t];
    const FrameArgs a = table[s];
    const uint32_t t0 = (t - first_tile[s]) * tile_px;
    process_tile<M, S, BLOCK, MEASURE>(a, t0, tile_px, lane, lds[wv]);
  }
}

template <int M, typename S, bool MEASURE>
static hipError_t launch_batch_msm(int block, dim3 grid, const FrameArgs* table, const uint32_t* map,
                                   const uint32_t* first, uint32_t n_tiles, uint32_t tile_px, hipStream_t s) {
  if (block == 256)
    batch_kernel<M, S, 256, MEASURE><<<grid, dim3(256), 0, s>>>(table, map, first, n_tiles, tile_px);
  else if (block == 512)
    batch_kernel<M, S, 512, MEASURE><<<grid, dim3(512), 0, s>>>(table, map, first, n_tiles, tile_px);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int M, typename S>
static hipError_t launch_batch_ms(int block, dim3 grid, const FrameArgs* table, const uint32_t* map,
                                  const uint32_t* first, uint32_t n_tiles, uint32_t tile_px, bool measure,
                                  hipStream_t s) {
  return measure ? launch_batch_msm<M, S, true>(block, grid, table, map, first, n_tiles, tile_px, s)
                 : launch_batch_msm<M, S, false>(block, grid, table, map, first, n_tiles, tile_px, s);
}

template <typename S>
static hipError_t launch_batch_s(int M, int block, dim3 grid, const FrameArgs* table, const uint32_t* map,
                                 const uint32_t* first, uint32_t n_tiles, uint32_t tile_px, bool measure,
                                 hipStream_t s) {
  switch (M) {
    case 1: return launch_batch_ms<1, S>(block, grid, table, map, first, n_tiles, tile_px, measure, s);
    case 2: return launch_batch_ms<2, S>(block, grid, table, map, first, n_tiles, tile_px, measure, s);
    case 3: return launch_batch_ms<3, S>(block, grid, table, map, first, n_tiles, tile_px, measure, s);
    case 4: return launch_batch_ms<4, S>(block, grid, table, map, first, n_tiles, tile_px, measure, s);
    case 5: return launch_batch_ms<5, S>(block, grid, table, map, first, n_tiles, tile_px, measure, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch(int M, int dtype, int block, dim3 grid, const FrameArgs* table,
                               const uint32_t* map, const uint32_t* first, uint32_t n_tiles,
                               uint32_t tile_px, bool measure, hipStream_t s) {
  switch (dtype) {
    case GMM_F32: return launch_batch_s<float>(M, block, grid, table, map, first, n_tiles, tile_px, measure, s);
    case GMM_F16: return launch_batch_s<f16s>(M, block, grid, table, map, first, n_tiles, tile_px, measure, s);
    case GMM_BF16: return launch_batch_s<bf16s>(M, block, grid, table, map, first, n_tiles, tile_px, measure, s);
    default: return hipErrorInvalidValue;
  }
}

// Tunings found by the autotuner, per (device, M, dtype, stream mix), for this process.
static std::mutex g_tune_mu;
static std::map<std::string, std::pair<gmm_batch_tuning, double>> g_tune_cache;

}  // namespace rgbd

using namespace rgbd;

struct gmm_batch {
  int device = 0;
  int M = 0;
  int dtype = 0;
  int cu_count = 0;
  std::vector<gmm_handle*> handles;
  int n_slots = 0;
  FrameArgs* d_table = nullptr;              // n_slots x n descriptors
  std::vector<FrameArgs*> h_staging;         // pinned, one per slot
  std::vector<hipEvent_t> staging_done;      // last upload from each staging buffer
  std::vector<uint8_t> slot_ready;
  std::vector<uint8_t> slot_measure;         // a stream of the slot's descriptors has a traffic record
  uint32_t* d_tile_map = nullptr;
  size_t tile_map_cap = 0;
  uint32_t* d_first_tile = nullptr;
  uint32_t n_tiles = 0;
  gmm_batch_tuning tuning{256, 1024, 8};
  hipStream_t last_stream = nullptr;
};

static size_t n_streams(const gmm_batch* b) { return b->handles.size(); }

static gmm_status validate_tuning(const gmm_batch_tuning* t) {
  if (!t) return fail(GMM_ERR_INVALID_ARG, "tuning is NULL");
  if (t->block_threads != 256 && t->block_threads != 512)
    return fail(GMM_ERR_INVALID_ARG, "block_threads must be 256 or 512");
  if (t->tile_pixels < t->block_threads || t->tile_pixels % t->block_threads ||
      t->tile_pixels > 64 * t->block_threads)
    return fail(GMM_ERR_INVALID_ARG, "tile_pixels must be a multiple of block_threads, at most 64x it");
  if (t->blocks_per_cu < 1 || t->blocks_per_cu > 32) return fail(GMM_ERR_INVALID_ARG, "blocks_per_cu must be in 1..32");
  return GMM_OK;
}

// Rebuild the tile map for tile size `tile_px` (synchronous; not for use under capture).
static gmm_status build_tiles(gmm_batch* b, uint32_t tile_px) {
  std::vector<uint32_t> first(n_streams(b));
  uint64_t total = 0;
  for (size_t i = 0; i < n_streams(b); ++i) {
    first[i] = static_cast<uint32_t>(total);
    total += (static_cast<uint64_t>(b->handles[i]->npix) + tile_px - 1) / tile_px;
  }
  if (total >= (1ull << 31)) return fail(GMM_ERR_INVALID_ARG, "too many tiles in one batch");
  std::vector<uint32_t> map(total);
  for (size_t i = 0; i < n_streams(b); ++i) {
    const uint32_t end = i + 1 < n_streams(b) ? first[i + 1] : static_cast<uint32_t>(total);
    std::fill(map.begin() + first[i], map.begin() + end, static_cast<uint32_t>(i));
  }
  hipError_t e = hipSuccess;
  if (total > b->tile_map_cap) {
    if (b->d_tile_map) (void)hipFree(b->d_tile_map);
    b->d_tile_map = nullptr;
    b->tile_map_cap = 0;
    e = hipMalloc(&b->d_tile_map, total * sizeof(uint32_t));
    if (e != hipSuccess) return fail(GMM_ERR_OUT_OF_MEMORY, "tile map allocation failed");
    b->tile_map_cap = total;
  }
  e = hipMemcpy(b->d_tile_map, map.data(), total * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_first_tile, first.data(), first.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "tile map upload");
  b->n_tiles = static_cast<uint32_t>(total);
  return GMM_OK;
}

static gmm_status apply_tuning(gmm_batch* b, const gmm_batch_tuning& t) {
  if (t.tile_pixels != b->tuning.tile_pixels || b->n_tiles == 0) {
    gmm_status st = build_tiles(b, static_cast<uint32_t>(t.tile_pixels));
    if (st != GMM_OK) return st;
  }
  b->tuning = t;
  return GMM_OK;
}

static hipError_t run_slot(gmm_batch* b, int slot, hipStream_t s) {
  const uint32_t want = static_cast<uint32_t>(b->tuning.blocks_per_cu) * static_cast<uint32_t>(b->cu_count);
  const dim3 grid(std::max(1u, std::min(want, b->n_tiles)));
  return launch_batch(b->M, b->dtype, b->tuning.block_threads, grid, b->d_table + static_cast<size_t>(slot) * n_streams(b),
                      b->d_tile_map, b->d_first_tile, b->n_tiles, static_cast<uint32_t>(b->tuning.tile_pixels),
                      b->slot_measure[slot] != 0, s);
}

static void free_batch(gmm_batch* b) {
  for (auto* p : b->h_staging)
    if (p) (void)hipHostFree(p);
  for (auto ev : b->staging_done)
    if (ev) (void)hipEventDestroy(ev);
  if (b->d_table) (void)hipFree(b->d_table);
  if (b->d_tile_map) (void)hipFree(b->d_tile_map);
  if (b->d_first_tile) (void)hipFree(b->d_first_tile);
  delete b;
}

static std::string mix_key(const gmm_batch* b) {
  hipDeviceProp_t prop;
  std::ostringstream k;
  if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) k << prop.gcnArchName << "/" << prop.multiProcessorCount;
  k << "|M" << b->M << "|d" << b->dtype;
  std::vector<std::string> parts;
  for (auto* h : b->handles) {
    std::ostringstream s;
    s << h->cfg.width << "x" << h->cfg.height << "m" << h->cfg.modalities;
    parts.push_back(s.str());
  }
  std::sort(parts.begin(), parts.end());
  for (auto& p : parts) k << "|" << p;
  return k.str();
}

extern "C" {

gmm_status gmm_batch_create(gmm_handle* const* handles, int32_t n, int32_t n_slots, gmm_batch** out) {
  if (!out) return fail(GMM_ERR_INVALID_ARG, "out is NULL");
  if (!handles || n <= 0) return fail(GMM_ERR_INVALID_ARG, "a batch needs at least one handle");
  if (n_slots < 1 || n_slots > 4096) return fail(GMM_ERR_INVALID_ARG, "n_slots must be in 1..4096");
  std::set<const gmm_handle*> seen;
  for (int32_t i = 0; i < n; ++i) {
    const gmm_handle* h = handles[i];
    if (!h) return fail(GMM_ERR_INVALID_ARG, "NULL handle in batch");
    if (!seen.insert(h).second) return fail(GMM_ERR_INVALID_ARG, "a handle appears twice in the batch");
    if (is_augmented(h)) return fail(GMM_ERR_UNSUPPORTED, "augmented handles run one at a time");
    if (h->cfg.device != handles[0]->cfg.device || h->cfg.M != handles[0]->cfg.M ||
        h->cfg.state_dtype != handles[0]->cfg.state_dtype)
      return fail(GMM_ERR_INVALID_ARG, "all handles of a batch need the same device, M and state dtype");
  }
  gmm_batch* b = new (std::nothrow) gmm_batch();
  if (!b) return fail(GMM_ERR_OUT_OF_MEMORY, "host allocation of the batch failed");
  b->handles.assign(handles, handles + n);
  b->device = handles[0]->cfg.device;
  b->M = handles[0]->cfg.M;
  b->dtype = handles[0]->cfg.state_dtype;
  b->n_slots = n_slots;
  DeviceGuard g(b->device);
  if (!g.ok()) {
    delete b;
    return fail(GMM_ERR_DEVICE, "cannot select the handles' device");
  }
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, b->device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipGetDeviceProperties");
  }
  b->cu_count = prop.multiProcessorCount;
  const size_t tbytes = static_cast<size_t>(n_slots) * n * sizeof(FrameArgs);
  e = hipMalloc(&b->d_table, tbytes);
  if (e == hipSuccess) e = hipMalloc(&b->d_first_tile, static_cast<size_t>(n) * sizeof(uint32_t));
  if (e != hipSuccess) {
    free_batch(b);
    return fail(GMM_ERR_OUT_OF_MEMORY, "device allocation of the batch tables failed");
  }
  b->h_staging.assign(n_slots, nullptr);
  b->staging_done.assign(n_slots, nullptr);
  b->slot_ready.assign(n_slots, 0);
  b->slot_measure.assign(n_slots, 0);
  for (int32_t s = 0; s < n_slots; ++s) {
    e = hipHostMalloc(reinterpret_cast<void**>(&b->h_staging[s]), static_cast<size_t>(n) * sizeof(FrameArgs),
                      hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staging_done[s], hipEventDisableTiming);
    if (e != hipSuccess) {
      free_batch(b);
      return fail(GMM_ERR_OUT_OF_MEMORY, "pinned staging allocation failed");
    }
  }
  gmm_status st = build_tiles(b, static_cast<uint32_t>(b->tuning.tile_pixels));
  if (st != GMM_OK) {
    free_batch(b);
    return st;
  }
  *out = b;
  return GMM_OK;
}

gmm_status gmm_batch_destroy(gmm_batch* b) {
  if (!b) return GMM_OK;
  gmm_status st = GMM_OK;
  {
    DeviceGuard g(b->device);
    hipError_t e = hipStreamSynchronize(b->last_stream);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize in batch destroy");
    for (auto ev : b->staging_done) (void)hipEventSynchronize(ev);
    free_batch(b);
  }
  return st;
}

gmm_status gmm_batch_set_tuning(gmm_batch* b, const gmm_batch_tuning* t) {
  if (!b) return fail(GMM_ERR_INVALID_ARG, "batch is NULL");
  gmm_status st = validate_tuning(t);
  if (st != GMM_OK) return st;
  DeviceGuard g(b->device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the batch's device");
  (void)hipStreamSynchronize(b->last_stream);  // the tile map may be rebuilt
  return apply_tuning(b, *t);
}

gmm_status gmm_batch_get_tuning(const gmm_batch* b, gmm_batch_tuning* t) {
  if (!b || !t) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  *t = b->tuning;
  return GMM_OK;
}

gmm_status gmm_batch_set_frames(gmm_batch* b, int32_t slot, const gmm_stream_io* io, void* stream) {
  if (!b || !io) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  if (slot < 0 || slot >= b->n_slots) return fail(GMM_ERR_INVALID_ARG, "slot out of range");
  // validate every stream before touching anything
  for (size_t i = 0; i < n_streams(b); ++i) {
    gmm_handle* h = b->handles[i];
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
  }
  DeviceGuard g(b->device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the batch's device");
  hipError_t e = hipEventSynchronize(b->staging_done[slot]);  // previous upload from this buffer
  if (e != hipSuccess) return hip_fail(e, "staging event");
  FrameArgs* host = b->h_staging[slot];
  bool measure = false;
  for (size_t i = 0; i < n_streams(b); ++i) {
    const gmm_stream_io& s = io[i];
    host[i] = frame_args(b->handles[i], s.rgb, s.rgb_pitch_bytes, s.depth, s.depth_pitch_bytes, s.fg_rgb,
                         s.fg_depth, s.fused);
    measure = measure || host[i].wave_bytes != nullptr;
  }
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const size_t bytes = n_streams(b) * sizeof(FrameArgs);
  e = hipMemcpyAsync(b->d_table + static_cast<size_t>(slot) * n_streams(b), host, bytes, hipMemcpyHostToDevice, hs);
  if (e == hipSuccess) e = hipEventRecord(b->staging_done[slot], hs);
  if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  b->slot_ready[slot] = 1;
  b->slot_measure[slot] = measure ? 1 : 0;
  b->last_stream = hs;
  return GMM_OK;
}

gmm_status gmm_batch_run(gmm_batch* b, int32_t slot, void* stream) {
  if (!b) return fail(GMM_ERR_INVALID_ARG, "batch is NULL");
  if (slot < 0 || slot >= b->n_slots) return fail(GMM_ERR_INVALID_ARG, "slot out of range");
  if (!b->slot_ready[slot]) return fail(GMM_ERR_STATE, "slot has no frames (call gmm_batch_set_frames first)");
  DeviceGuard g(b->device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the batch's device");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e = run_slot(b, slot, hs);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  b->last_stream = hs;
  for (auto* h : b->handles) h->last_stream = hs;
  return GMM_OK;
}

gmm_status gmm_batch_apply(gmm_batch* b, const gmm_stream_io* io, void* stream) {
  gmm_status st = gmm_batch_set_frames(b, 0, io, stream);
  if (st != GMM_OK) return st;
  return gmm_batch_run(b, 0, stream);
}

gmm_status gmm_batch_autotune(gmm_batch* b, int32_t slot, void* stream, gmm_batch_tuning* best_out,
                              double* best_ms_out) {
  if (!b) return fail(GMM_ERR_INVALID_ARG, "batch is NULL");
  if (slot < 0 || slot >= b->n_slots) return fail(GMM_ERR_INVALID_ARG, "slot out of range");
  if (!b->slot_ready[slot]) return fail(GMM_ERR_STATE, "slot has no frames (call gmm_batch_set_frames first)");
  DeviceGuard g(b->device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the batch's device");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const std::string key = mix_key(b);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      (void)hipStreamSynchronize(hs);
      gmm_status st = apply_tuning(b, it->second.first);
      if (st != GMM_OK) return st;
      if (best_out) *best_out = it->second.first;
      if (best_ms_out) *best_ms_out = it->second.second;
      return GMM_OK;
    }
  }
  // trial launches advance the streams: keep a copy of every state and put it back afterwards
  size_t total = 0;
  for (auto* h : b->handles) total += h->rgb_bytes + h->depth_bytes + h->fuse_bytes;
  void* backup = nullptr;
  hipError_t e = hipMalloc(&backup, total);
  if (e != hipSuccess) return fail(GMM_ERR_OUT_OF_MEMORY, "autotune state backup allocation failed");
  auto copy_states = [&](bool save) -> hipError_t {
    size_t off = 0;
    for (auto* h : b->handles) {
      const size_t nb = h->rgb_bytes + h->depth_bytes + h->fuse_bytes;
      char* bk = static_cast<char*>(backup) + off;
      hipError_t r = save ? hipMemcpyAsync(bk, h->mem, nb, hipMemcpyDeviceToDevice, hs)
                          : hipMemcpyAsync(h->mem, bk, nb, hipMemcpyDeviceToDevice, hs);
      if (r != hipSuccess) return r;
      off += nb;
    }
    return hipStreamSynchronize(hs);
  };
  e = copy_states(true);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const gmm_batch_tuning start = b->tuning;
  gmm_batch_tuning best = start;
  double best_ms = 1e30;
  gmm_status st = GMM_OK;
  // every candidate is timed from the same saved state on the same frame-sets (`slot` and the
  // prepared slots after it, cyclically), so all see the same mix of pixels that keep their
  // top component and pixels that do not
  std::vector<int32_t> slots;
  for (int32_t i = 0; i < b->n_slots && slots.size() < 4; ++i) {
    const int32_t sl = (slot + i) % b->n_slots;
    if (b->slot_ready[sl]) slots.push_back(sl);
  }
  if (e == hipSuccess) {
    const int blocks[] = {256, 512};
    const int tile_mult[] = {1, 2, 4, 8, 16};
    const int per_cu[] = {2, 4, 8, 16};
    for (int bt : blocks) {
      for (int tm : tile_mult) {
        for (int pc : per_cu) {
          gmm_batch_tuning t{bt, bt * tm, pc};
          st = apply_tuning(b, t);
          if (st != GMM_OK) break;
          e = run_slot(b, slot, hs);  // warm-up
          if (e == hipSuccess) e = copy_states(false);
          if (e == hipSuccess) e = hipEventRecord(e0, hs);
          const int reps = static_cast<int>(slots.size());
          for (int r = 0; r < reps && e == hipSuccess; ++r) e = run_slot(b, slots[r], hs);
          if (e == hipSuccess) e = hipEventRecord(e1, hs);
          if (e == hipSuccess) e = copy_states(false);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess) break;
          const double avg = ms / reps;
          if (avg < best_ms) {
            best_ms = avg;
            best = t;
          }
        }
        if (e != hipSuccess || st != GMM_OK) break;
      }
      if (e != hipSuccess || st != GMM_OK) break;
    }
  }
  hipError_t er = copy_states(false);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(backup);
  if (e != hipSuccess) return hip_fail(e, "autotune trial");
  if (er != hipSuccess) return hip_fail(er, "autotune state restore");
  if (st != GMM_OK) return st;
  st = apply_tuning(b, best);
  if (st != GMM_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {best, best_ms};
  }
  if (best_out) *best_out = best;
  if (best_ms_out) *best_ms_out = best_ms;
  b->last_stream = hs;
  return GMM_OK;
}

gmm_status gmm_batch_tiles(const gmm_batch* b, uint32_t* n_tiles) {
  if (!b || !n_tiles) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  *n_tiles = b->n_tiles;
  return GMM_OK;
}

}  // extern "C"
