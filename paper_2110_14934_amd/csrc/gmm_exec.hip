// Serving executor: one call advances an arbitrary set of attached streams by one frame each,
// taking their frames from (pinned) host memory and returning masks to host memory.
//
// Per tick, HIP streams form the pipeline of the paper's Fig. 4(a): the frames of tick N+1 are
// copied host->device while tick N is computed and the masks of tick N-1 are copied back.
// Within a tick: host->device frame copies (spread over four copy-in streams, so several DMA
// engines share the host link) -> descriptor upload, a
// device-built tile map and one persistent batched launch (compute stream) -> mask copies
// device->host (copy-out stream). A ring of `ring` tick slots bounds the work in flight; a
// completion thread waits on each tick's last event in order and records its completion time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "gmm.h"
#include "gmm_frame.hpp"
#include "gmm_internal.hpp"

namespace rgbd {

// tile_map[t] = the entry e with first[e] <= t < first[e + 1] (first has n + 1 entries)
__global__ void __launch_bounds__(kBlock) tile_map_kernel(const uint32_t* __restrict__ first, uint32_t n,
                                                         uint32_t* __restrict__ tile_map) {
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= first[n]) return;
  uint32_t lo = 0, hi = n;  // invariant: first[lo] <= t < first[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (first[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  tile_map[t] = lo;
}

static double now_s() {
  using namespace std::chrono;
  return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace rgbd

using namespace rgbd;

namespace {

// A stream's two device frame slots: its frames alternate between them, so frame n+1 can be
// copied in while the tick holding frame n still computes (the state itself is ordered by the
// compute stream). At most two frames of a stream are in flight.
constexpr int kFramesInFlight = 2;

struct Attached {
  void* base = nullptr;                        // the device allocation holding the slots (or none)
  uint8_t* d_rgb[kFramesInFlight] = {};        // dense colour slots (3 bytes per pixel)
  uint16_t* d_depth[kFramesInFlight] = {};     // dense depth slots (2 bytes per pixel)
  size_t bytes = 0;
  int in_flight = 0;
  uint64_t frames = 0;                         // frames launched; frame f uses slot f % 2
};

// Bytes of one frame slot of h: colour then depth, each rounded up to 256 bytes.
static size_t frame_slot_bytes(const gmm_handle* h) {
  const size_t n = static_cast<size_t>(h->npix);
  return (has_rgb(h) ? (n * 3 + 255) / 256 * 256 : 0) + (has_depth(h) ? (n * 2 + 255) / 256 * 256 : 0);
}

// Lays the two frame slots of h out from p (256-byte aligned).
static void place_slots(Attached& a, const gmm_handle* h, uint8_t* p) {
  const size_t n = static_cast<size_t>(h->npix), rgb = has_rgb(h) ? (n * 3 + 255) / 256 * 256 : 0;
  for (int k = 0; k < kFramesInFlight; ++k) {
    uint8_t* q = p + static_cast<size_t>(k) * frame_slot_bytes(h);
    a.d_rgb[k] = has_rgb(h) ? q : nullptr;
    a.d_depth[k] = has_depth(h) ? reinterpret_cast<uint16_t*>(q + rgb) : nullptr;
  }
}

constexpr int kCopyInStreams = 4;  // host->device copies spread over several DMA queues

struct Slot {
  hipEvent_t h2d_done[kCopyInStreams] = {};
  hipEvent_t compute_done = nullptr, done = nullptr;
  FrameArgs* h_table = nullptr;   // pinned: n FrameArgs then n+1 uint32 tile starts
  size_t h_cap = 0;               // bytes
  void* d_table = nullptr;        // device copy of the same
  size_t d_cap = 0;
  uint32_t* d_tile_map = nullptr;
  size_t map_cap = 0;             // entries
  uint64_t* d_masks = nullptr;    // every mask of the tick, back to back (device)
  uint64_t* h_masks = nullptr;    // its pinned host copy
  size_t mask_cap = 0;            // bytes
  struct Out {
    void* dst;
    size_t off, bytes;
  };
  std::vector<Out> outs;          // where each mask goes once the tick has completed
  uint64_t tick = 0;
  bool busy = false;
  std::vector<gmm_handle*> handles;
};

}  // namespace

struct gmm_exec {
  int device = 0;
  int M = -1, dtype = -1;
  int cu_count = 0;
  gmm_batch_tuning tuning{256, 1024, 8};
  hipStream_t s_in[kCopyInStreams] = {};
  hipStream_t s_compute = nullptr, s_out = nullptr;
  std::vector<Slot> slots;
  std::map<const gmm_handle*, Attached> attached;
  uint64_t next_tick = 1;
  // completion thread
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int> pending;                         // slot indices in launch order
  std::deque<std::pair<uint64_t, double>> done;    // (tick, completion time)
  bool stop = false;
  hipError_t thread_error = hipSuccess;
  std::thread worker;
};

static void completion_loop(gmm_exec* x) {
  (void)hipSetDevice(x->device);
  for (;;) {
    int slot = -1;
    {
      std::unique_lock<std::mutex> lk(x->mu);
      x->cv.wait(lk, [&] { return x->stop || !x->pending.empty(); });
      if (x->pending.empty()) return;  // stop requested and nothing left
      slot = x->pending.front();
    }
    Slot& s = x->slots[slot];
    hipError_t e = hipEventSynchronize(s.done);
    if (e == hipSuccess)
      for (const auto& o : s.outs) std::memcpy(o.dst, reinterpret_cast<const char*>(s.h_masks) + o.off, o.bytes);
    const double t = now_s();
    std::lock_guard<std::mutex> lk(x->mu);
    if (e != hipSuccess && x->thread_error == hipSuccess) x->thread_error = e;
    x->pending.pop_front();
    x->done.emplace_back(s.tick, t);
    for (auto* h : s.handles) {
      auto it = x->attached.find(h);
      if (it != x->attached.end()) it->second.in_flight--;
    }
    s.busy = false;
    x->cv.notify_all();
  }
}

static void destroy_exec(gmm_exec* x) {
  if (x->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(x->mu);
      x->stop = true;
    }
    x->cv.notify_all();
    x->worker.join();
  }
  for (auto& s : x->slots) {
    for (auto ev : s.h2d_done)
      if (ev) (void)hipEventDestroy(ev);
    if (s.compute_done) (void)hipEventDestroy(s.compute_done);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.h_table) (void)hipHostFree(s.h_table);
    if (s.d_table) (void)hipFree(s.d_table);
    if (s.d_tile_map) (void)hipFree(s.d_tile_map);
    if (s.d_masks) (void)hipFree(s.d_masks);
    if (s.h_masks) (void)hipHostFree(s.h_masks);
  }
  for (auto& kv : x->attached)
    if (kv.second.base) (void)hipFree(kv.second.base);
  for (auto st : x->s_in)
    if (st) (void)hipStreamDestroy(st);
  if (x->s_compute) (void)hipStreamDestroy(x->s_compute);
  if (x->s_out) (void)hipStreamDestroy(x->s_out);
  delete x;
}

static size_t mask_bytes(const gmm_handle* h) { return static_cast<size_t>((h->npix + 63) / 64) * 8; }

extern "C" {

double gmm_exec_now(void) { return now_s(); }

gmm_status gmm_exec_create(int32_t device, int32_t ring, gmm_exec** out) {
  if (!out) return fail(GMM_ERR_INVALID_ARG, "out is NULL");
  if (ring < 1 || ring > 64) return fail(GMM_ERR_INVALID_ARG, "ring must be in 1..64");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(GMM_ERR_INVALID_ARG, "device ordinal out of range");
  gmm_exec* x = new (std::nothrow) gmm_exec();
  if (!x) return fail(GMM_ERR_OUT_OF_MEMORY, "host allocation of the executor failed");
  x->device = device;
  DeviceGuard g(device);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e == hipSuccess) x->cu_count = prop.multiProcessorCount;
  // default-priority, non-blocking streams
  for (auto& st : x->s_in)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&x->s_compute, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&x->s_out, hipStreamNonBlocking);
  x->slots.resize(ring);
  for (auto& s : x->slots) {
    for (auto& ev : s.h2d_done)
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.compute_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    destroy_exec(x);
    return hip_fail(e, "executor set-up");
  }
  x->worker = std::thread(completion_loop, x);
  *out = x;
  return GMM_OK;
}

gmm_status gmm_exec_destroy(gmm_exec* x) {
  if (!x) return GMM_OK;
  DeviceGuard g(x->device);
  for (auto st : x->s_in) (void)hipStreamSynchronize(st);
  (void)hipStreamSynchronize(x->s_compute);
  (void)hipStreamSynchronize(x->s_out);
  destroy_exec(x);
  return GMM_OK;
}

gmm_status gmm_exec_set_tuning(gmm_exec* x, const gmm_batch_tuning* t) {
  if (!x || !t) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  if (t->block_threads != 256 && t->block_threads != 512)
    return fail(GMM_ERR_INVALID_ARG, "block_threads must be 256 or 512");
  if (t->tile_pixels < t->block_threads || t->tile_pixels % t->block_threads || t->tile_pixels > 64 * t->block_threads)
    return fail(GMM_ERR_INVALID_ARG, "tile_pixels must be a multiple of block_threads, at most 64x it");
  if (t->blocks_per_cu < 1 || t->blocks_per_cu > 32) return fail(GMM_ERR_INVALID_ARG, "blocks_per_cu must be in 1..32");
  std::lock_guard<std::mutex> lk(x->mu);
  x->tuning = *t;
  return GMM_OK;
}

gmm_status gmm_exec_attach(gmm_exec* x, gmm_handle* h, size_t* device_bytes) {
  if (!x || !h) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  if (h->cfg.device != x->device) return fail(GMM_ERR_INVALID_ARG, "handle lives on another device");
  if (is_augmented(h)) return fail(GMM_ERR_UNSUPPORTED, "augmented handles run one at a time");
  std::lock_guard<std::mutex> lk(x->mu);
  if (x->attached.count(h)) return fail(GMM_ERR_INVALID_ARG, "handle already attached");
  if (x->M >= 0 && (h->cfg.M != x->M || h->cfg.state_dtype != x->dtype))
    return fail(GMM_ERR_INVALID_ARG, "all streams of an executor need the same M and state dtype");
  const size_t slots = kFramesInFlight * frame_slot_bytes(h);
  DeviceGuard g(x->device);
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, slots);
  if (e != hipSuccess) return fail(GMM_ERR_OUT_OF_MEMORY, "device allocation of the stream's frame slots failed");
  Attached a;
  a.base = mem;
  place_slots(a, h, static_cast<uint8_t*>(mem));
  a.bytes = slots;
  x->attached[h] = a;
  x->M = h->cfg.M;
  x->dtype = h->cfg.state_dtype;
  if (device_bytes) *device_bytes = a.bytes;
  return GMM_OK;
}

gmm_status gmm_exec_detach(gmm_exec* x, gmm_handle* h) {
  if (!x || !h) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(x->mu);
  auto it = x->attached.find(h);
  if (it == x->attached.end()) return fail(GMM_ERR_INVALID_ARG, "handle not attached");
  x->cv.wait(lk, [&] { return it->second.in_flight == 0; });  // its last frame has completed
  void* base = it->second.base;
  x->attached.erase(it);
  lk.unlock();
  DeviceGuard g(x->device);
  if (base) (void)hipFree(base);
  return GMM_OK;
}

gmm_status gmm_exec_launch(gmm_exec* x, const gmm_exec_item* items, int32_t n, uint64_t* tick_id) {
  if (!x || !items || n <= 0) return fail(GMM_ERR_INVALID_ARG, "an executor tick needs at least one item");
  // validate before touching anything
  std::vector<Attached> att(n);
  {
    std::lock_guard<std::mutex> lk(x->mu);
    if (x->thread_error != hipSuccess) return hip_fail(x->thread_error, "earlier tick");
    for (int32_t i = 0; i < n; ++i) {
      const gmm_exec_item& it = items[i];
      auto f = it.handle ? x->attached.find(it.handle) : x->attached.end();
      if (f == x->attached.end()) return fail(GMM_ERR_INVALID_ARG, "item " + std::to_string(i) + ": handle not attached");
      if (f->second.in_flight >= kFramesInFlight)
        return fail(GMM_ERR_STATE, "item " + std::to_string(i) + ": stream already has two frames in flight");
      for (int32_t j = 0; j < i; ++j)
        if (items[j].handle == it.handle) return fail(GMM_ERR_INVALID_ARG, "a stream appears twice in one tick");
      const gmm_handle* h = it.handle;
      if (has_rgb(h) != (it.host_rgb != nullptr) || has_depth(h) != (it.host_depth != nullptr))
        return fail(GMM_ERR_INVALID_ARG, "item " + std::to_string(i) + ": frames must match the stream's modalities");
      if ((it.host_fg_rgb && !has_rgb(h)) || (it.host_fg_depth && !has_depth(h)))
        return fail(GMM_ERR_INVALID_ARG, "item " + std::to_string(i) + ": mask output for an absent modality");
      if (it.host_fused && !has_both(h))
        return fail(GMM_ERR_STATE, "item " + std::to_string(i) + ": fusion needs both modalities");
      att[i] = f->second;
    }
  }
  DeviceGuard g(x->device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the executor's device");
  const uint64_t tick = x->next_tick;
  const int si = static_cast<int>(tick % x->slots.size());
  Slot& s = x->slots[si];
  {  // back-pressure: the slot's previous tick must have completed
    std::unique_lock<std::mutex> lk(x->mu);
    x->cv.wait(lk, [&] { return !s.busy; });
  }
  gmm_batch_tuning tun;
  {
    std::lock_guard<std::mutex> lk(x->mu);
    tun = x->tuning;
  }
  const uint32_t tile_px = static_cast<uint32_t>(tun.tile_pixels);
  // work list: n descriptors followed by n+1 tile starts
  const size_t tab = static_cast<size_t>(n) * sizeof(FrameArgs);
  const size_t bytes = tab + (static_cast<size_t>(n) + 1) * sizeof(uint32_t);
  hipError_t e = hipSuccess;
  if (bytes > s.h_cap) {
    if (s.h_table) (void)hipHostFree(s.h_table);
    s.h_table = nullptr;
    s.h_cap = 0;
    e = hipHostMalloc(reinterpret_cast<void**>(&s.h_table), bytes * 2, hipHostMallocDefault);
    if (e != hipSuccess) return fail(GMM_ERR_OUT_OF_MEMORY, "pinned work-list allocation failed");
    s.h_cap = bytes * 2;
  }
  if (bytes > s.d_cap) {
    if (s.d_table) (void)hipFree(s.d_table);
    s.d_table = nullptr;
    s.d_cap = 0;
    e = hipMalloc(&s.d_table, bytes * 2);
    if (e != hipSuccess) return fail(GMM_ERR_OUT_OF_MEMORY, "device work-list allocation failed");
    s.d_cap = bytes * 2;
  }
  // masks of the tick: one region per requested mask, 256-byte aligned, in one device arena
  size_t mask_total = 0;
  std::vector<size_t> moff(static_cast<size_t>(n) * 3, SIZE_MAX);
  for (int32_t i = 0; i < n; ++i) {
    const size_t mb = (mask_bytes(items[i].handle) + 255) / 256 * 256;
    const gmm_handle* h = items[i].handle;
    // the kernel writes a stream's masks whenever the modality is present; keep room for all
    if (has_rgb(h)) moff[3 * i] = mask_total, mask_total += mb;
    if (has_depth(h)) moff[3 * i + 1] = mask_total, mask_total += mb;
    if (items[i].host_fused) moff[3 * i + 2] = mask_total, mask_total += mb;
  }
  if (mask_total > s.mask_cap) {
    if (s.d_masks) (void)hipFree(s.d_masks);
    if (s.h_masks) (void)hipHostFree(s.h_masks);
    s.d_masks = nullptr;
    s.h_masks = nullptr;
    s.mask_cap = 0;
    e = hipMalloc(reinterpret_cast<void**>(&s.d_masks), mask_total * 2);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s.h_masks), mask_total * 2, hipHostMallocDefault);
    if (e != hipSuccess) return fail(GMM_ERR_OUT_OF_MEMORY, "mask arena allocation failed");
    s.mask_cap = mask_total * 2;
  }
  s.outs.clear();
  uint32_t* h_first = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(s.h_table) + tab);
  uint64_t total_tiles = 0;
  bool measure = false;
  for (int32_t i = 0; i < n; ++i) {
    const gmm_exec_item& it = items[i];
    gmm_handle* h = it.handle;
    auto dm = [&](int k) { return moff[3 * i + k] == SIZE_MAX ? nullptr : s.d_masks + moff[3 * i + k] / 8; };
    const int k = static_cast<int>(att[i].frames % kFramesInFlight);
    s.h_table[i] = frame_args(h, att[i].d_rgb[k], 3 * static_cast<int64_t>(h->cfg.width), att[i].d_depth[k],
                              2 * static_cast<int64_t>(h->cfg.width), dm(0), dm(1), dm(2));
    measure = measure || s.h_table[i].wave_bytes != nullptr;
    const size_t mb = mask_bytes(h);
    if (it.host_fg_rgb) s.outs.push_back({it.host_fg_rgb, moff[3 * i], mb});
    if (it.host_fg_depth) s.outs.push_back({it.host_fg_depth, moff[3 * i + 1], mb});
    if (it.host_fused) s.outs.push_back({it.host_fused, moff[3 * i + 2], mb});
    h_first[i] = static_cast<uint32_t>(total_tiles);
    total_tiles += (static_cast<uint64_t>(h->npix) + tile_px - 1) / tile_px;
  }
  if (total_tiles >= (1ull << 31)) return fail(GMM_ERR_INVALID_ARG, "too many tiles in one tick");
  h_first[n] = static_cast<uint32_t>(total_tiles);
  if (total_tiles > s.map_cap) {
    if (s.d_tile_map) (void)hipFree(s.d_tile_map);
    s.d_tile_map = nullptr;
    s.map_cap = 0;
    e = hipMalloc(&s.d_tile_map, total_tiles * 2 * sizeof(uint32_t));
    if (e != hipSuccess) return fail(GMM_ERR_OUT_OF_MEMORY, "device tile-map allocation failed");
    s.map_cap = total_tiles * 2;
  }
  // copy-in: frames from host memory into the streams' device frame slots, each frame on the
  // least loaded of the copy-in streams (by bytes), so several DMA engines work at once. DMA
  // engines need no compute units, so the copies of one tick overlap the previous tick's kernel.
  // The slot a frame goes to was last read by the stream's frame before last, whose tick has
  // completed: a stream is accepted here only with at most one frame in flight.
  size_t queued[kCopyInStreams] = {};
  for (int32_t i = 0; i < n && e == hipSuccess; ++i) {
    const gmm_handle* h = items[i].handle;
    const size_t px = static_cast<size_t>(h->npix);
    const int k = static_cast<int>(att[i].frames % kFramesInFlight);
    int q = 0;
    for (int c = 1; c < kCopyInStreams; ++c)
      if (queued[c] < queued[q]) q = c;
    if (items[i].host_rgb) {
      e = hipMemcpyAsync(att[i].d_rgb[k], items[i].host_rgb, px * 3, hipMemcpyHostToDevice, x->s_in[q]);
      queued[q] += px * 3;
    }
    if (e == hipSuccess && items[i].host_depth) {
      e = hipMemcpyAsync(att[i].d_depth[k], items[i].host_depth, px * 2, hipMemcpyHostToDevice, x->s_in[q]);
      queued[q] += px * 2;
    }
  }
  for (int c = 0; c < kCopyInStreams && e == hipSuccess; ++c) e = hipEventRecord(s.h2d_done[c], x->s_in[c]);
  // compute: work list, tile map, one persistent launch over every item
  for (int c = 0; c < kCopyInStreams && e == hipSuccess; ++c) e = hipStreamWaitEvent(x->s_compute, s.h2d_done[c], 0);
  if (e == hipSuccess) e = hipMemcpyAsync(s.d_table, s.h_table, bytes, hipMemcpyHostToDevice, x->s_compute);
  const FrameArgs* d_tab = static_cast<const FrameArgs*>(s.d_table);
  const uint32_t* d_first = reinterpret_cast<const uint32_t*>(static_cast<const char*>(s.d_table) + tab);
  if (e == hipSuccess) {
    tile_map_kernel<<<dim3(static_cast<unsigned>((total_tiles + kBlock - 1) / kBlock)), dim3(kBlock), 0, x->s_compute>>>(
        d_first, static_cast<uint32_t>(n), s.d_tile_map);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const uint32_t want = static_cast<uint32_t>(tun.blocks_per_cu) * static_cast<uint32_t>(x->cu_count);
    const dim3 grid(std::max(1u, std::min(want, static_cast<uint32_t>(total_tiles))));
    e = launch_batch(x->M, x->dtype, tun.block_threads, grid, d_tab, s.d_tile_map, d_first,
                     static_cast<uint32_t>(total_tiles), tile_px, measure, x->s_compute);
  }
  if (e == hipSuccess) e = hipEventRecord(s.compute_done, x->s_compute);
  // copy-out: the whole mask arena in one copy; the completion thread scatters it
  if (e == hipSuccess) e = hipStreamWaitEvent(x->s_out, s.compute_done, 0);
  if (e == hipSuccess && !s.outs.empty())
    e = hipMemcpyAsync(s.h_masks, s.d_masks, mask_total, hipMemcpyDeviceToHost, x->s_out);
  if (e == hipSuccess) e = hipEventRecord(s.done, x->s_out);
  if (e != hipSuccess) return hip_fail(e, "executor tick");
  {
    std::lock_guard<std::mutex> lk(x->mu);
    s.tick = tick;
    s.busy = true;
    s.handles.clear();
    for (int32_t i = 0; i < n; ++i) {
      s.handles.push_back(items[i].handle);
      Attached& a = x->attached[items[i].handle];
      a.in_flight++;
      a.frames++;
      items[i].handle->last_stream = x->s_compute;
    }
    x->pending.push_back(si);
    x->next_tick++;
  }
  x->cv.notify_all();
  if (tick_id) *tick_id = tick;
  return GMM_OK;
}

gmm_status gmm_exec_stream_bytes(const gmm_config* cfg, size_t* bytes) {
  if (!cfg || !bytes) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  gmm_handle* h = nullptr;
  gmm_status st = new_handle(cfg, &h);
  if (st != GMM_OK) return st;
  if (is_augmented(h)) {
    delete h;
    return fail(GMM_ERR_UNSUPPORTED, "augmented handles run one at a time");
  }
  *bytes = (state_bytes(h) + 255) / 256 * 256 + kFramesInFlight * frame_slot_bytes(h);
  delete h;
  return GMM_OK;
}

gmm_status gmm_exec_create_stream(gmm_exec* x, const gmm_config* cfg, void* mem, size_t bytes, gmm_handle** out) {
  if (!x || !out || !mem) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(mem) % 256) return fail(GMM_ERR_INVALID_ARG, "mem must be 256-byte aligned");
  if (cfg && cfg->device != x->device) return fail(GMM_ERR_INVALID_ARG, "configuration names another device");
  size_t need = 0;
  gmm_status st = gmm_exec_stream_bytes(cfg, &need);
  if (st != GMM_OK) return st;
  if (bytes < need) return fail(GMM_ERR_INVALID_ARG, "mem is smaller than gmm_exec_stream_bytes");
  gmm_handle* h = nullptr;
  st = new_handle(cfg, &h);
  if (st != GMM_OK) return st;
  std::lock_guard<std::mutex> lk(x->mu);
  if (x->M >= 0 && (h->cfg.M != x->M || h->cfg.state_dtype != x->dtype)) {
    delete h;
    return fail(GMM_ERR_INVALID_ARG, "all streams of an executor need the same M and state dtype");
  }
  uint8_t* base = static_cast<uint8_t*>(mem);
  place_state(h, base);
  const size_t sb = (state_bytes(h) + 255) / 256 * 256;
  Attached a;
  a.base = nullptr;  // the caller's memory: never freed here
  place_slots(a, h, base + sb);
  a.bytes = need;
  DeviceGuard g(x->device);
  // initialised on the compute stream: ordered before any tick that uses the stream
  hipError_t e = init_state(h, x->s_compute);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "state initialisation");
  }
  h->last_stream = x->s_compute;
  x->attached[h] = a;
  x->M = h->cfg.M;
  x->dtype = h->cfg.state_dtype;
  *out = h;
  return GMM_OK;
}

gmm_status gmm_exec_destroy_stream(gmm_exec* x, gmm_handle* h) {
  if (!x || !h) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  if (h->owns_mem) return fail(GMM_ERR_INVALID_ARG, "not a stream created by gmm_exec_create_stream");
  std::unique_lock<std::mutex> lk(x->mu);
  auto it = x->attached.find(h);
  if (it == x->attached.end()) return fail(GMM_ERR_INVALID_ARG, "handle not attached");
  x->cv.wait(lk, [&] { return it->second.in_flight == 0; });  // its last frame has completed
  x->attached.erase(it);
  lk.unlock();
  delete h;
  return GMM_OK;
}

gmm_status gmm_exec_poll(gmm_exec* x, uint64_t* tick_ids, double* t_done, int32_t cap, int32_t* n_out) {
  if (!x || !n_out || cap < 0 || (cap > 0 && (!tick_ids || !t_done))) return fail(GMM_ERR_INVALID_ARG, "bad poll arguments");
  std::lock_guard<std::mutex> lk(x->mu);
  if (x->thread_error != hipSuccess) return hip_fail(x->thread_error, "tick execution");
  int32_t k = 0;
  while (k < cap && !x->done.empty()) {
    tick_ids[k] = x->done.front().first;
    t_done[k] = x->done.front().second;
    x->done.pop_front();
    ++k;
  }
  *n_out = k;
  return GMM_OK;
}

gmm_status gmm_exec_drain(gmm_exec* x) {
  if (!x) return fail(GMM_ERR_INVALID_ARG, "executor is NULL");
  std::unique_lock<std::mutex> lk(x->mu);
  x->cv.wait(lk, [&] { return x->pending.empty(); });
  if (x->thread_error != hipSuccess) return hip_fail(x->thread_error, "tick execution");
  return GMM_OK;
}

}  // extern "C"
