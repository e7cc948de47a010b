// Host-side internals shared by the ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "gmm.h"
#include "gmm_device.hpp"

namespace rgbd {

// Everything one frame-kernel launch needs for one stream.
struct FrameArgs {
  int64_t npix;
  uint32_t tiles64;        // 64-pixel tiles of the state layout (ceil(npix / 64))
  uint32_t pad0_;
  int32_t width;
  int32_t rgb_dense;       // rgb rows are contiguous (pitch == 3*width) and 4-byte aligned
  int32_t depth_dense;     // depth rows are contiguous (pitch == 2*width)
  const uint8_t* rgb;
  int64_t rgb_pitch;
  const uint16_t* depth;
  int64_t depth_pitch;
  void* st_rgb;            // colour state block: 5*M values per pixel (four-channel variant: 6*M), plus rank
                           // 1's key and one scale per tile in the fp32 form
  void* st_depth;          // depth state block: 3*M values per pixel (and the same extras)
  uint8_t* fstate;         // List 1 state bytes
  uint64_t* fg_rgb;
  uint64_t* fg_depth;
  uint64_t* fused;
  ModelConsts kc;          // colour constants
  ModelConsts kd;          // depth constants (the fields both modalities share equal kc's: depth_consts)
  int32_t mode;            // kModeRGB | kModeDepth | kModeFuse bits of this stream
  int32_t pad_;
  uint64_t* wave_bytes;    // optional: per-wave running total of state bytes moved (measurement)
};

enum FrameMode : int { kModeRGB = 1, kModeDepth = 2, kModeFuse = 4, kModeAug = 8 };

// Launchers (return hipSuccess or the launch error).
// `stream`: the kernel's rows and frames take the non-temporal cache policy (kStream), for a state
// too large to stay in the last-level cache between frames (streams_state).
hipError_t launch_frame(const FrameArgs& a, int M, int dtype, int mode, bool stream, hipStream_t s);
constexpr size_t kStreamStateBytes = size_t(128) << 20;  // half the 256 MB last-level cache
hipError_t launch_fuse(const uint64_t* fr, const uint64_t* fd, uint64_t* out, uint8_t* fstate,
                       int64_t npix, hipStream_t s);
hipError_t launch_init(void* st, int dtype, uint32_t tiles64, int M, int C, float var0, hipStream_t s);
// Rank 1's key of every pixel from the stored values (scaled form; a no-op otherwise).
hipError_t launch_rekey(void* st, int dtype, uint32_t tiles64, int M, int C, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);

bool frame_variant_compiled(int M, int dtype);
// `measure`: some descriptor of the table has a traffic record (wave_bytes); otherwise the kernel
// that never counts bytes runs.
hipError_t launch_batch(int M, int dtype, int block, dim3 grid, const FrameArgs* table, const uint32_t* map,
                        const uint32_t* first, uint32_t n_tiles, uint32_t tile_px, bool measure, hipStream_t s);

inline size_t dtype_size(int dtype) { return dtype == GMM_F32 ? 4 : 2; }

void set_error(const std::string& msg);
gmm_status fail(gmm_status st, const std::string& msg);
gmm_status hip_fail(hipError_t e, const char* what);

// Switches to a device for the duration of a call, restoring the caller's.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    ok_ = hipGetDevice(&prev_) == hipSuccess;
    if (ok_ && prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
    switched_ = ok_ && prev_ != dev;
  }
  ~DeviceGuard() {
    if (switched_) (void)hipSetDevice(prev_);
  }
  bool ok() const { return ok_; }

 private:
  int prev_ = 0;
  bool ok_ = false;
  bool switched_ = false;
};

}  // namespace rgbd

struct gmm_handle {  // the library's per-stream object (opaque in gmm.h)
  gmm_config cfg;
  int64_t npix = 0;
  uint32_t tiles64 = 0;     // 64-pixel tiles of the state layout
  size_t esize = 0;         // bytes per stored value
  size_t rgb_bytes = 0;     // colour block
  size_t depth_bytes = 0;   // depth block
  size_t fuse_bytes = 0;    // List 1 state bytes (padded)
  void* mem = nullptr;      // device state: [colour][depth][fusion]
  bool owns_mem = false;    // allocated by gmm_create (else provided by the caller)
  uint64_t* wave_bytes = nullptr;  // optional per-wave traffic record (gmm_set_traffic_record)
  void* st_rgb = nullptr;
  void* st_depth = nullptr;
  uint8_t* fstate = nullptr;
  hipStream_t last_stream = nullptr;
  rgbd::ModelConsts kc{}, kd{};
};

inline bool has_rgb(const gmm_handle* h) { return (h->cfg.modalities & GMM_RGB) != 0; }
inline bool has_depth(const gmm_handle* h) { return (h->cfg.modalities & GMM_DEPTH) != 0; }
inline bool has_both(const gmm_handle* h) { return has_rgb(h) && has_depth(h); }
// the four-channel (R, G, B, depth byte) variant: one mixture, no separate models, no fusion
inline bool is_augmented(const gmm_handle* h) { return h->cfg.variant == GMM_AUGMENTED; }
// the per-modality separate models of the method (colour block, depth block, List 1 state)
inline bool sep_rgb(const gmm_handle* h) { return has_rgb(h) && !is_augmented(h); }
inline bool sep_depth(const gmm_handle* h) { return has_depth(h) && !is_augmented(h); }
inline bool sep_both(const gmm_handle* h) { return has_both(h) && !is_augmented(h); }

namespace rgbd {
// Validation and kernel arguments of one stream's frame (shared by the plain and batched paths).
gmm_status check_frame_args(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch, const uint16_t* depth,
                            int64_t depth_pitch, uint64_t* fg_rgb, uint64_t* fg_depth);
FrameArgs frame_args(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch, const uint16_t* depth,
                     int64_t depth_pitch, uint64_t* fg_rgb, uint64_t* fg_depth, uint64_t* fused);
// A validated handle with its sizes and constants, no device memory yet.
gmm_status new_handle(const gmm_config* cfg, gmm_handle** out);
// Point the handle's state at `mem` (state_bytes(h) bytes, 256-byte aligned).
void place_state(gmm_handle* h, void* mem);
// Enqueue the initial (all components empty) state on `s`.
hipError_t init_state(gmm_handle* h, hipStream_t s);
size_t state_bytes(const gmm_handle* h);
// Whether a single-stream launch streams its state (at least kStreamStateBytes of it).
inline bool streams_state(const gmm_handle* h) { return state_bytes(h) >= kStreamStateBytes; }
}  // namespace rgbd
