// The per-pixel body shared by every frame kernel (one stream per launch, or a persistent
// launch over many streams): ingest, colour and/or depth mixture step, List 1 fusion, mask
// ballots. Keeping one body makes the plain and batched paths bit-identical by construction.
#pragma once

#include <hip/hip_runtime.h>

#include "gmm_device.hpp"
#include "gmm_internal.hpp"

namespace rgbd {

// Colour pixel p of the frame. When rows are dense and the whole wave is inside the frame, the
// wave's 192 interleaved bytes are fetched with 48 dword loads into the wave's LDS slice and
// de-interleaved from there; otherwise each lane reads its own three bytes.
__device__ __forceinline__ void load_rgb_pixel(const FrameArgs& a, uint32_t p, uint32_t wave_base,
                                               int lane, uint32_t* lds_wave, bool valid,
                                               float (&x)[3]) {
  const bool fast = a.rgb_dense && (wave_base + kWave <= a.npix);  // uniform over the wave
  if (fast) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.rgb + 3 * static_cast<uint64_t>(wave_base));
    if (lane < 48) lds_wave[lane] = src[lane];
    wave_lds_sync();
    const uint8_t* b = reinterpret_cast<const uint8_t*>(lds_wave) + 3 * lane;
    x[0] = b[0];
    x[1] = b[1];
    x[2] = b[2];
    wave_lds_sync();  // the slice is reused by the wave's next pixels
  } else if (valid) {
    const uint32_t y = p / static_cast<uint32_t>(a.width);
    const uint32_t xx = p - y * static_cast<uint32_t>(a.width);
    const uint8_t* b = a.rgb + static_cast<int64_t>(y) * a.rgb_pitch + 3 * xx;
    x[0] = b[0];
    x[1] = b[1];
    x[2] = b[2];
  } else {
    x[0] = x[1] = x[2] = 0.f;
  }
}

__device__ __forceinline__ float load_depth_pixel(const FrameArgs& a, uint32_t p) {
  if (a.depth_dense) return static_cast<float>(a.depth[p]);
  const uint32_t y = p / static_cast<uint32_t>(a.width);
  const uint32_t xx = p - y * static_cast<uint32_t>(a.width);
  const uint16_t* row = reinterpret_cast<const uint16_t*>(
      reinterpret_cast<const uint8_t*>(a.depth) + static_cast<int64_t>(y) * a.depth_pitch);
  return static_cast<float>(row[xx]);
}

// Pixel p of stream `a` (p may lie past the end: such lanes only take part in the ballots).
// `mode` must be uniform over the wave.
template <int M, typename S>
__device__ __forceinline__ void process_pixel(const FrameArgs& a, int mode, uint32_t p, int lane,
                                              uint32_t* lds_wave) {
  const uint32_t wave_base = p - lane;
  const bool valid = p < a.npix;
  bool fgc = false, fgd = false;
  if ((mode & kModeRGB) != 0) {
    float x[3];
    load_rgb_pixel(a, p, wave_base, lane, lds_wave, valid, x);
    if (valid) {
      Mix<M, 3> m;
      const StateBlock blk = make_block(a.st_rgb, a.tiles64, sizeof(S), 5 * M);
      load_mix<M, 3, S>(m, blk, p);
      fgc = mix_step<M, 3>(m, x, a.kc);
      store_mix<M, 3, S>(m, blk, p);
    }
    const uint64_t bits = __ballot(fgc);
    if (lane == 0 && valid) a.fg_rgb[wave_base >> 6] = bits;
  }
  if ((mode & kModeDepth) != 0) {
    if (valid) {
      const float xd = load_depth_pixel(a, p);
      if (!(a.kd.hole_skip && xd == 0.f)) {
        Mix<M, 1> m;
        const StateBlock blk = make_block(a.st_depth, a.tiles64, sizeof(S), 3 * M);
        load_mix<M, 1, S>(m, blk, p);
        const float x1[1] = {xd};
        fgd = mix_step<M, 1>(m, x1, a.kd);
        store_mix<M, 1, S>(m, blk, p);
      }
    }
    const uint64_t bits = __ballot(fgd);
    if (lane == 0 && valid) a.fg_depth[wave_base >> 6] = bits;
  }
  if ((mode & kModeFuse) != 0) {
    bool fgf = false;
    if (valid) {
      const uint32_t st = fuse_transition(a.fstate[p], fgc, fgd);
      a.fstate[p] = static_cast<uint8_t>(st);
      fgf = (st >> 3) & 1u;
    }
    const uint64_t bits = __ballot(fgf);
    if (lane == 0 && valid) a.fused[wave_base >> 6] = bits;
  }
}

}  // namespace rgbd
