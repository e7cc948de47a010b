// The C ABI (include/gmm.h): validation, state ownership, dispatch, state I/O.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gmm.h"
#include "gmm_internal.hpp"

namespace rgbd {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

gmm_status fail(gmm_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

gmm_status hip_fail(hipError_t e, const char* what) {
  return fail(GMM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Round a double to a binary format with `p` significant bits and smallest normal exponent
// `emin`, to nearest with ties to even; returns the rounded value as a double.
static double round_to_format(double v, int p, int emin, double maxv) {
  if (v == 0.0 || !std::isfinite(v)) return v;
  int e = 0;
  (void)std::frexp(v, &e);  // |v| in [2^(e-1), 2^e)
  const int qexp = std::max(e - p, emin - p + 1);
  double r = std::ldexp(std::nearbyint(std::ldexp(v, -qexp)), qexp);
  if (std::fabs(r) > maxv) r = std::copysign(INFINITY, r);
  return r;
}

static uint16_t half_bits_exact(double r) {  // r exactly representable as binary16
  uint16_t sign = std::signbit(r) ? 0x8000u : 0u;
  double a = std::fabs(r);
  if (a == 0.0) return sign;
  if (std::isinf(a)) return sign | 0x7C00u;
  int e = std::ilogb(a);
  if (e >= -14) {
    const uint16_t mant = static_cast<uint16_t>(std::ldexp(a, -e) * 1024.0 - 1024.0);
    return sign | static_cast<uint16_t>((e + 15) << 10) | mant;
  }
  return sign | static_cast<uint16_t>(std::ldexp(a, 24));
}

static double half_value(uint16_t h) {
  const double s = (h & 0x8000u) ? -1.0 : 1.0;
  const int ex = (h >> 10) & 0x1F;
  const int m = h & 0x3FF;
  if (ex == 0) return s * std::ldexp(static_cast<double>(m), -24);
  if (ex == 31) return m ? NAN : s * INFINITY;
  return s * std::ldexp(1024.0 + m, ex - 25);
}

static void pack_values(const double* in, void* out, size_t n, int dtype) {
  if (dtype == GMM_F32) {
    float* o = static_cast<float*>(out);
    for (size_t i = 0; i < n; ++i) o[i] = static_cast<float>(in[i]);  // round to nearest even
  } else if (dtype == GMM_F16) {
    uint16_t* o = static_cast<uint16_t*>(out);
    for (size_t i = 0; i < n; ++i) o[i] = half_bits_exact(round_to_format(in[i], 11, -14, 65504.0));
  } else {
    uint16_t* o = static_cast<uint16_t*>(out);
    for (size_t i = 0; i < n; ++i) {
      const float f = static_cast<float>(round_to_format(in[i], 8, -126, 3.3895313892515355e38));
      uint32_t u;
      std::memcpy(&u, &f, 4);
      o[i] = static_cast<uint16_t>(u >> 16);
    }
  }
}

static void unpack_values(const void* in, double* out, size_t n, int dtype) {
  if (dtype == GMM_F32) {
    const float* s = static_cast<const float*>(in);
    for (size_t i = 0; i < n; ++i) out[i] = s[i];
  } else if (dtype == GMM_F16) {
    const uint16_t* s = static_cast<const uint16_t*>(in);
    for (size_t i = 0; i < n; ++i) out[i] = half_value(s[i]);
  } else {
    const uint16_t* s = static_cast<const uint16_t*>(in);
    for (size_t i = 0; i < n; ++i) {
      const uint32_t u = static_cast<uint32_t>(s[i]) << 16;
      float f;
      std::memcpy(&f, &u, 4);
      out[i] = f;
    }
  }
}

}  // namespace rgbd

using namespace rgbd;


static gmm_status validate_config(const gmm_config* c) {
  if (!c) return fail(GMM_ERR_INVALID_ARG, "config is NULL");
  if (c->width <= 0 || c->height <= 0) return fail(GMM_ERR_INVALID_ARG, "width and height must be > 0");
  if (static_cast<int64_t>(c->width) * c->height >= (int64_t(1) << 29))
    return fail(GMM_ERR_INVALID_ARG, "width*height must be < 2^29");
  if (c->modalities != GMM_RGB && c->modalities != GMM_DEPTH && c->modalities != (GMM_RGB | GMM_DEPTH))
    return fail(GMM_ERR_INVALID_ARG, "modalities must be GMM_RGB, GMM_DEPTH or both");
  if (c->M < 1 || c->M > 5) return fail(GMM_ERR_INVALID_ARG, "M must be in 1..5");
  if (!(c->alpha > 0.f && c->alpha <= 1.f)) return fail(GMM_ERR_INVALID_ARG, "alpha must be in (0, 1]");
  if (!(c->k > 0.f) || !std::isfinite(c->k)) return fail(GMM_ERR_INVALID_ARG, "k must be > 0");
  if (!(c->T > 0.f && c->T < 1.f)) return fail(GMM_ERR_INVALID_ARG, "T must be in (0, 1)");
  for (int i = 0; i < 2; ++i) {
    if (!(c->sigma0[i] > 0.f) || !std::isfinite(c->sigma0[i]))
      return fail(GMM_ERR_INVALID_ARG, "sigma0 must be > 0");
    if (!(c->var_min[i] > 0.f && c->var_min[i] <= c->sigma0[i] * c->sigma0[i]))
      return fail(GMM_ERR_INVALID_ARG, "var_min must be in (0, sigma0^2]");
  }
  if (!(c->w_init > 0.f && c->w_init <= 1.f)) return fail(GMM_ERR_INVALID_ARG, "w_init must be in (0, 1]");
  if (c->hole_policy != GMM_HOLE_SKIP && c->hole_policy != GMM_HOLE_AS_VALUE)
    return fail(GMM_ERR_INVALID_ARG, "hole_policy must be GMM_HOLE_SKIP or GMM_HOLE_AS_VALUE");
  if (c->state_dtype != GMM_F32 && c->state_dtype != GMM_F16 && c->state_dtype != GMM_BF16)
    return fail(GMM_ERR_INVALID_ARG, "state_dtype must be GMM_F32, GMM_F16 or GMM_BF16");
  if (c->device < 0) return fail(GMM_ERR_INVALID_ARG, "device must be >= 0");
  if (c->variant != GMM_SEPARATE && c->variant != GMM_AUGMENTED)
    return fail(GMM_ERR_INVALID_ARG, "variant must be GMM_SEPARATE or GMM_AUGMENTED");
  if (c->variant == GMM_AUGMENTED && c->modalities != (GMM_RGB | GMM_DEPTH))
    return fail(GMM_ERR_INVALID_ARG, "the augmented variant needs both modalities");
  if (c->rho_mode != GMM_RHO_ALPHA && c->rho_mode != GMM_RHO_DENSITY)
    return fail(GMM_ERR_INVALID_ARG, "rho_mode must be GMM_RHO_ALPHA or GMM_RHO_DENSITY");
  if (!frame_variant_compiled(c->M, c->state_dtype))
    return fail(GMM_ERR_UNSUPPORTED, "this (M, state dtype) is not compiled");
  return GMM_OK;
}

// Constants of one mixture over C channels; `mod` picks sigma0 / var_min (0 colour, 1 depth). Only
// var0, var_min, hole_skip and rho_scale depend on the modality: the kernels read every other field
// of a handle's depth constants from its colour constants (depth_consts).
static ModelConsts make_consts(const gmm_config& c, int mod, int C, bool hole_skip) {
  ModelConsts k{};
  k.alpha = c.alpha;
  k.oma = 1.0f - c.alpha;
  k.k2 = c.k * c.k;
  k.T = c.T;
  k.var0 = c.sigma0[mod] * c.sigma0[mod];
  k.var_min = c.var_min[mod];
  k.w_init = c.w_init;
  k.hole_skip = hole_skip ? 1 : 0;
  k.rho_density = c.rho_mode == GMM_RHO_DENSITY ? 1 : 0;
  k.rho_scale = static_cast<float>(static_cast<double>(c.alpha) * std::pow(2.0 * M_PI, -0.5 * C));
  // (1 / (1 - alpha))^(1, 2, 4, 8), each from the previous in fp32 (hole_factor)
  k.dk[0] = 1.0f / k.oma;
  k.dk[1] = k.dk[0] * k.dk[0];
  k.dk[2] = k.dk[1] * k.dk[1];
  k.dk[3] = k.dk[2] * k.dk[2];
  return k;
}

extern "C" {

int32_t gmm_version(void) { return 10000; }

const char* gmm_last_error(void) { return g_last_error.c_str(); }

gmm_status gmm_config_default(gmm_config* cfg, int32_t width, int32_t height, int32_t modalities,
                              int32_t M) {
  if (!cfg) return fail(GMM_ERR_INVALID_ARG, "config is NULL");
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->width = width;
  cfg->height = height;
  cfg->modalities = modalities;
  cfg->M = M;
  cfg->alpha = 0.01f;
  cfg->k = 2.5f;
  cfg->T = 0.7f;
  cfg->sigma0[0] = 30.f;
  cfg->sigma0[1] = 50.f;
  cfg->var_min[0] = 9.f;
  cfg->var_min[1] = 25.f;
  cfg->w_init = 0.01f;
  cfg->hole_policy = GMM_HOLE_SKIP;
  cfg->state_dtype = GMM_F32;
  cfg->device = 0;
  cfg->variant = GMM_SEPARATE;
  cfg->rho_mode = GMM_RHO_ALPHA;
  return GMM_OK;
}

}  // extern "C"

// Handle sizes, constants and pointers for `cfg` with its state at `mem` (not allocated here).
gmm_status rgbd::new_handle(const gmm_config* cfg, gmm_handle** out) {
  gmm_status st = validate_config(cfg);
  if (st != GMM_OK) return st;
  gmm_handle* h = new (std::nothrow) gmm_handle();
  if (!h) return fail(GMM_ERR_OUT_OF_MEMORY, "host allocation of the handle failed");
  h->cfg = *cfg;
  h->npix = static_cast<int64_t>(cfg->width) * cfg->height;
  h->tiles64 = static_cast<uint32_t>((h->npix + kWave - 1) / kWave);
  h->esize = dtype_size(cfg->state_dtype);
  const uint32_t M = static_cast<uint32_t>(cfg->M), es = static_cast<uint32_t>(h->esize);
  const size_t tiles = h->tiles64;
  // each block rounded up to 256 bytes, so that the next one starts aligned
  h->rgb_bytes = is_augmented(h) ? round_up(tiles * tile_layout(M, 4, es).bytes, 256)
                                 : (has_rgb(h) ? round_up(tiles * tile_layout(M, 3, es).bytes, 256) : 0);
  h->depth_bytes = sep_depth(h) ? round_up(tiles * tile_layout(M, 1, es).bytes, 256) : 0;
  // one flags byte per pixel for a handle with a depth model: its List 1 state (two modalities)
  // and its hole count (fp32 state)
  h->fuse_bytes = sep_depth(h) ? static_cast<size_t>(round_up(h->npix, 256)) : 0;
  // below 2 GiB: the kernels address a block with 32-bit offsets and use offset 2^31 for "no access"
  if (std::max(h->rgb_bytes, h->depth_bytes) >= 0x80000000ull) {
    delete h;
    return fail(GMM_ERR_INVALID_ARG, "one modality's state must stay below 2 GiB (too many pixels for this M)");
  }
  if (is_augmented(h)) {
    h->kc = make_consts(*cfg, 0, 4, cfg->hole_policy == GMM_HOLE_SKIP);
    h->kd = h->kc;
  } else {
    h->kc = make_consts(*cfg, 0, 3, false);
    h->kd = make_consts(*cfg, 1, 1, cfg->hole_policy == GMM_HOLE_SKIP);
  }
  *out = h;
  return GMM_OK;
}

void rgbd::place_state(gmm_handle* h, void* mem) {
  h->mem = mem;
  uint8_t* base = static_cast<uint8_t*>(mem);
  h->st_rgb = has_rgb(h) ? base : nullptr;
  h->st_depth = sep_depth(h) ? base + h->rgb_bytes : nullptr;
  h->fstate = sep_depth(h) ? base + h->rgb_bytes + h->depth_bytes : nullptr;
}

hipError_t rgbd::init_state(gmm_handle* h, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (has_rgb(h))
    e = launch_init(h->st_rgb, h->cfg.state_dtype, h->tiles64, h->cfg.M, is_augmented(h) ? 4 : 3, h->kc.var0, s);
  if (e == hipSuccess && sep_depth(h))
    e = launch_init(h->st_depth, h->cfg.state_dtype, h->tiles64, h->cfg.M, 1, h->kd.var0, s);
  if (e == hipSuccess && sep_depth(h)) e = launch_fill_u8(h->fstate, kFuseInit, h->fuse_bytes, s);
  return e;
}

size_t rgbd::state_bytes(const gmm_handle* h) { return h->rgb_bytes + h->depth_bytes + h->fuse_bytes; }

extern "C" {

gmm_status gmm_create(const gmm_config* cfg, gmm_handle** out) {
  if (!out) return fail(GMM_ERR_INVALID_ARG, "out is NULL");
  gmm_handle* h = nullptr;
  gmm_status st = new_handle(cfg, &h);
  if (st != GMM_OK) return st;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || cfg->device >= ndev) {
    delete h;
    return e != hipSuccess ? hip_fail(e, "hipGetDeviceCount") : fail(GMM_ERR_INVALID_ARG, "device ordinal out of range");
  }
  DeviceGuard g(cfg->device);
  if (!g.ok()) {
    delete h;
    return fail(GMM_ERR_DEVICE, "cannot select the configured device");
  }
  void* mem = nullptr;
  e = hipMalloc(&mem, state_bytes(h));
  if (e != hipSuccess) {
    delete h;
    return fail(GMM_ERR_OUT_OF_MEMORY, std::string("hipMalloc of the state failed: ") + hipGetErrorString(e));
  }
  place_state(h, mem);
  h->owns_mem = true;
  e = init_state(h, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    (void)hipFree(h->mem);
    delete h;
    return hip_fail(e, "state initialisation");
  }
  *out = h;
  return GMM_OK;
}

gmm_status gmm_destroy(gmm_handle* h) {
  if (!h) return GMM_OK;
  gmm_status st = GMM_OK;
  if (h->owns_mem) {
    DeviceGuard g(h->cfg.device);
    hipError_t e = hipStreamSynchronize(h->last_stream);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize in destroy");
    e = hipFree(h->mem);
    if (e != hipSuccess && st == GMM_OK) st = hip_fail(e, "hipFree");
  }
  delete h;
  return st;
}

gmm_status gmm_set_traffic_record(gmm_handle* h, uint64_t* wave_bytes) {
  if (!h) return fail(GMM_ERR_INVALID_ARG, "handle is NULL");
  if (reinterpret_cast<uintptr_t>(wave_bytes) % 8) return fail(GMM_ERR_INVALID_ARG, "wave_bytes not 8-byte aligned");
  h->wave_bytes = wave_bytes;
  return GMM_OK;
}

gmm_status gmm_state_bytes(const gmm_handle* h, size_t* device_bytes) {
  if (!h || !device_bytes) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  *device_bytes = h->rgb_bytes + h->depth_bytes + h->fuse_bytes;
  return GMM_OK;
}

gmm_status gmm_state_size(const gmm_handle* h, size_t* n_doubles) {
  if (!h || !n_doubles) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  const size_t n = static_cast<size_t>(h->npix), M = static_cast<size_t>(h->cfg.M);
  *n_doubles = is_augmented(h) ? 6 * M * n
                               : (has_rgb(h) ? 5 * M * n : 0) + (has_depth(h) ? 3 * M * n : 0) + (has_both(h) ? 2 * n : 0);
  return GMM_OK;
}

// Raw device copies of the state (the device layout, gmm_state_bytes bytes), ordered on `stream`.
static gmm_status copy_state_raw(gmm_handle* h, void* dst, const void* src, void* stream, const char* what) {
  DeviceGuard g(h->cfg.device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the handle's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(dst, src, state_bytes(h), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, what);
  h->last_stream = s;
  return GMM_OK;
}

gmm_status gmm_state_save(gmm_handle* h, void* device_dst, void* stream) {
  if (!h || !device_dst) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  return copy_state_raw(h, device_dst, h->mem, stream, "state save");
}

gmm_status gmm_state_restore(gmm_handle* h, const void* device_src, void* stream) {
  if (!h || !device_src) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  return copy_state_raw(h, h->mem, device_src, stream, "state restore");
}

}  // extern "C"

gmm_status rgbd::check_frame_args(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch,
                                   const uint16_t* depth, int64_t depth_pitch, uint64_t* fg_rgb,
                                   uint64_t* fg_depth) {
  if (!h) return fail(GMM_ERR_INVALID_ARG, "handle is NULL");
  if (is_augmented(h)) return fail(GMM_ERR_STATE, "an augmented handle runs through gmm_apply_frame_augmented");
  const gmm_config& c = h->cfg;
  if (has_rgb(h)) {
    if (!rgb || !fg_rgb) return fail(GMM_ERR_INVALID_ARG, "colour handle needs rgb and fg_rgb");
    if (rgb_pitch < 3 * static_cast<int64_t>(c.width)) return fail(GMM_ERR_INVALID_ARG, "rgb pitch < 3*width");
    if (reinterpret_cast<uintptr_t>(fg_rgb) % 8) return fail(GMM_ERR_INVALID_ARG, "fg_rgb not 8-byte aligned");
  } else if (rgb || fg_rgb) {
    return fail(GMM_ERR_INVALID_ARG, "rgb and fg_rgb must be NULL without the colour modality");
  }
  if (has_depth(h)) {
    if (!depth || !fg_depth) return fail(GMM_ERR_INVALID_ARG, "depth handle needs depth and fg_depth");
    if (depth_pitch < 2 * static_cast<int64_t>(c.width) || depth_pitch % 2)
      return fail(GMM_ERR_INVALID_ARG, "depth pitch must be even and >= 2*width");
    if (reinterpret_cast<uintptr_t>(depth) % 2) return fail(GMM_ERR_INVALID_ARG, "depth not 2-byte aligned");
    if (reinterpret_cast<uintptr_t>(fg_depth) % 8)
      return fail(GMM_ERR_INVALID_ARG, "fg_depth not 8-byte aligned");
  } else if (depth || fg_depth) {
    return fail(GMM_ERR_INVALID_ARG, "depth and fg_depth must be NULL without the depth modality");
  }
  return GMM_OK;
}

FrameArgs rgbd::frame_args(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch,
                            const uint16_t* depth, int64_t depth_pitch, uint64_t* fg_rgb,
                            uint64_t* fg_depth, uint64_t* fused) {
  FrameArgs a{};
  a.npix = h->npix;
  a.tiles64 = h->tiles64;
  a.width = h->cfg.width;
  a.rgb = rgb;
  a.rgb_pitch = rgb_pitch;
  a.rgb_dense = rgb && rgb_pitch == 3 * static_cast<int64_t>(h->cfg.width) &&
                reinterpret_cast<uintptr_t>(rgb) % 4 == 0;
  a.depth = depth;
  a.depth_pitch = depth_pitch;
  a.depth_dense = depth && depth_pitch == 2 * static_cast<int64_t>(h->cfg.width);
  a.st_rgb = h->st_rgb;
  a.st_depth = h->st_depth;
  a.fstate = h->fstate;
  a.fg_rgb = fg_rgb;
  a.fg_depth = fg_depth;
  a.fused = fused;
  a.kc = h->kc;
  a.kd = h->kd;
  a.mode = is_augmented(h) ? kModeAug
                           : (has_rgb(h) ? kModeRGB : 0) | (has_depth(h) ? kModeDepth : 0) | (fused ? kModeFuse : 0);
  a.wave_bytes = h->wave_bytes;
  return a;
}

extern "C" {

gmm_status gmm_apply_frame(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch_bytes,
                           const uint16_t* depth, int64_t depth_pitch_bytes, uint64_t* fg_rgb,
                           uint64_t* fg_depth, void* stream) {
  gmm_status st = check_frame_args(h, rgb, rgb_pitch_bytes, depth, depth_pitch_bytes, fg_rgb, fg_depth);
  if (st != GMM_OK) return st;
  DeviceGuard g(h->cfg.device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the handle's device");
  const FrameArgs a = frame_args(h, rgb, rgb_pitch_bytes, depth, depth_pitch_bytes, fg_rgb, fg_depth, nullptr);
  const int mode = (has_rgb(h) ? kModeRGB : 0) | (has_depth(h) ? kModeDepth : 0);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_frame(a, h->cfg.M, h->cfg.state_dtype, mode, streams_state(h), s);
  if (e != hipSuccess) return hip_fail(e, "frame kernel launch");
  h->last_stream = s;
  return GMM_OK;
}

gmm_status gmm_fuse(gmm_handle* h, const uint64_t* fg_rgb, const uint64_t* fg_depth, uint64_t* fused,
                    void* stream) {
  if (!h) return fail(GMM_ERR_INVALID_ARG, "handle is NULL");
  if (!sep_both(h)) return fail(GMM_ERR_STATE, "fusion needs a handle with both separate modalities");
  if (!fg_rgb || !fg_depth || !fused) return fail(GMM_ERR_INVALID_ARG, "NULL mask");
  if ((reinterpret_cast<uintptr_t>(fg_rgb) | reinterpret_cast<uintptr_t>(fg_depth) |
       reinterpret_cast<uintptr_t>(fused)) % 8)
    return fail(GMM_ERR_INVALID_ARG, "masks must be 8-byte aligned");
  DeviceGuard g(h->cfg.device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the handle's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_fuse(fg_rgb, fg_depth, fused, h->fstate, h->npix, s);
  if (e != hipSuccess) return hip_fail(e, "fuse kernel launch");
  h->last_stream = s;
  return GMM_OK;
}

gmm_status gmm_apply_frame_fused(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch_bytes,
                                 const uint16_t* depth, int64_t depth_pitch_bytes,
                                 uint64_t* fg_rgb, uint64_t* fg_depth, uint64_t* fused,
                                 void* stream) {
  if (!h) return fail(GMM_ERR_INVALID_ARG, "handle is NULL");
  if (!sep_both(h)) return fail(GMM_ERR_STATE, "fusion needs a handle with both separate modalities");
  gmm_status st = check_frame_args(h, rgb, rgb_pitch_bytes, depth, depth_pitch_bytes, fg_rgb, fg_depth);
  if (st != GMM_OK) return st;
  if (!fused || reinterpret_cast<uintptr_t>(fused) % 8)
    return fail(GMM_ERR_INVALID_ARG, "fused must be a non-NULL 8-byte aligned mask");
  DeviceGuard g(h->cfg.device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the handle's device");
  const FrameArgs a = frame_args(h, rgb, rgb_pitch_bytes, depth, depth_pitch_bytes, fg_rgb, fg_depth, fused);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_frame(a, h->cfg.M, h->cfg.state_dtype, kModeRGB | kModeDepth | kModeFuse, streams_state(h), s);
  if (e != hipSuccess) return hip_fail(e, "fused frame kernel launch");
  h->last_stream = s;
  return GMM_OK;
}

gmm_status gmm_apply_frame_augmented(gmm_handle* h, const uint8_t* rgb, int64_t rgb_pitch_bytes,
                                     const uint16_t* depth, int64_t depth_pitch_bytes, uint64_t* fg,
                                     void* stream) {
  if (!h) return fail(GMM_ERR_INVALID_ARG, "handle is NULL");
  if (!is_augmented(h)) return fail(GMM_ERR_STATE, "not a GMM_AUGMENTED handle");
  if (!rgb || !depth || !fg) return fail(GMM_ERR_INVALID_ARG, "rgb, depth and fg are required");
  const int64_t w = h->cfg.width;
  if (rgb_pitch_bytes < 3 * w) return fail(GMM_ERR_INVALID_ARG, "rgb pitch < 3*width");
  if (depth_pitch_bytes < 2 * w || depth_pitch_bytes % 2)
    return fail(GMM_ERR_INVALID_ARG, "depth pitch must be even and >= 2*width");
  if (reinterpret_cast<uintptr_t>(depth) % 2) return fail(GMM_ERR_INVALID_ARG, "depth not 2-byte aligned");
  if (reinterpret_cast<uintptr_t>(fg) % 8) return fail(GMM_ERR_INVALID_ARG, "fg not 8-byte aligned");
  DeviceGuard g(h->cfg.device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the handle's device");
  const FrameArgs a = frame_args(h, rgb, rgb_pitch_bytes, depth, depth_pitch_bytes, fg, nullptr, nullptr);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_frame(a, h->cfg.M, h->cfg.state_dtype, kModeAug, streams_state(h), s);
  if (e != hipSuccess) return hip_fail(e, "augmented frame kernel launch");
  h->last_stream = s;
  return GMM_OK;
}

gmm_status gmm_read_state(gmm_handle* h, double* host_out, void* stream) {
  if (!h || !host_out) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  DeviceGuard g(h->cfg.device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the handle's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t total = h->rgb_bytes + h->depth_bytes + h->fuse_bytes;
  std::vector<uint8_t> raw;
  try {
    raw.resize(total);
  } catch (...) {
    return fail(GMM_ERR_OUT_OF_MEMORY, "host staging buffer");
  }
  hipError_t e = hipMemcpyAsync(raw.data(), h->mem, total, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "state copy to host");
  const size_t n = static_cast<size_t>(h->npix), M = static_cast<size_t>(h->cfg.M);
  double* o = host_out;
  size_t off = 0;
  for (int blk = 0; blk < 2; ++blk) {
    const bool present = blk == 0 ? has_rgb(h) : sep_depth(h);
    if (!present) continue;
    const size_t P = blk == 0 ? (is_augmented(h) ? 6 : 5) : 3;
    const uint32_t C = static_cast<uint32_t>(P - 2);
    const uint32_t es = static_cast<uint32_t>(h->esize);
    // scaled weights: the weight is the pixel's effective scale (the tile's scale times the
    // pixel's hole factor, one fp32 product as the kernels form it) times the scaled weight (a
    // product of two floats, exact in double)
    const uint8_t* flags = sep_depth(h) ? raw.data() + h->rgb_bytes + h->depth_bytes : nullptr;
    const rgbd::ModelConsts& kcon = blk == 0 ? h->kc : h->kd;
    std::vector<double> scale;
    if (scaled_weights(es)) {
      try {
        scale.resize(h->tiles64);
      } catch (...) {
        return fail(GMM_ERR_OUT_OF_MEMORY, "host staging buffer");
      }
      for (size_t t = 0; t < h->tiles64; ++t)
        unpack_values(raw.data() + off + state_scale_offset(t, h->tiles64, static_cast<uint32_t>(M), C, es),
                      &scale[t], 1, h->cfg.state_dtype);
    }
    // two-plane device layout -> canonical [param][rank][pixel]
    for (size_t k = 0; k < P * M; ++k) {
      const uint32_t param = static_cast<uint32_t>(k / M);
      const uint32_t v = value_index(param, static_cast<uint32_t>(k % M), static_cast<uint32_t>(M), C, es);
      for (size_t i = 0; i < n; ++i) {
        const size_t at = off + state_value_offset(v, i, h->tiles64, static_cast<uint32_t>(M), C, es);
        unpack_values(raw.data() + at, o + i, 1, h->cfg.state_dtype);
        if (param == C + 1 && !scale.empty()) {
          float gi = static_cast<float>(scale[i / kWave]);
          if (blk == 1 && flags) gi = gi * hole_factor(flags[i] >> kHoleShift, kcon.dk);
          o[i] *= static_cast<double>(gi);
        }
      }
      o += n;
    }
    off += blk == 0 ? h->rgb_bytes : h->depth_bytes;
  }
  if (sep_both(h)) {
    const uint8_t* f = raw.data() + off;
    for (size_t i = 0; i < n; ++i) o[i] = static_cast<double>((f[i] >> 3) & 1u);
    o += n;
    for (size_t i = 0; i < n; ++i) o[i] = static_cast<double>(static_cast<int>(f[i] & 7u) - 3);
  }
  return GMM_OK;
}

gmm_status gmm_write_state(gmm_handle* h, const double* host_in, void* stream) {
  if (!h || !host_in) return fail(GMM_ERR_INVALID_ARG, "NULL argument");
  const size_t n = static_cast<size_t>(h->npix), M = static_cast<size_t>(h->cfg.M);
  const size_t total = h->rgb_bytes + h->depth_bytes + h->fuse_bytes;
  std::vector<uint8_t> raw;
  try {
    raw.assign(total, 0);
  } catch (...) {
    return fail(GMM_ERR_OUT_OF_MEMORY, "host staging buffer");
  }
  const double* in = host_in;
  size_t off = 0;
  for (int blk = 0; blk < 2; ++blk) {
    const bool present = blk == 0 ? has_rgb(h) : sep_depth(h);
    if (!present) continue;
    const size_t P = blk == 0 ? (is_augmented(h) ? 6 : 5) : 3;
    const uint32_t C = static_cast<uint32_t>(P - 2);
    const uint32_t es = static_cast<uint32_t>(h->esize);
    // scaled weights are written with scale 1 (rank 1's key is computed on the device below)
    if (scaled_weights(es)) {
      const double one = 1.0;
      for (size_t t = 0; t < h->tiles64; ++t)
        pack_values(&one, raw.data() + off + state_scale_offset(t, h->tiles64, static_cast<uint32_t>(M), C, es), 1,
                    h->cfg.state_dtype);
    }
    // canonical [param][rank][pixel] -> two-plane device layout
    for (size_t k = 0; k < P * M; ++k) {
      const uint32_t v = value_index(static_cast<uint32_t>(k / M), static_cast<uint32_t>(k % M),
                                     static_cast<uint32_t>(M), C, es);
      for (size_t i = 0; i < n; ++i) {
        const size_t at = off + state_value_offset(v, i, h->tiles64, static_cast<uint32_t>(M), C, es);
        pack_values(in + i, raw.data() + at, 1, h->cfg.state_dtype);
      }
      in += n;
    }
    off += blk == 0 ? h->rgb_bytes : h->depth_bytes;
  }
  if (sep_both(h)) {
    uint8_t* f = raw.data() + off;
    for (size_t i = 0; i < n; ++i) {
      const double I = in[i], c = in[n + i];
      if (!(I == 0.0 || I == 1.0)) return fail(GMM_ERR_INVALID_ARG, "fusion bit I must be 0 or 1");
      if (!(c == std::floor(c) && c >= -3.0 && c <= 3.0))
        return fail(GMM_ERR_INVALID_ARG, "fusion counter cpt must be an integer in [-3, 3]");
      f[i] = static_cast<uint8_t>((static_cast<int>(c) + 3) | (static_cast<int>(I) << 3));
    }
    for (size_t i = n; i < h->fuse_bytes; ++i) f[i] = static_cast<uint8_t>(kFuseInit);
  } else if (sep_depth(h)) {  // the flags bytes of a depth-only handle: no List 1 state, no holes counted
    uint8_t* f = raw.data() + off;
    for (size_t i = 0; i < h->fuse_bytes; ++i) f[i] = static_cast<uint8_t>(kFuseInit);
  }
  DeviceGuard g(h->cfg.device);
  if (!g.ok()) return fail(GMM_ERR_DEVICE, "cannot select the handle's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(h->mem, raw.data(), total, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && has_rgb(h))
    e = launch_rekey(h->st_rgb, h->cfg.state_dtype, h->tiles64, h->cfg.M, is_augmented(h) ? 4 : 3, s);
  if (e == hipSuccess && sep_depth(h)) e = launch_rekey(h->st_depth, h->cfg.state_dtype, h->tiles64, h->cfg.M, 1, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "state copy to device");
  h->last_stream = s;
  return GMM_OK;
}

}  // extern "C"
