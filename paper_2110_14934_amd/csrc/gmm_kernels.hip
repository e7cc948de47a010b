// Per-frame kernels of one stream: colour and/or depth mixture step, optional List 1 fusion.
//
// Mapping: one lane per pixel of the row-major frame; a wave covers 64 consecutive pixels, so
// its foreground bits form exactly one uint64 word of the output mask (one ballot, one store).
// The interleaved RGB8 input of a wave (192 contiguous bytes when rows are dense) is staged
// through LDS with 48 dword loads and de-interleaved on chip - the structure-of-arrays split of
// the colour image done without a separate pass. The state is kept in planes per modality (see
// gmm_device.hpp): rows of the fast-path values (a wave's row load or store moves up to 1 KB of
// contiguous memory, and the rows of consecutive waves follow each other), then each pixel's
// remaining values, contiguous per pixel, then (fp32 state) one weight scale per 64-pixel tile.
#include <hip/hip_runtime.h>

#include "gmm_device.hpp"
#include "gmm_internal.hpp"
#include "gmm_frame.hpp"

namespace rgbd {

// One stream, one frame. MODE is a combination of kModeRGB, kModeDepth, kModeFuse, or kModeAug
// alone (the four-channel variant).
template <int M, typename S, int MODE, int CP>
__global__ void __launch_bounds__(kBlock) frame_kernel(FrameArgs a) {
  __shared__ uint32_t lds[kWavesPerBlock][48];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  process_pixel<M, S, MODE, CP>(a, blockIdx.x * kBlock + threadIdx.x, lane, lds[wv]);
}

// Standalone List 1 over two given masks.
__global__ void __launch_bounds__(kBlock) fuse_kernel(const uint64_t* __restrict__ fr,
                                                      const uint64_t* __restrict__ fd,
                                                      uint64_t* __restrict__ out,
                                                      uint8_t* __restrict__ fstate, int64_t npix) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t word = (p - lane) >> 6;
  const bool valid = p < npix;
  bool fgf = false;
  if (valid) {
    const bool r = (fr[word] >> lane) & 1ull;
    const bool d = (fd[word] >> lane) & 1ull;
    const uint32_t st = fuse_transition(fstate[p], r, d);
    fstate[p] = static_cast<uint8_t>(st);
    fgf = (st >> 3) & 1u;
  }
  const uint64_t bits = __ballot(fgf);
  if (lane == 0 && valid) out[word] = bits;
}

// Empty components: mu = 0, var = sigma0^2, w = 0 (C+2 parameters x M ranks; in the scaled
// form rank 1's key 0, which is 0 / sigma0, and the scale of every tile 1), two-plane layout.
// (Padding halves of 16-bit words are never read.)
template <int M, int C, typename S>
__global__ void __launch_bounds__(kBlock) init_kernel(S* st, uint32_t tiles64, float var0) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  constexpr uint32_t nv = value_count(M, C, sizeof(S));
  const int64_t values = static_cast<int64_t>(nv) * kWave * tiles64;
  if constexpr (kScaled<S>) {
    if (i >= values && i < values + tiles64) {
      using P = Plan<M, C, S>;  // (constants: a layout object built at run time would live in scratch)
      const uint64_t byte = static_cast<uint64_t>(tiles64) * 64u * (P::hot + P::sb) + 4u * static_cast<uint64_t>(i - values);
      *reinterpret_cast<float*>(reinterpret_cast<char*>(st) + byte) = 1.f;
    }
  }
  if (i >= values) return;
  const uint32_t lane = static_cast<uint32_t>(i % kWave);
  const uint32_t v = static_cast<uint32_t>((i / kWave) % nv);
  const int64_t tile = i / (static_cast<int64_t>(kWave) * nv);
  const uint64_t byte = value_offset<M, C, S>(v, static_cast<uint64_t>(tile) * kWave + lane, tiles64);
  // value order: direct - M weights, then per rank (variance, C means); scaled - rank 0's
  // (scaled weight, variance, C means), rank 1's key, then the same for ranks 1 .. M-1
  float init = 0.f;
  if constexpr (kScaled<S>) {
    const bool key = M > 1 && v == key_index(C);
    const uint32_t pos = v < C + 2 ? v : (v - 1) % (C + 2);
    init = !key && pos == 1 ? var0 : 0.f;
  } else {
    const bool is_var = v >= static_cast<uint32_t>(M) && (v - static_cast<uint32_t>(M)) % static_cast<uint32_t>(C + 1) == 0;
    init = is_var ? var0 : 0.f;
  }
  *reinterpret_cast<S*>(reinterpret_cast<char*>(st) + byte) = Storage<S>::pack(init);
}

// Rank 1's key of every pixel from its stored scaled weight and variance (scaled form, M > 1),
// computed as the frame kernels compute it: after a state written from the host.
template <int M, int C>
__global__ void __launch_bounds__(kBlock) rekey_kernel(float* st, uint32_t tiles64) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= static_cast<int64_t>(tiles64) * kWave) return;
  char* b = reinterpret_cast<char*>(st);
  const uint64_t pp = static_cast<uint64_t>(p);
  const float w1 = *reinterpret_cast<const float*>(b + value_offset<M, C, float>(value_index(C + 1, 1, M, C, 4), pp, tiles64));
  const float v1 = *reinterpret_cast<const float*>(b + value_offset<M, C, float>(value_index(C, 1, M, C, 4), pp, tiles64));
  *reinterpret_cast<float*>(b + value_offset<M, C, float>(key_index(C), pp, tiles64)) = w1 * __builtin_amdgcn_rsqf(v1);
}

__global__ void __launch_bounds__(kBlock) fill_u8_kernel(uint8_t* p, uint8_t v, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- dispatch ----------------------------------------------------------------------------

static inline dim3 grid_for(int64_t n) {
  return dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock));
}

template <int M, typename S, int CP>
static hipError_t launch_frame_msc(const FrameArgs& a, int mode, hipStream_t s) {
  const dim3 g = grid_for(a.npix), b(kBlock);
  switch (mode) {
    case kModeRGB: frame_kernel<M, S, kModeRGB, CP><<<g, b, 0, s>>>(a); break;
    case kModeDepth: frame_kernel<M, S, kModeDepth, CP><<<g, b, 0, s>>>(a); break;
    case kModeRGB | kModeDepth: frame_kernel<M, S, kModeRGB | kModeDepth, CP><<<g, b, 0, s>>>(a); break;
    case kModeRGB | kModeDepth | kModeFuse:
      frame_kernel<M, S, kModeRGB | kModeDepth | kModeFuse, CP><<<g, b, 0, s>>>(a);
      break;
    case kModeAug: frame_kernel<M, S, kModeAug, CP><<<g, b, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int M, typename S>
static hipError_t launch_frame_ms(const FrameArgs& a, int mode, bool stream, hipStream_t s) {
  return stream ? launch_frame_msc<M, S, kStream>(a, mode, s) : launch_frame_msc<M, S, kCached>(a, mode, s);
}

template <typename S>
static hipError_t launch_frame_s(const FrameArgs& a, int M, int mode, bool stream, hipStream_t s) {
  switch (M) {
    case 1: return launch_frame_ms<1, S>(a, mode, stream, s);
    case 2: return launch_frame_ms<2, S>(a, mode, stream, s);
    case 3: return launch_frame_ms<3, S>(a, mode, stream, s);
    case 4: return launch_frame_ms<4, S>(a, mode, stream, s);
    case 5: return launch_frame_ms<5, S>(a, mode, stream, s);
    default: return hipErrorInvalidValue;
  }
}

bool frame_variant_compiled(int M, int dtype) {
  return M >= 1 && M <= 5 && (dtype == GMM_F32 || dtype == GMM_F16 || dtype == GMM_BF16);
}

hipError_t launch_frame(const FrameArgs& a, int M, int dtype, int mode, bool stream, hipStream_t s) {
  switch (dtype) {
    case GMM_F32: return launch_frame_s<float>(a, M, mode, stream, s);
    case GMM_F16: return launch_frame_s<f16s>(a, M, mode, stream, s);
    case GMM_BF16: return launch_frame_s<bf16s>(a, M, mode, stream, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fuse(const uint64_t* fr, const uint64_t* fd, uint64_t* out, uint8_t* fstate,
                       int64_t npix, hipStream_t s) {
  fuse_kernel<<<grid_for(npix), dim3(kBlock), 0, s>>>(fr, fd, out, fstate, npix);
  return hipGetLastError();
}

template <int M, int C>
static void init_mc(void* st, int dtype, uint32_t tiles64, float var0, dim3 g, hipStream_t s) {
  switch (dtype) {
    case GMM_F32: init_kernel<M, C, float><<<g, dim3(kBlock), 0, s>>>(static_cast<float*>(st), tiles64, var0); break;
    case GMM_F16: init_kernel<M, C, f16s><<<g, dim3(kBlock), 0, s>>>(static_cast<f16s*>(st), tiles64, var0); break;
    default: init_kernel<M, C, bf16s><<<g, dim3(kBlock), 0, s>>>(static_cast<bf16s*>(st), tiles64, var0); break;
  }
}

template <int C>
static hipError_t init_c(void* st, int dtype, uint32_t tiles64, int M, float var0, dim3 g, hipStream_t s) {
  switch (M) {
    case 1: init_mc<1, C>(st, dtype, tiles64, var0, g, s); break;
    case 2: init_mc<2, C>(st, dtype, tiles64, var0, g, s); break;
    case 3: init_mc<3, C>(st, dtype, tiles64, var0, g, s); break;
    case 4: init_mc<4, C>(st, dtype, tiles64, var0, g, s); break;
    case 5: init_mc<5, C>(st, dtype, tiles64, var0, g, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int C>
static hipError_t rekey_c(void* st, uint32_t tiles64, int M, dim3 g, hipStream_t s) {
  float* f = static_cast<float*>(st);
  switch (M) {
    case 1: return hipSuccess;  // no rank 1
    case 2: rekey_kernel<2, C><<<g, dim3(kBlock), 0, s>>>(f, tiles64); break;
    case 3: rekey_kernel<3, C><<<g, dim3(kBlock), 0, s>>>(f, tiles64); break;
    case 4: rekey_kernel<4, C><<<g, dim3(kBlock), 0, s>>>(f, tiles64); break;
    case 5: rekey_kernel<5, C><<<g, dim3(kBlock), 0, s>>>(f, tiles64); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rekey(void* st, int dtype, uint32_t tiles64, int M, int C, hipStream_t s) {
  if (!scaled_weights(static_cast<uint32_t>(dtype_size(dtype)))) return hipSuccess;
  const dim3 g = grid_for(static_cast<int64_t>(tiles64) * kWave);
  switch (C) {
    case 1: return rekey_c<1>(st, tiles64, M, g, s);
    case 3: return rekey_c<3>(st, tiles64, M, g, s);
    case 4: return rekey_c<4>(st, tiles64, M, g, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init(void* st, int dtype, uint32_t tiles64, int M, int C, float var0, hipStream_t s) {
  if (dtype != GMM_F32 && dtype != GMM_F16 && dtype != GMM_BF16) return hipErrorInvalidValue;
  const uint32_t es = static_cast<uint32_t>(dtype_size(dtype));
  const int64_t total = static_cast<int64_t>(value_count(static_cast<uint32_t>(M), static_cast<uint32_t>(C), es)) *
                            kWave * tiles64 +
                        (scaled_weights(es) ? tiles64 : 0);
  const dim3 g = grid_for(total);
  switch (C) {
    case 1: return init_c<1>(st, dtype, tiles64, M, var0, g, s);
    case 3: return init_c<3>(st, dtype, tiles64, M, var0, g, s);
    case 4: return init_c<4>(st, dtype, tiles64, M, var0, g, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) {
  fill_u8_kernel<<<grid_for(n), dim3(kBlock), 0, s>>>(p, v, n);
  return hipGetLastError();
}

}  // namespace rgbd
