// Device-side building blocks of the per-pixel mixture step (gfx950, wave64).
//
// One lane owns one pixel of one modality. Its M components are loaded from structure-of-
// arrays planes (one plane per parameter and rank, so a wave's 64 lanes read 64 consecutive
// values), advanced one frame in fp32 registers, re-sorted in registers and written back.
// Every kernel of the library (plain, fused, batched) calls the same functions below, so all
// of them produce bit-identical results for the same pixel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgbd {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// Per-modality constants of the model (Sec. III.A), prepared once on the host in fp32.
struct ModelConsts {
  float alpha;     // learning rate of weights, means and variances
  float oma;       // 1 - alpha
  float k2;        // k^2, the match threshold squared (strict d^2 < k^2 var)
  float T;         // background weight threshold
  float var0;      // sigma0^2 of a new component
  float var_min;   // variance floor
  float w_init;    // weight of a new component before renormalisation
  int32_t hole_skip;  // depth: value 0 leaves the state untouched, pixel background
};

// ---- storage types of the mixture state --------------------------------------------------
struct f16s { uint16_t b; };
struct bf16s { uint16_t b; };

template <typename S> struct Storage;
template <> struct Storage<float> {
  static __device__ __forceinline__ float load(float v) { return v; }
  static __device__ __forceinline__ float pack(float f) { return f; }
};
template <> struct Storage<f16s> {
  static __device__ __forceinline__ float load(f16s v) {
    return static_cast<float>(__builtin_bit_cast(_Float16, v.b));
  }
  static __device__ __forceinline__ f16s pack(float f) {
    return f16s{__builtin_bit_cast(uint16_t, static_cast<_Float16>(f))};  // round to nearest even
  }
};
template <> struct Storage<bf16s> {
  static __device__ __forceinline__ float load(bf16s v) {
    return __builtin_bit_cast(float, static_cast<uint32_t>(v.b) << 16);
  }
  static __device__ __forceinline__ bf16s pack(float f) {
    // round to nearest even on the upper 16 bits (finite values; overflow goes to infinity)
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return bf16s{static_cast<uint16_t>(u >> 16)};
  }
};

// ---- the mixture of one pixel ----------------------------------------------------------
template <int M, int C>
struct Mix {
  float mu[C][M];
  float var[M];
  float w[M];
};

// One modality's state block as a buffer resource, in a tiled structure-of-arrays layout:
// pixels are grouped in tiles of 64 (one wave); a tile stores its P*M planes back to back
// (plane order: mu channel 0..C-1, var, w; each parameter M rank-major planes), each plane-row
// holding the tile's 64 values. A wave's accesses therefore stay one coalesced 64-value segment
// per instruction AND fall in one contiguous region per tile (P*M*64 values), instead of P*M
// regions spread over the whole frame. A lane's tile+lane byte offset lives in one VGPR and the
// plane offset is a compile-time immediate, so every state access is one buffer instruction.
// The range checked by the hardware (num_records) is the whole block: an access outside it reads
// 0 and drops its write instead of touching other memory. The host keeps every block < 4 GiB.
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, gfx9-family descriptor word 3

struct StateBlock {
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t tile_bytes;  // P*M*64*sizeof(S)
};

__device__ __forceinline__ StateBlock make_block(void* base, uint32_t tiles64, int esize, int planes) {
  const uint32_t tb = static_cast<uint32_t>(planes * kWave * esize);
  return StateBlock{__builtin_amdgcn_make_buffer_rsrc(base, 0, static_cast<int>(tb * tiles64), kRsrcWord3), tb};
}

__device__ __forceinline__ uint32_t lane_offset(const StateBlock& b, uint32_t p, uint32_t esize) {
  return (p >> 6) * b.tile_bytes + (p & 63u) * esize;
}

template <typename S> struct BufIO;
template <> struct BufIO<float> {
  static __device__ __forceinline__ float ld(const StateBlock& b, uint32_t off, uint32_t so) {
    // the b32 builtins move raw 32-bit words: reinterpret, never convert
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.rsrc, off, so, 0));
  }
  static __device__ __forceinline__ void st(const StateBlock& b, uint32_t off, uint32_t so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), b.rsrc, off, so, 0);
  }
};
template <> struct BufIO<f16s> {
  static __device__ __forceinline__ f16s ld(const StateBlock& b, uint32_t off, uint32_t so) {
    return f16s{__builtin_amdgcn_raw_buffer_load_b16(b.rsrc, off, so, 0)};
  }
  static __device__ __forceinline__ void st(const StateBlock& b, uint32_t off, uint32_t so, f16s v) {
    __builtin_amdgcn_raw_buffer_store_b16(v.b, b.rsrc, off, so, 0);
  }
};
template <> struct BufIO<bf16s> {
  static __device__ __forceinline__ bf16s ld(const StateBlock& b, uint32_t off, uint32_t so) {
    return bf16s{__builtin_amdgcn_raw_buffer_load_b16(b.rsrc, off, so, 0)};
  }
  static __device__ __forceinline__ void st(const StateBlock& b, uint32_t off, uint32_t so, bf16s v) {
    __builtin_amdgcn_raw_buffer_store_b16(v.b, b.rsrc, off, so, 0);
  }
};

template <int M, int C, typename S>
__device__ __forceinline__ void load_mix(Mix<M, C>& m, const StateBlock& b, uint32_t p) {
  constexpr uint32_t es = sizeof(S);
  constexpr uint32_t row = kWave * es;  // bytes of one plane-row of a tile
  const uint32_t off = lane_offset(b, p, es);
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int r = 0; r < M; ++r) m.mu[c][r] = Storage<S>::load(BufIO<S>::ld(b, off + (c * M + r) * row, 0));
#pragma unroll
  for (int r = 0; r < M; ++r) m.var[r] = Storage<S>::load(BufIO<S>::ld(b, off + (C * M + r) * row, 0));
#pragma unroll
  for (int r = 0; r < M; ++r) m.w[r] = Storage<S>::load(BufIO<S>::ld(b, off + ((C + 1) * M + r) * row, 0));
}

template <int M, int C, typename S>
__device__ __forceinline__ void store_mix(const Mix<M, C>& m, const StateBlock& b, uint32_t p) {
  constexpr uint32_t es = sizeof(S);
  constexpr uint32_t row = kWave * es;
  const uint32_t off = lane_offset(b, p, es);
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int r = 0; r < M; ++r) BufIO<S>::st(b, off + (c * M + r) * row, 0, Storage<S>::pack(m.mu[c][r]));
#pragma unroll
  for (int r = 0; r < M; ++r) BufIO<S>::st(b, off + (C * M + r) * row, 0, Storage<S>::pack(m.var[r]));
#pragma unroll
  for (int r = 0; r < M; ++r) BufIO<S>::st(b, off + ((C + 1) * M + r) * row, 0, Storage<S>::pack(m.w[r]));
}

template <typename T>
__device__ __forceinline__ void cswap(bool s, T& a, T& b) {
  const T ta = a, tb = b;
  a = s ? tb : ta;
  b = s ? ta : tb;
}

// One frame of the mixture model for one pixel (Sec. III.A with the update rules of the
// paper's reference [6]). Returns the foreground bit.
//   match    : first live rank, in stored (w/sigma descending) order, with |x-mu|^2 < k^2 var
//   weights  : w <- (1-alpha) w + alpha [matched]
//   matched  : mu <- (1-alpha) mu + alpha x ; var <- max(var_min, (1-alpha) var + alpha |x-mu_new|^2)
//   no match : the last rank becomes (x, sigma0^2, w_init)
//   then     : w <- w / sum(w); stable sort by w/sigma descending;
//              B = min{b : w_0+...+w_{b-1} > T}; foreground = no match or new rank >= B
template <int M, int C>
__device__ __forceinline__ bool mix_step(Mix<M, C>& s, const float (&x)[C], const ModelConsts& k) {
  // match, in rank order
  int j = M;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    float d2 = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float t = x[c] - s.mu[c][r];
      d2 = fmaf(t, t, d2);
    }
    const bool hit = (s.w[r] > 0.f) & (d2 < k.k2 * s.var[r]);  // no short-circuit: no branch
    j = ((j == M) & hit) ? r : j;
  }
  const bool matched = j < M;

  // weight decay; the matched component is gathered, updated once and scattered back
  // (branch-free: every rank is a select, no per-rank divergent region)
  float mj[C], vj = s.var[0];
#pragma unroll
  for (int c = 0; c < C; ++c) mj[c] = s.mu[c][0];
#pragma unroll
  for (int r = 1; r < M; ++r) {
    const bool isj = (r == j);
    vj = isj ? s.var[r] : vj;
#pragma unroll
    for (int c = 0; c < C; ++c) mj[c] = isj ? s.mu[c][r] : mj[c];
  }
  float d2n = 0.f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    mj[c] = fmaf(k.oma, mj[c], k.alpha * x[c]);
    const float t = x[c] - mj[c];
    d2n = fmaf(t, t, d2n);
  }
  vj = fmaxf(k.var_min, fmaf(k.oma, vj, k.alpha * d2n));
#pragma unroll
  for (int r = 0; r < M; ++r) {
    const bool isj = (r == j);
    s.w[r] = fmaf(k.oma, s.w[r], isj ? k.alpha : 0.f);
    s.var[r] = isj ? vj : s.var[r];
#pragma unroll
    for (int c = 0; c < C; ++c) s.mu[c][r] = isj ? mj[c] : s.mu[c][r];
  }
  // no match: the least probable (last-ranked) component is replaced
  if (!matched) {
#pragma unroll
    for (int c = 0; c < C; ++c) s.mu[c][M - 1] = x[c];
    s.var[M - 1] = k.var0;
    s.w[M - 1] = k.w_init;
  }

  // renormalise
  float S = s.w[0];
#pragma unroll
  for (int r = 1; r < M; ++r) S += s.w[r];
  const float inv = 1.0f / S;
#pragma unroll
  for (int r = 0; r < M; ++r) s.w[r] *= inv;

  // stable sort by w/sigma, descending (bubble network of adjacent compare-exchanges that swap
  // only on a strictly larger key, hence stable); q follows the updated / new component
  float key[M];
#pragma unroll
  for (int r = 0; r < M; ++r) key[r] = s.w[r] * __builtin_amdgcn_rsqf(s.var[r]);
  int q = matched ? j : M - 1;
#pragma unroll
  for (int i = 0; i < M - 1; ++i) {
#pragma unroll
    for (int r = 0; r < M - 1 - i; ++r) {
      const bool sw = key[r + 1] > key[r];
      cswap(sw, key[r], key[r + 1]);
      cswap(sw, s.w[r], s.w[r + 1]);
      cswap(sw, s.var[r], s.var[r + 1]);
#pragma unroll
      for (int c = 0; c < C; ++c) cswap(sw, s.mu[c][r], s.mu[c][r + 1]);
      const int qs = (q == r) ? r + 1 : ((q == r + 1) ? r : q);
      q = sw ? qs : q;
    }
  }

  // background set: the first B ranks whose cumulative weight exceeds T
  int B = M;
  float run = 0.f;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    run += s.w[r];
    B = (B == M && run > k.T) ? r + 1 : B;
  }
  return !matched || q >= B;
}

// List 1 (Sec. III.C): one transition of the fused bit I and counter cpt of a pixel.
// Encoded state byte: bits 0-2 hold cpt + 3 (0..6), bit 3 holds I.
__device__ __forceinline__ uint32_t fuse_transition(uint32_t st, bool r, bool d) {
  int c = static_cast<int>(st & 7u) - 3;
  bool I = (st >> 3) & 1u;
  if (r == d) {
    I = d;
    c = 0;
  } else if (c == 3) {
    I = r;
    c = 0;
  } else if (c == -3) {
    I = d;
    c = 0;
  } else {
    c += (I == r) ? 1 : -1;
  }
  return static_cast<uint32_t>(c + 3) | (static_cast<uint32_t>(I) << 3);
}

constexpr uint32_t kFuseInit = 3u;  // I = 0, cpt = 0

// Make this wave's LDS writes visible to its own later LDS reads (no block barrier needed:
// each wave stages only its own pixels).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace rgbd
