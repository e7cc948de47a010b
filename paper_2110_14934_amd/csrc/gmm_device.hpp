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

// One modality's state block as a buffer resource, in a tiled layout. Pixels are grouped in
// tiles of 64 (one wave); each pixel has NV = P*M values (plane order: mu channel 0..C-1, var,
// w; each parameter M ranks). Inside a tile, values are stored in 16-byte chunks per lane: chunk
// c holds values [c*VPC, (c+1)*VPC) of all 64 lanes as [lane][VPC] (VPC = 16/sizeof(value)), so
// one wave instruction moves 1 KB of contiguous memory; the NV % VPC values left over are
// stored as single rows [lane]. A wave's accesses to one modality fall in one contiguous region
// of NV*64 values, with no padding. A lane's tile + lane byte offset lives in one VGPR and the
// chunk offsets are compile-time constants, so every state access is one buffer instruction.
// The range checked by the hardware (num_records) is the whole block: an access outside it
// reads 0 and drops its write instead of touching other memory. The host keeps every block
// below 4 GiB.
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, gfx9-family descriptor word 3
constexpr uint32_t kChunkBytes = 16;

// Byte offset, inside its tile, of value v of lane `lane` (nv values per pixel, es bytes each).
__host__ __device__ constexpr uint32_t tile_value_offset(uint32_t v, uint32_t lane, uint32_t nv, uint32_t es) {
  const uint32_t vpc = kChunkBytes / es;
  const uint32_t nc = nv / vpc;
  const uint32_t nf = nc * vpc;
  return v < nf ? (v / vpc) * (64u * kChunkBytes) + lane * kChunkBytes + (v % vpc) * es
                : nc * (64u * kChunkBytes) + (v - nf) * 64u * es + lane * es;
}

struct StateBlock {
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t tile_bytes;  // P*M*64*sizeof(S)
};

__device__ __forceinline__ StateBlock make_block(void* base, uint32_t tiles64, int esize, int planes) {
  const uint32_t tb = static_cast<uint32_t>(planes * kWave * esize);
  return StateBlock{__builtin_amdgcn_make_buffer_rsrc(base, 0, static_cast<int>(tb * tiles64), kRsrcWord3), tb};
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename S> struct BufIO;
template <> struct BufIO<float> {
  // the b32 builtins move raw 32-bit words: reinterpret, never convert
  static __device__ __forceinline__ float ld(const StateBlock& b, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.rsrc, off, 0, 0));
  }
  static __device__ __forceinline__ void st(const StateBlock& b, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), b.rsrc, off, 0, 0);
  }
  static __device__ __forceinline__ float from_word(uint32_t w, int) { return __builtin_bit_cast(float, w); }
  static __device__ __forceinline__ uint32_t word(const float* v) { return __builtin_bit_cast(uint32_t, v[0]); }
};
template <> struct BufIO<f16s> {
  static __device__ __forceinline__ float ld(const StateBlock& b, uint32_t off) {
    return Storage<f16s>::load(f16s{__builtin_amdgcn_raw_buffer_load_b16(b.rsrc, off, 0, 0)});
  }
  static __device__ __forceinline__ void st(const StateBlock& b, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(Storage<f16s>::pack(v).b, b.rsrc, off, 0, 0);
  }
  // a word holds two values, the lower-addressed one in the low half
  static __device__ __forceinline__ float from_word(uint32_t w, int half) {
    return Storage<f16s>::load(f16s{static_cast<uint16_t>(half ? (w >> 16) : (w & 0xFFFFu))});
  }
  static __device__ __forceinline__ uint32_t word(const float* v) {
    return static_cast<uint32_t>(Storage<f16s>::pack(v[0]).b) | (static_cast<uint32_t>(Storage<f16s>::pack(v[1]).b) << 16);
  }
};
template <> struct BufIO<bf16s> {
  static __device__ __forceinline__ float ld(const StateBlock& b, uint32_t off) {
    return Storage<bf16s>::load(bf16s{__builtin_amdgcn_raw_buffer_load_b16(b.rsrc, off, 0, 0)});
  }
  static __device__ __forceinline__ void st(const StateBlock& b, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(Storage<bf16s>::pack(v).b, b.rsrc, off, 0, 0);
  }
  static __device__ __forceinline__ float from_word(uint32_t w, int half) {
    return __builtin_bit_cast(float, half ? (w & 0xFFFF0000u) : (w << 16));
  }
  static __device__ __forceinline__ uint32_t word(const float* v) {
    return static_cast<uint32_t>(Storage<bf16s>::pack(v[0]).b) | (static_cast<uint32_t>(Storage<bf16s>::pack(v[1]).b) << 16);
  }
};

// All NV values of pixel p (16-byte chunks, then single values).
template <int NV, typename S>
__device__ __forceinline__ void load_values(float (&v)[NV], const StateBlock& b, uint32_t p) {
  constexpr uint32_t es = sizeof(S), vpc = kChunkBytes / es, nc = NV / vpc, nf = nc * vpc, vpw = 4 / es;
  const uint32_t lane = p & 63u;
  const uint32_t base = (p >> 6) * b.tile_bytes;
#pragma unroll
  for (uint32_t c = 0; c < nc; ++c) {
    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(b.rsrc, base + lane * kChunkBytes + c * 64u * kChunkBytes, 0, 0);
#pragma unroll
    for (uint32_t i = 0; i < vpc; ++i) v[c * vpc + i] = BufIO<S>::from_word(w[i / vpw], static_cast<int>(i % vpw));
  }
#pragma unroll
  for (uint32_t j = nf; j < static_cast<uint32_t>(NV); ++j) v[j] = BufIO<S>::ld(b, base + tile_value_offset(j, lane, NV, es));
}

template <int NV, typename S>
__device__ __forceinline__ void store_values(const float (&v)[NV], const StateBlock& b, uint32_t p) {
  constexpr uint32_t es = sizeof(S), vpc = kChunkBytes / es, nc = NV / vpc, nf = nc * vpc, vpw = 4 / es;
  const uint32_t lane = p & 63u;
  const uint32_t base = (p >> 6) * b.tile_bytes;
#pragma unroll
  for (uint32_t c = 0; c < nc; ++c) {
    u32x4 w;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) w[i] = BufIO<S>::word(&v[c * vpc + i * vpw]);
    __builtin_amdgcn_raw_buffer_store_b128(w, b.rsrc, base + lane * kChunkBytes + c * 64u * kChunkBytes, 0, 0);
  }
#pragma unroll
  for (uint32_t j = nf; j < static_cast<uint32_t>(NV); ++j) BufIO<S>::st(b, base + tile_value_offset(j, lane, NV, es), v[j]);
}

template <int M, int C, typename S>
__device__ __forceinline__ void load_mix(Mix<M, C>& m, const StateBlock& b, uint32_t p) {
  float v[(C + 2) * M];
  load_values<(C + 2) * M, S>(v, b, p);
#pragma unroll
  for (int r = 0; r < M; ++r) {
#pragma unroll
    for (int c = 0; c < C; ++c) m.mu[c][r] = v[c * M + r];
    m.var[r] = v[C * M + r];
    m.w[r] = v[(C + 1) * M + r];
  }
}

template <int M, int C, typename S>
__device__ __forceinline__ void store_mix(const Mix<M, C>& m, const StateBlock& b, uint32_t p) {
  float v[(C + 2) * M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
#pragma unroll
    for (int c = 0; c < C; ++c) v[c * M + r] = m.mu[c][r];
    v[C * M + r] = m.var[r];
    v[(C + 1) * M + r] = m.w[r];
  }
  store_values<(C + 2) * M, S>(v, b, p);
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
