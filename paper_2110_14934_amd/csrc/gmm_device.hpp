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

#include <type_traits>

namespace rgbd {

// Compile-time loop: f(std::integral_constant<int, I>{}) for I = B .. E-1. The per-pixel code
// indexes its arrays only through such constants, so every index is fixed before any
// optimisation runs and the whole mixture stays in registers. (With ordinary unrolled loops the
// compiler may turn "a ? v[r-1] : v[r]" into a load from a selected address before the loop is
// unrolled; the array then needs memory and lands in LDS, one round trip per access.)
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
#define RGBD_I(i_) decltype(i_)::value
// loop bodies are inlined before any other optimisation sees them (see static_for)
#define RGBD_BODY __attribute__((always_inline))

// c ? a : b on values. (A conditional whose operands are both lvalues - two array elements, or
// an element and a local - is itself an lvalue: it selects an address and loads from it, which
// keeps the arrays in memory. Passing by value selects the values.)
__device__ __forceinline__ float pick(bool c, float a, float b) { return c ? a : b; }
__device__ __forceinline__ int pick(bool c, int a, int b) { return c ? a : b; }

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
  int32_t rho_density;  // 0: mean/variance rate alpha; 1: alpha times the matched density
  float rho_scale;      // alpha (2 pi)^(-C/2), the constant factor of that density rate
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

// Order of a pixel's NV = (C+2)*M values: the M weights first, then rank by rank the variance
// and the C means. The values a frame needs when the pixel matches its top-ranked component and
// keeps its rank - every weight, rank 0, and rank 1's variance - are then a prefix.
__host__ __device__ constexpr uint32_t value_index(uint32_t param, uint32_t rank, uint32_t M, uint32_t C) {
  // param: 0..C-1 = mean channel, C = variance, C+1 = weight
  return param == C + 1 ? rank : M + rank * (C + 1) + (param == C ? 0 : 1 + param);
}

// One modality's state block as a buffer resource, in a tiled layout. Pixels are grouped in
// tiles of 64 (one wave); each pixel has NV values (in value_index order). Inside a tile, values
// are stored in 16-byte chunks per lane: chunk
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
  // the 32-bit word holding value a (and b, for 16-bit types, in the high half); by value, so
  // the values stay in registers
  static __device__ __forceinline__ uint32_t word(float a, float) { return __builtin_bit_cast(uint32_t, a); }
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
  static __device__ __forceinline__ uint32_t word(float a, float b) {
    return static_cast<uint32_t>(Storage<f16s>::pack(a).b) | (static_cast<uint32_t>(Storage<f16s>::pack(b).b) << 16);
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
  static __device__ __forceinline__ uint32_t word(float a, float b) {
    return static_cast<uint32_t>(Storage<bf16s>::pack(a).b) | (static_cast<uint32_t>(Storage<bf16s>::pack(b).b) << 16);
  }
};

// Bytes of state one wave moves when it reads (or writes) values [0, LIMIT): whole chunks and
// single rows that start below LIMIT, for all 64 lanes.
template <int NV, int LIMIT, typename S>
__host__ __device__ constexpr uint32_t prefix_bytes() {
  constexpr uint32_t es = sizeof(S), vpc = kChunkBytes / es, nc = NV / vpc, nf = nc * vpc;
  uint32_t chunks = 0, singles = 0;
  for (uint32_t c = 0; c < nc; ++c)
    if (c * vpc < static_cast<uint32_t>(LIMIT)) ++chunks;
  for (uint32_t j = nf; j < static_cast<uint32_t>(NV); ++j)
    if (j < static_cast<uint32_t>(LIMIT)) ++singles;
  return chunks * 64u * kChunkBytes + singles * 64u * es;
}

// Whether load_values<NV, LIMIT, S> reads value v: its whole 16-byte chunk comes along when the
// chunk starts below LIMIT, so a chunk may carry values at or beyond LIMIT.
template <int NV, int LIMIT, typename S>
__host__ __device__ constexpr bool value_read(uint32_t v) {
  constexpr uint32_t vpc = kChunkBytes / sizeof(S), nf = (NV / vpc) * vpc;
  return v < nf ? (v / vpc) * vpc < static_cast<uint32_t>(LIMIT) : v < static_cast<uint32_t>(LIMIT);
}

// Every value a store of [0, SF) writes (whole chunks) is one a load of [0, LF) read.
template <int NV, int LF, int SF, typename S>
__host__ __device__ constexpr bool stores_only_read() {
  for (uint32_t v = 0; v < static_cast<uint32_t>(NV); ++v)
    if (value_read<NV, SF, S>(v) && !value_read<NV, LF, S>(v)) return false;
  return true;
}

// Values that are only read (not written) by the frame of a pixel that matches rank 0 and keeps
// it: all weights, rank 0 (variance, means) and the variance of rank 1.
template <int M, int C>
constexpr int kFastLoad = M > 1 ? M + (C + 1) + 1 : M + (C + 1);
// ... and the values such a frame changes: all weights and rank 0.
template <int M, int C>
constexpr int kFastStore = M + (C + 1);

// Value V (in value_index order) of a pixel's mixture, as the Mix field that holds it.
template <int M, int C, int V>
__device__ __forceinline__ float& field(Mix<M, C>& m) {
  if constexpr (V < M) {
    return m.w[V];
  } else {
    constexpr int r = (V - M) / (C + 1), pos = (V - M) % (C + 1);
    if constexpr (pos == 0) return m.var[r];
    else return m.mu[pos - 1][r];
  }
}
template <int M, int C, int V>
__device__ __forceinline__ float field(const Mix<M, C>& m) {
  return field<M, C, V>(const_cast<Mix<M, C>&>(m));
}

// Values [0, LIMIT) of pixel p, straight into the Mix: every 16-byte chunk and single value
// that starts below LIMIT (whole chunks, so a little beyond LIMIT may come along; see
// value_read). A value not read is left at 0 - a variance at 1, so that keys stay finite (any
// use of it is discarded by the caller). LIMIT = NV reads everything.
template <int M, int C, typename S, int LIMIT = (C + 2) * M>
__device__ __forceinline__ void load_mix(Mix<M, C>& m, const StateBlock& b, uint32_t p) {
  constexpr int NV = (C + 2) * M, es = sizeof(S), vpc = kChunkBytes / es, nc = NV / vpc, nf = nc * vpc,
                vpw = 4 / es;
  const uint32_t lane = p & 63u;
  const uint32_t base = (p >> 6) * b.tile_bytes;
  static_for<0, NV>([&](auto v_) RGBD_BODY {
    constexpr int v = RGBD_I(v_);
    if constexpr (!value_read<NV, LIMIT, S>(v)) field<M, C, v>(m) = (v >= M && (v - M) % (C + 1) == 0) ? 1.f : 0.f;
  });
  static_for<0, nc>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    if constexpr (c * vpc < LIMIT) {
      const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(b.rsrc, base + lane * kChunkBytes + c * 64u * kChunkBytes, 0, 0);
      static_for<0, vpc>([&](auto i_) RGBD_BODY {
        constexpr int i = RGBD_I(i_);
        field<M, C, c * vpc + i>(m) = BufIO<S>::from_word(w[i / vpw], i % vpw);
      });
    }
  });
  static_for<nf, NV>([&](auto j_) RGBD_BODY {
    constexpr int j = RGBD_I(j_);
    if constexpr (j < LIMIT) field<M, C, j>(m) = BufIO<S>::ld(b, base + tile_value_offset(j, lane, NV, es));
  });
}

// Values [0, LIMIT) of pixel p from the Mix (whole chunks, as load_mix reads them).
template <int M, int C, typename S, int LIMIT = (C + 2) * M>
__device__ __forceinline__ void store_mix(const Mix<M, C>& m, const StateBlock& b, uint32_t p) {
  constexpr int NV = (C + 2) * M, es = sizeof(S), vpc = kChunkBytes / es, nc = NV / vpc, nf = nc * vpc,
                vpw = 4 / es;
  const uint32_t lane = p & 63u;
  const uint32_t base = (p >> 6) * b.tile_bytes;
  static_for<0, nc>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    if constexpr (c * vpc < LIMIT) {
      // a zero (not undefined) start: element 0 is then never widened into a 16-byte load
      // from the mixture, which would pin the mixture in memory
      u32x4 w = {0u, 0u, 0u, 0u};
      static_for<0, 4>([&](auto i_) RGBD_BODY {
        constexpr int i = RGBD_I(i_);
        w[i] = BufIO<S>::word(field<M, C, c * vpc + i * vpw>(m), field<M, C, c * vpc + i * vpw + vpw - 1>(m));
      });
      __builtin_amdgcn_raw_buffer_store_b128(w, b.rsrc, base + lane * kChunkBytes + c * 64u * kChunkBytes, 0, 0);
    }
  });
  static_for<nf, NV>([&](auto j_) RGBD_BODY {
    constexpr int j = RGBD_I(j_);
    if constexpr (j < LIMIT) BufIO<S>::st(b, base + tile_value_offset(j, lane, NV, es), field<M, C, j>(m));
  });
}

// The matched component's new mean, variance and weight (from the values before the update and
// the squared distance d2j of x to its mean); shared by mix_step and fast_step.
template <int C>
__device__ __forceinline__ void update_matched(float (&mj)[C], float& vj, float& wj, float d2j, const float (&x)[C],
                                               const ModelConsts& k) {
  float d2n = 0.f;
  if (k.rho_density) {  // uniform over the wave
    // rho = alpha (2 pi var)^(-C/2) exp(-d2 / (2 var)), with exp(y) = 2^(y log2 e); the
    // update is written as an increment, which keeps a rate of 1e-5 from drowning in rounding
    const float rv = __builtin_amdgcn_rcpf(vj);
    float dens = (C & 1) ? __builtin_amdgcn_rsqf(vj) : 1.f;
    static_for<0, C / 2>([&](auto) RGBD_BODY { dens *= rv; });
    const float rho = k.rho_scale * dens * __builtin_amdgcn_exp2f(-0.72134752f * d2j * rv);  // -log2(e)/2
    static_for<0, C>([&](auto c_) RGBD_BODY {
      constexpr int c = RGBD_I(c_);
      mj[c] = fmaf(rho, x[c] - mj[c], mj[c]);
      const float tt = x[c] - mj[c];
      d2n = fmaf(tt, tt, d2n);
    });
    vj = fmaxf(k.var_min, fmaf(rho, d2n - vj, vj));
  } else {
    static_for<0, C>([&](auto c_) RGBD_BODY {
      constexpr int c = RGBD_I(c_);
      mj[c] = fmaf(k.oma, mj[c], k.alpha * x[c]);
      const float tt = x[c] - mj[c];
      d2n = fmaf(tt, tt, d2n);
    });
    vj = fmaxf(k.var_min, fmaf(k.oma, vj, k.alpha * d2n));
  }
  wj = fmaf(k.oma, wj, k.alpha);
}

// Weights after the decay (w_old scaled by 1 - alpha, rank t set to tw), renormalised to sum to
// one; tw is renormalised with them. Shared by mix_step and fast_step; products and sums are
// rounded separately (never fused), so both round identically whatever they know of t.
template <int M>
__device__ __forceinline__ void renormalise(float (&w)[M], float& tw, const float (&w_old)[M], int t, float oma) {
  float S = 0.f;
  static_for<0, M>([&](auto r_) RGBD_BODY {
#pragma clang fp contract(off)
    constexpr int r = RGBD_I(r_);
    w[r] = pick(r == t, tw, oma * w_old[r]);
    S += w[r];
  });
  const float inv = 1.0f / S;
  static_for<0, M>([&](auto r_) RGBD_BODY { w[RGBD_I(r_)] *= inv; });
  tw = tw * inv;
}

// One frame of the mixture model for one pixel (Sec. III.A with the update rules of the
// paper's reference [6]). Returns the foreground bit; `j_out` is the matched rank (M if none)
// and `q_out` the rank the updated (or new) component ends up at.
//   match    : first live rank, in stored (w/sigma descending) order, with |x-mu|^2 < k^2 var
//   weights  : w <- (1-alpha) w + alpha [matched]
//   matched  : mu <- (1-rho) mu + rho x ; var <- max(var_min, (1-rho) var + rho |x-mu_new|^2), with
//              rho = alpha, or (variant) rho = alpha * N(x | mu, var I), the isotropic Gaussian
//              density of x under the matched component before its update
//   no match : the last rank becomes (x, sigma0^2, w_init)
//   then     : w <- w / sum(w); re-sort by w/sigma descending; B = min{b : w_0+...+w_{b-1} > T};
//              foreground = no match or new rank >= B
// Re-sort: the renormalisation scales every unchanged weight by the same factor, so the
// unchanged components keep their order and only the updated one (t) can be out of place. It
// walks up past neighbours with a strictly smaller key and down past neighbours with a strictly
// larger key - the stable sort of the stored order. The walk stops at the first neighbour it may
// not pass, so ranks beyond that neighbour are never consulted.
template <int M, int C>
__device__ __forceinline__ bool mix_step(Mix<M, C>& s, const float (&x)[C], const ModelConsts& k, int& j_out,
                                         int& q_out) {
  // match, in rank order
  int j = M;
  float d2j = 0.f;  // squared distance to the matched component
  static_for<0, M>([&](auto r_) RGBD_BODY {
    constexpr int r = RGBD_I(r_);
    float d2 = 0.f;
    static_for<0, C>([&](auto c_) RGBD_BODY {
      constexpr int c = RGBD_I(c_);
      const float t = x[c] - s.mu[c][r];
      d2 = fmaf(t, t, d2);
    });
    const bool hit = (s.w[r] > 0.f) & (d2 < k.k2 * s.var[r]);  // no short-circuit: no branch
    const bool take = (j == M) & hit;
    d2j = pick(take, d2, d2j);
    j = pick(take, r, j);
  });
  const bool matched = j < M;
  const int t = matched ? j : M - 1;

  // the changed component: gathered, updated once (branch-free selects over the ranks)
  float mj[C], vj = s.var[0], wj = s.w[0];
  static_for<0, C>([&](auto c_) RGBD_BODY { mj[RGBD_I(c_)] = s.mu[RGBD_I(c_)][0]; });
  static_for<1, M>([&](auto r_) RGBD_BODY {
    constexpr int r = RGBD_I(r_);
    const bool isj = (r == j);
    vj = pick(isj, s.var[r], vj);
    wj = pick(isj, s.w[r], wj);
    static_for<0, C>([&](auto c_) RGBD_BODY {
      constexpr int c = RGBD_I(c_);
      mj[c] = pick(isj, s.mu[c][r], mj[c]);
    });
  });
  update_matched<C>(mj, vj, wj, d2j, x, k);
  // no match: the least probable (last-ranked) component is replaced
  float tmu[C];
  static_for<0, C>([&](auto c_) RGBD_BODY { tmu[RGBD_I(c_)] = pick(matched, mj[RGBD_I(c_)], x[RGBD_I(c_)]); });
  const float tvar = pick(matched, vj, k.var0);
  float tw = pick(matched, wj, k.w_init);

  // decay of the other weights, renormalisation of all
  float w[M];
  renormalise<M>(w, tw, s.w, t, k.oma);

  // re-sort: walk the changed component to its place
  const float kt = tw * __builtin_amdgcn_rsqf(tvar);
  float key[M];
  static_for<0, M>([&](auto r_) RGBD_BODY { key[RGBD_I(r_)] = w[RGBD_I(r_)] * __builtin_amdgcn_rsqf(s.var[RGBD_I(r_)]); });
  int down = 0, up = 0;
  bool go_down = true, go_up = true;
  static_for<1, M>([&](auto r_) RGBD_BODY {  // ranks below t, nearest first
    constexpr int r = RGBD_I(r_);
    const bool below = r > t;
    go_down = go_down & (!below | (key[r] > kt));
    down += (below & go_down) ? 1 : 0;
  });
  static_for<0, M - 1>([&](auto i_) RGBD_BODY {  // ranks above t, nearest first
    constexpr int r = M - 2 - RGBD_I(i_);
    const bool above = r < t;
    go_up = go_up & (!above | (key[r] < kt));
    up += (above & go_up) ? 1 : 0;
  });
  const int q = t + down - up;

  // rank o takes: the changed component at q; above q the old rank o (or o+1 once past t);
  // below q the old rank o (or o-1 once past t)
  Mix<M, C> o;
  static_for<0, M>([&](auto r_) RGBD_BODY {
    constexpr int r = RGBD_I(r_);
    constexpr int rp = r > 0 ? r - 1 : 0, rn = r < M - 1 ? r + 1 : M - 1;
    const int src = r < q ? (r < t ? r : r + 1) : (r > t ? r : r - 1);
    const bool from_prev = src == r - 1, from_next = src == r + 1;
    const float v = pick(from_prev, s.var[rp], pick(from_next, s.var[rn], s.var[r]));
    const float ww = pick(from_prev, w[rp], pick(from_next, w[rn], w[r]));
    o.var[r] = pick(r == q, tvar, v);
    o.w[r] = pick(r == q, tw, ww);
    static_for<0, C>([&](auto c_) RGBD_BODY {
      constexpr int c = RGBD_I(c_);
      const float mv = pick(from_prev, s.mu[c][rp], pick(from_next, s.mu[c][rn], s.mu[c][r]));
      o.mu[c][r] = pick(r == q, tmu[c], mv);
    });
  });
  s = o;

  // background set: the first B ranks whose cumulative weight exceeds T
  int B = M;
  float run = 0.f;
  static_for<0, M>([&](auto r_) RGBD_BODY {
    constexpr int r = RGBD_I(r_);
    run += s.w[r];
    B = (B == M && run > k.T) ? r + 1 : B;
  });
  j_out = j;
  q_out = q;
  return !matched || q >= B;
}

// The frame of a pixel whose rank-0 component matches x and keeps rank 0, on the values
// load_prefix reads (all weights, rank 0, rank 1's variance). For such a pixel it computes
// exactly what mix_step computes (same helpers, same order), far more cheaply: no gather over
// the ranks, no permutation, and the pixel is background (rank 0 < B, since B >= 1). Returns
// whether the pixel is such a pixel; if not, `s` holds partial results and the caller runs
// mix_step on the whole state instead.
template <int M, int C>
__device__ __forceinline__ bool fast_step(Mix<M, C>& s, const float (&x)[C], const ModelConsts& k) {
  float d2 = 0.f;
  static_for<0, C>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    const float t = x[c] - s.mu[c][0];
    d2 = fmaf(t, t, d2);
  });
  const bool hit = (s.w[0] > 0.f) & (d2 < k.k2 * s.var[0]);
  float mj[C], vj = s.var[0], wj = s.w[0];
  static_for<0, C>([&](auto c_) RGBD_BODY { mj[RGBD_I(c_)] = s.mu[RGBD_I(c_)][0]; });
  update_matched<C>(mj, vj, wj, d2, x, k);
  float w[M];
  renormalise<M>(w, wj, s.w, 0, k.oma);
  // rank 0 keeps its place unless rank 1's key is strictly larger
  bool keeps = true;
  if constexpr (M > 1) keeps = !(w[1] * __builtin_amdgcn_rsqf(s.var[1]) > wj * __builtin_amdgcn_rsqf(vj));
  static_for<0, C>([&](auto c_) RGBD_BODY { s.mu[RGBD_I(c_)][0] = mj[RGBD_I(c_)]; });
  s.var[0] = vj;
  s.w[0] = wj;
  static_for<1, M>([&](auto r_) RGBD_BODY { s.w[RGBD_I(r_)] = w[RGBD_I(r_)]; });
  return hit & keeps;
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
