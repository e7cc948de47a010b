// Device-side building blocks of the per-pixel mixture step (gfx950, wave64).
//
// One lane owns one pixel of one modality. Its M components are loaded from the planar state
// layout (below: rows of 16-, 8- or 4-byte pieces shared by the 64 lanes of a tile, tile after
// tile, then each pixel's remaining values contiguous in a second plane, and in fp32 state one
// weight scale per tile in a third), advanced one frame in fp32 registers, re-sorted in
// registers and written back.
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
__host__ __device__ __forceinline__ void static_for(F&& f) {
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
  float dk[4];          // (1 / (1 - alpha))^(1, 2, 4, 8) in fp32: factors of hole_factor
};

// A pixel's deferred hole frames (scaled form; see the Mix comment): up to kHoleMax, held in bits
// 4-7 of the pixel's flags byte (bits 0-3 hold the List 1 state).
constexpr uint32_t kHoleShift = 4, kHoleMax = 15;

// (1 / (1 - alpha))^k for 0 <= k <= kHoleMax, as fp32 products in a fixed order, so that the host
// (reading the state) and every kernel compute the same value.
__host__ __device__ inline float hole_factor(uint32_t k, const float (&dk)[4]) {
  float d = 1.f;
  d = (k & 1u) ? d * dk[0] : d;
  d = (k & 2u) ? d * dk[1] : d;
  d = (k & 4u) ? d * dk[2] : d;
  d = (k & 8u) ? d * dk[3] : d;
  return d;
}

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
// Weights are held in one of two forms, fixed by the storage type:
//   direct (16-bit storage): w[r] is the weight itself;
//   scaled (fp32 storage):   w[r] is a scaled weight w'_r and the weight is g * w'_r, with one
//                            positive scale g shared by the 64 pixels of a tile (stored once per
//                            tile). A frame multiplies every weight by (1 - alpha); in this form
//                            that is g <- g (1 - alpha), once per tile, and only the updated
//                            component's w' changes, so a frame that keeps a pixel on its top
//                            component writes rank 0 alone. The form also stores the key of rank
//                            1 (key1 = w'_1 / sigma_1, as the re-sort computes it), which such a
//                            frame compares with rank 0's new key and never changes.
//                            A frame in which a pixel keeps its state (a depth hole) must keep
//                            each weight g * w' while g decays; instead of rescaling every w',
//                            the pixel counts such frames, k, and its weights are d * g * w' with
//                            d = (1 / (1 - alpha))^k (hole_factor): every step of the pixel works
//                            with the effective scale d * g. k returns to 0 when the tile's scale
//                            is folded, or when it would pass kHoleMax (the w' are then rescaled).
template <int M, int C>
struct Mix {
  float mu[C][M];
  float var[M];
  float w[M];
  float g;     // the tile's scale of the weights (scaled form only)
  float d;     // the pixel's hole factor (scaled form only; 1 when k = 0)
  float key1;  // rank 1's key w'_1 / sigma_1 as stored (scaled form only)
};

__host__ __device__ constexpr bool scaled_weights(uint32_t es) { return es == 4; }
template <typename S>
constexpr bool kScaled = scaled_weights(sizeof(S));

// Number of stored values per pixel: (C+2)*M, plus rank 1's key in the scaled form.
__host__ __device__ constexpr uint32_t value_count(uint32_t M, uint32_t C, uint32_t es) {
  return (C + 2) * M + (scaled_weights(es) && M > 1 ? 1u : 0u);
}

// First value of rank r's component: direct - its variance (the weights come first, apart);
// scaled - its scaled weight (rank 0's values, then rank 1's key, then ranks 1.. M-1).
__host__ __device__ constexpr uint32_t rank_first(uint32_t rank, uint32_t M, uint32_t C, uint32_t es) {
  if (scaled_weights(es)) return rank * (C + 2) + (rank > 0 ? 1u : 0u);
  return M + rank * (C + 1);
}
// Values of rank r stored from rank_first on.
__host__ __device__ constexpr uint32_t rank_values(uint32_t C, uint32_t es) {
  return scaled_weights(es) ? C + 2 : C + 1;
}

// Order of a pixel's values.
//   direct: the M weights first, then rank by rank the variance and the C means;
//   scaled: rank 0's scaled weight, variance and C means, rank 1's key, then rank by rank
//           (1 .. M-1) the scaled weight, the variance and the C means.
// The values a frame needs when the pixel matches its top-ranked component and keeps its rank
// are then a prefix: every weight, rank 0 and rank 1's variance (direct); rank 0 and rank 1's
// key (scaled).
__host__ __device__ constexpr uint32_t value_index(uint32_t param, uint32_t rank, uint32_t M, uint32_t C,
                                                   uint32_t es) {
  // param: 0..C-1 = mean channel, C = variance, C+1 = weight
  if (scaled_weights(es)) return rank_first(rank, M, C, es) + (param == C + 1 ? 0 : (param == C ? 1 : 2 + param));
  return param == C + 1 ? rank : rank_first(rank, M, C, es) + (param == C ? 0 : 1 + param);
}
// rank 1's key (scaled form, M > 1)
__host__ __device__ constexpr uint32_t key_index(uint32_t C) { return C + 2; }

// Values that are only read (not written) by the frame of a pixel that matches rank 0 and keeps
// it come after the values such a frame changes; both sets are prefixes of the value order.
//   direct: changes every weight and rank 0; also reads rank 1's variance;
//   scaled: changes rank 0; also reads rank 1's key.
__host__ __device__ constexpr uint32_t fast_store_count(uint32_t M, uint32_t C, uint32_t es) {
  return scaled_weights(es) ? C + 2 : M + (C + 1);
}
__host__ __device__ constexpr uint32_t fast_load_count(uint32_t M, uint32_t C, uint32_t es) {
  return fast_store_count(M, C, es) + (M > 1 ? 1u : 0u);
}
template <int M, int C, typename S>
constexpr int kFastLoad = static_cast<int>(fast_load_count(M, C, sizeof(S)));
template <int M, int C, typename S>
constexpr int kFastStore = static_cast<int>(fast_store_count(M, C, sizeof(S)));
template <int M, int C, typename S>
constexpr int kNV = static_cast<int>(value_count(M, C, sizeof(S)));

// One modality's state block as a buffer resource, in two planes (three in the scaled form).
// Pixels are grouped in tiles of 64 (one wave); each pixel has NV values (in value_index order).
//   hot plane  - rows holding the values a steady-state frame touches, tile after tile. Row c
//                holds values [first[c], first[c+1]) of the tile's 64 lanes as [lane][width[c]]
//                with width[c] = 16, 8 or 4 bytes, so one wave instruction moves 1 KB, 512 B or
//                256 B of contiguous memory, and the rows of consecutive tiles are contiguous
//                too. The rows end exactly where the fast path's stores end and where its loads
//                end (whole 32-bit words), so a frame on the fast path moves no value it does not
//                need;
//   cold plane - after the hot plane of all tiles: the remaining values of each pixel,
//                contiguous per pixel and padded to whole 32-bit words (sb bytes), pixel p's at
//                cold + p*sb. A pixel that leaves the fast path reads and writes its suffix as a
//                few contiguous bytes;
//   scale plane - scaled form: after the cold plane, the scale g of each tile (4 bytes).
// A frame whose pixels keep to the fast path therefore streams through one dense plane and
// skips the other. A lane's offsets are a VGPR plus compile-time constants, so each state access
// is one buffer instruction. The range checked by the hardware (num_records) is the whole block:
// an access outside it reads 0 and drops its write instead of touching other memory. The host
// keeps every block below 2 GiB, so that an offset of kNoAccess (plus a few bytes) is always
// outside: a lane that must not touch memory issues the same instruction with that offset. Loads
// and stores are thereby never skipped by a branch, and the compiler, which counts outstanding
// memory instructions to place its waits (stores included, on this GPU), can count them exactly
// and wait for just the loads a value comes from instead of for everything issued.
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, gfx9-family descriptor word 3
constexpr uint32_t kNoAccess = 0x80000000u;
__device__ __forceinline__ uint32_t at_if(bool on, uint32_t off) { return on ? off : kNoAccess; }
constexpr uint32_t kMaxRows = 8;

struct TileLayout {
  uint32_t nrows = 0;                // hot rows
  uint32_t width[kMaxRows] = {};     // bytes per lane of each row: 16, 8 or 4
  uint32_t first[kMaxRows + 1] = {};  // first value of each row; first[nrows] = nf
  uint32_t off[kMaxRows + 1] = {};    // byte offset of each row inside the tile's hot bytes
  uint32_t hot = 0;                  // hot bytes per lane (sum of the widths)
  uint32_t nf = 0;                   // values held by the hot rows
  uint32_t rest = 0;                 // values per pixel in the cold plane
  uint32_t sb = 0;                   // cold bytes per pixel (whole 32-bit words)
  uint32_t scale = 0;                // scale-plane bytes per tile (4 in the scaled form, else 0)
  uint32_t bytes = 0;                // bytes per tile of 64 pixels: 64 * (hot + sb) + scale
};

// Rows covering values [0, fast_store_count) and then [fast_store_count, fast_load_count), each
// range rounded up to whole 32-bit words and cut greedily into 16-, 8- and 4-byte rows (a 16-bit
// value left alone shares its word with the next value, or with padding past the last one).
__host__ __device__ constexpr TileLayout tile_layout(uint32_t M, uint32_t C, uint32_t es) {
  TileLayout L{};
  const uint32_t nv = value_count(M, C, es);
  const uint32_t ends[2] = {fast_store_count(M, C, es), fast_load_count(M, C, es)};
  uint32_t v = 0;
  for (uint32_t seg = 0; seg < 2; ++seg) {
    const uint32_t end = ends[seg] < nv ? ends[seg] : nv;
    while (v < end && L.nrows < kMaxRows) {
      const uint32_t left = ((end - v) * es + 3u) / 4u * 4u;  // whole 32-bit words
      const uint32_t w = left >= 16 ? 16u : (left >= 8 ? 8u : 4u);
      L.width[L.nrows] = w;
      L.first[L.nrows] = v;
      L.off[L.nrows] = 64u * L.hot;
      L.hot += w;
      ++L.nrows;
      v += w / es;
    }
  }
  L.nf = v < nv ? v : nv;
  L.first[L.nrows] = L.nf;
  L.off[L.nrows] = 64u * L.hot;
  L.rest = nv - L.nf;
  L.sb = (L.rest * es + 3u) / 4u * 4u;
  L.scale = scaled_weights(es) ? 4u : 0u;
  L.bytes = 64u * (L.hot + L.sb) + L.scale;
  return L;
}

// The layout of one (M, C, storage type), as a constant every kernel can index at compile time.
template <int M, int C, typename S>
struct Plan {
  static constexpr TileLayout L = tile_layout(M, C, sizeof(S));
  // the scalars device code uses, so that no layout object is ever built at run time
  static constexpr uint32_t nrows = L.nrows, hot = L.hot, nf = L.nf, sb = L.sb, bytes = L.bytes;
};

// Byte offset, inside a block of `tiles64` tiles, of the scale of tile `tile` (scaled form).
__host__ __device__ constexpr uint64_t state_scale_offset(uint64_t tile, uint64_t tiles64, uint32_t M, uint32_t C,
                                                          uint32_t es) {
  const TileLayout L = tile_layout(M, C, es);
  return tiles64 * 64u * (L.hot + L.sb) + 4u * tile;
}

// Byte offset, inside a block of `tiles64` tiles, of value v of pixel p.
__host__ __device__ constexpr uint64_t state_value_offset(uint32_t v, uint64_t p, uint64_t tiles64, uint32_t M,
                                                          uint32_t C, uint32_t es) {
  const TileLayout L = tile_layout(M, C, es);
  if (v >= L.nf) return tiles64 * 64u * L.hot + p * L.sb + (v - L.nf) * es;
  uint32_t c = 0;
  while (L.first[c + 1] <= v) ++c;
  return (p / 64u) * 64u * L.hot + L.off[c] + (p % 64u) * L.width[c] + (v - L.first[c]) * es;
}

// The same offset in device code, for a layout known at compile time (the row is found by
// comparisons with constants, so no layout table is built at run time).
template <int M, int C, typename S>
__host__ __device__ __forceinline__ uint64_t value_offset(uint32_t v, uint64_t p, uint64_t tiles64) {
  using P = Plan<M, C, S>;
  constexpr uint32_t es = sizeof(S);
  uint64_t off = tiles64 * 64u * P::hot + p * P::sb + static_cast<uint64_t>(v - P::nf) * es;
  static_for<0, static_cast<int>(P::nrows)>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    constexpr uint32_t a = P::L.first[c], e = P::L.first[c + 1], W = P::L.width[c], o = P::L.off[c];
    if (v >= a && v < e) off = (p / 64u) * 64u * P::hot + o + (p % 64u) * W + (v - a) * es;
  });
  return off;
}

struct StateBlock {
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t tile_rows;  // hot bytes per tile: 64 * hot
  uint32_t cold;       // byte offset of the cold plane
  uint32_t scale;      // byte offset of the scale plane (scaled form)
};

template <int M, int C, typename S>
__device__ __forceinline__ StateBlock make_block(void* base, uint32_t tiles64) {
  using P = Plan<M, C, S>;
  return StateBlock{__builtin_amdgcn_make_buffer_rsrc(base, 0, static_cast<int>(P::bytes * tiles64), kRsrcWord3),
                    64u * P::hot, tiles64 * 64u * P::hot, tiles64 * 64u * (P::hot + P::sb)};
}

// The scale of the tile holding pixel p (scaled form), the same for every lane of the wave. It
// stays a per-lane value: moving it to a scalar register would make the wave wait for every load
// issued before it, right after issuing them.
__device__ __forceinline__ float load_scale(const StateBlock& b, uint32_t p) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.rsrc, b.scale + 4u * (p >> 6), 0, 0));
}
__device__ __forceinline__ void store_scale(float g, const StateBlock& b, uint32_t p, bool on) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, g), b.rsrc, at_if(on, b.scale + 4u * (p >> 6)), 0,
                                        0);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Cache policy of the hot rows' loads and stores (the buffer instructions' cache-policy operand).
// kStream marks them non-temporal: a frame streams through every row once, and a state far
// larger than the caches would otherwise evict from them the lines that the general path's
// scattered suffix accesses and the frames could still hit. A state that fits in the last-level
// cache keeps the default policy, so that it stays there from frame to frame.
constexpr int kCached = 0;
constexpr int kStream = 2;  // nt

// One lane's words of a row (W bytes), moved by one buffer instruction of that width.
template <uint32_t W>
struct RowWords {
  uint32_t w[W / 4];
};

template <uint32_t W, int CP>
__device__ __forceinline__ RowWords<W> load_row(const __amdgpu_buffer_rsrc_t& r, uint32_t off) {
  RowWords<W> o{};
  if constexpr (W == 16) {
    const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CP);
    o.w[0] = x[0];
    o.w[1] = x[1];
    o.w[2] = x[2];
    o.w[3] = x[3];
  } else if constexpr (W == 8) {
    const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CP);
    o.w[0] = x[0];
    o.w[1] = x[1];
  } else {
    static_assert(W == 4, "rows are 16, 8 or 4 bytes per lane");
    o.w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, CP);
  }
  return o;
}

template <uint32_t W, int CP>
__device__ __forceinline__ void store_row(const RowWords<W>& o, const __amdgpu_buffer_rsrc_t& r, uint32_t off) {
  if constexpr (W == 16) {
    const u32x4 x = {o.w[0], o.w[1], o.w[2], o.w[3]};
    __builtin_amdgcn_raw_buffer_store_b128(x, r, off, 0, CP);
  } else if constexpr (W == 8) {
    const u32x2 x = {o.w[0], o.w[1]};
    __builtin_amdgcn_raw_buffer_store_b64(x, r, off, 0, CP);
  } else {
    static_assert(W == 4, "rows are 16, 8 or 4 bytes per lane");
    __builtin_amdgcn_raw_buffer_store_b32(o.w[0], r, off, 0, CP);
  }
}

template <typename S> struct BufIO;
template <> struct BufIO<float> {
  // the 32-bit word holding value a (and b, for 16-bit types, in the high half); by value, so
  // the values stay in registers
  static __device__ __forceinline__ uint32_t word(float a, float) { return __builtin_bit_cast(uint32_t, a); }
  // value `half` of a word (the lower-addressed one first); the buffer builtins move raw
  // words: reinterpret, never convert
  static __device__ __forceinline__ float from_word(uint32_t w, int) { return __builtin_bit_cast(float, w); }
};
template <> struct BufIO<f16s> {
  static __device__ __forceinline__ float from_word(uint32_t w, int half) {
    return Storage<f16s>::load(f16s{static_cast<uint16_t>(half ? (w >> 16) : (w & 0xFFFFu))});
  }
  static __device__ __forceinline__ uint32_t word(float a, float b) {
    return static_cast<uint32_t>(Storage<f16s>::pack(a).b) | (static_cast<uint32_t>(Storage<f16s>::pack(b).b) << 16);
  }
};
template <> struct BufIO<bf16s> {
  static __device__ __forceinline__ float from_word(uint32_t w, int half) {
    return __builtin_bit_cast(float, half ? (w & 0xFFFF0000u) : (w << 16));
  }
  static __device__ __forceinline__ uint32_t word(float a, float b) {
    return static_cast<uint32_t>(Storage<bf16s>::pack(a).b) | (static_cast<uint32_t>(Storage<bf16s>::pack(b).b) << 16);
  }
};

// Whether a load of values [0, LIMIT) reads value v: a row comes whole when it starts below
// LIMIT (so it may carry values at or beyond LIMIT), and the suffix comes whole when LIMIT
// reaches into it.
template <int M, int C, int LIMIT, typename S>
__host__ __device__ constexpr bool value_read(uint32_t v) {
  using P = Plan<M, C, S>;
  if (v >= P::nf) return static_cast<uint32_t>(LIMIT) > P::nf;
  uint32_t c = 0;
  while (P::L.first[c + 1] <= v) ++c;
  return P::L.first[c] < static_cast<uint32_t>(LIMIT);
}

// Every value a store of [0, SF) writes is one a load of [0, LF) read.
template <int M, int C, int LF, int SF, typename S>
__host__ __device__ constexpr bool stores_only_read() {
  for (uint32_t v = 0; v < static_cast<uint32_t>(kNV<M, C, S>); ++v)
    if (value_read<M, C, SF, S>(v) && !value_read<M, C, LF, S>(v)) return false;
  return true;
}

// Bytes of state one wave moves when its 64 lanes read (or write) values [0, LIMIT), as
// load_mix / store_mix move them.
template <int M, int C, int LIMIT, typename S>
__host__ __device__ constexpr uint32_t prefix_bytes() {
  using P = Plan<M, C, S>;
  uint32_t b = 0;
  for (uint32_t c = 0; c < P::nrows; ++c)
    if (P::L.first[c] < static_cast<uint32_t>(LIMIT)) b += 64u * P::L.width[c];
  return b + (static_cast<uint32_t>(LIMIT) > P::nf ? 64u * P::sb : 0u);
}

// Whether some row starts at or after value FROM (rows a store of [0, FROM) leaves out).
template <int M, int C, int FROM, typename S>
__host__ __device__ constexpr bool rows_from_exist() {
  using P = Plan<M, C, S>;
  for (uint32_t c = 0; c < P::nrows; ++c)
    if (P::L.first[c] >= static_cast<uint32_t>(FROM)) return true;
  return false;
}

// Value V (in value_index order) of a pixel's mixture, as the Mix field that holds it.
template <int M, int C, typename S, int V>
__device__ __forceinline__ float& field(Mix<M, C>& m) {
  if constexpr (kScaled<S>) {
    if constexpr (M > 1 && V == static_cast<int>(key_index(C))) {
      return m.key1;
    } else {
      constexpr int r = V < C + 2 ? 0 : (V - 1) / (C + 2), pos = V < C + 2 ? V : (V - 1) % (C + 2);
      if constexpr (pos == 0) return m.w[r];
      else if constexpr (pos == 1) return m.var[r];
      else return m.mu[pos - 2][r];
    }
  } else if constexpr (V < M) {
    return m.w[V];
  } else {
    constexpr int r = (V - M) / (C + 1), pos = (V - M) % (C + 1);
    if constexpr (pos == 0) return m.var[r];
    else return m.mu[pos - 1][r];
  }
}
template <int M, int C, typename S, int V>
__device__ __forceinline__ float field(const Mix<M, C>& m) {
  return field<M, C, S, V>(const_cast<Mix<M, C>&>(m));
}

// What a value not read is left at: 1 for a variance (so that keys stay finite), 0 otherwise.
template <int M, int C, typename S, int V>
__host__ __device__ constexpr float unread_value() {
  if constexpr (kScaled<S>) {
    if constexpr (M > 1 && V == static_cast<int>(key_index(C))) return 0.f;
    else return (V < C + 2 ? V : (V - 1) % (C + 2)) == 1 ? 1.f : 0.f;
  } else {
    return (V >= M && (V - M) % (C + 1) == 0) ? 1.f : 0.f;
  }
}

// Value V, or 0 past the last value (the padding half of a 16-bit word).
template <int M, int C, typename S, int V>
__device__ __forceinline__ float value_or_pad(const Mix<M, C>& m) {
  if constexpr (V < kNV<M, C, S>) return field<M, C, S, V>(m);
  else return 0.f;
}

// Row c of pixel p into the Mix (values past the last one are padding and dropped).
template <int M, int C, typename S, int c, int CP>
__device__ __forceinline__ void read_row(Mix<M, C>& m, const StateBlock& b, uint32_t base, uint32_t lane, bool on) {
  constexpr int NV = kNV<M, C, S>, vpw = 4 / static_cast<int>(sizeof(S));
  constexpr uint32_t W = Plan<M, C, S>::L.width[c], off = Plan<M, C, S>::L.off[c];
  constexpr int v0 = static_cast<int>(Plan<M, C, S>::L.first[c]);
  const RowWords<W> o = load_row<W, CP>(b.rsrc, at_if(on, base + off + lane * W));
  static_for<0, static_cast<int>(W / sizeof(S))>([&](auto i_) RGBD_BODY {
    constexpr int i = RGBD_I(i_);
    if constexpr (v0 + i < NV) field<M, C, S, v0 + i>(m) = BufIO<S>::from_word(o.w[i / vpw], i % vpw);
  });
}

// Row c of pixel p from the Mix.
template <int M, int C, typename S, int c, int CP>
__device__ __forceinline__ void write_row(const Mix<M, C>& m, const StateBlock& b, uint32_t base, uint32_t lane,
                                          bool on) {
  constexpr int vpw = 4 / static_cast<int>(sizeof(S));
  constexpr uint32_t W = Plan<M, C, S>::L.width[c], off = Plan<M, C, S>::L.off[c];
  constexpr int v0 = static_cast<int>(Plan<M, C, S>::L.first[c]);
  RowWords<W> o{};
  static_for<0, static_cast<int>(W / 4)>([&](auto k_) RGBD_BODY {
    constexpr int k = RGBD_I(k_);
    o.w[k] = BufIO<S>::word(value_or_pad<M, C, S, v0 + k * vpw>(m), value_or_pad<M, C, S, v0 + k * vpw + vpw - 1>(m));
  });
  store_row<W, CP>(o, b.rsrc, at_if(on, base + off + lane * W));
}

// Values [0, LIMIT) of pixel p, straight into the Mix (see value_read for what comes along). A
// value not read is left at 0 - a variance at 1, so that keys stay finite (any use of it is
// discarded by the caller). LIMIT = NV reads everything. A lane with `on` false reads 0s.
template <int M, int C, typename S, int LIMIT = kNV<M, C, S>, int CP = kCached>
__device__ __forceinline__ void load_mix(Mix<M, C>& m, const StateBlock& b, uint32_t p, bool on = true) {
  constexpr int NV = kNV<M, C, S>, es = sizeof(S), vpw = 4 / es;
  using P = Plan<M, C, S>;
  constexpr int nf = static_cast<int>(P::nf), nw = static_cast<int>(P::sb / 4);
  const uint32_t lane = p & 63u;
  const uint32_t base = (p >> 6) * b.tile_rows;
  static_for<0, NV>([&](auto v_) RGBD_BODY {
    constexpr int v = RGBD_I(v_);
    if constexpr (!value_read<M, C, LIMIT, S>(v)) field<M, C, S, v>(m) = unread_value<M, C, S, v>();
  });
  static_for<0, static_cast<int>(P::nrows)>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    if constexpr (static_cast<int>(Plan<M, C, S>::L.first[c]) < LIMIT) read_row<M, C, S, c, CP>(m, b, base, lane, on);
  });
  if constexpr (LIMIT > nf && nw > 0) {
    const uint32_t sbase = at_if(on, b.cold + p * P::sb);
    // whole 16-byte groups of the suffix, then single words
    static_for<0, nw / 4>([&](auto g_) RGBD_BODY {
      constexpr int g = RGBD_I(g_);
      const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(b.rsrc, sbase + 16u * g, 0, 0);
      static_for<0, 4 * vpw>([&](auto i_) RGBD_BODY {
        constexpr int i = RGBD_I(i_);
        constexpr int v = nf + (4 * g) * vpw + i;
        if constexpr (v < NV) field<M, C, S, v>(m) = BufIO<S>::from_word(w[i / vpw], i % vpw);
      });
    });
    static_for<(nw / 4) * 4, nw>([&](auto w_) RGBD_BODY {
      constexpr int wi = RGBD_I(w_);
      const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(b.rsrc, sbase + 4u * wi, 0, 0);
      static_for<0, vpw>([&](auto i_) RGBD_BODY {
        constexpr int i = RGBD_I(i_);
        constexpr int v = nf + wi * vpw + i;
        if constexpr (v < NV) field<M, C, S, v>(m) = BufIO<S>::from_word(w, i);
      });
    });
  }
}

// The values of pixel p that a load of [0, LF) did not bring: the rows from the first one
// starting at or past LF, and the suffix unless that load read it. With load_mix<LF> before it,
// the Mix holds the whole state. A lane with `on` false reads 0s.
template <int M, int C, typename S, int LF, int CP = kCached>
__device__ __forceinline__ void load_rest(Mix<M, C>& m, const StateBlock& b, uint32_t p, bool on) {
  constexpr int NV = kNV<M, C, S>, es = sizeof(S), vpw = 4 / es;
  using P = Plan<M, C, S>;
  constexpr int nf = static_cast<int>(P::nf), nw = static_cast<int>(P::sb / 4);
  const uint32_t lane = p & 63u;
  const uint32_t base = (p >> 6) * b.tile_rows;
  static_for<0, static_cast<int>(P::nrows)>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    if constexpr (static_cast<int>(Plan<M, C, S>::L.first[c]) >= LF) read_row<M, C, S, c, CP>(m, b, base, lane, on);
  });
  if constexpr (LF <= nf && nw > 0) {
    const uint32_t sbase = at_if(on, b.cold + p * P::sb);
    static_for<0, nw / 4>([&](auto g_) RGBD_BODY {
      constexpr int g = RGBD_I(g_);
      const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(b.rsrc, sbase + 16u * g, 0, 0);
      static_for<0, 4 * vpw>([&](auto i_) RGBD_BODY {
        constexpr int i = RGBD_I(i_);
        constexpr int v = nf + (4 * g) * vpw + i;
        if constexpr (v < NV) field<M, C, S, v>(m) = BufIO<S>::from_word(w[i / vpw], i % vpw);
      });
    });
    static_for<(nw / 4) * 4, nw>([&](auto w_) RGBD_BODY {
      constexpr int wi = RGBD_I(w_);
      const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(b.rsrc, sbase + 4u * wi, 0, 0);
      static_for<0, vpw>([&](auto i_) RGBD_BODY {
        constexpr int i = RGBD_I(i_);
        constexpr int v = nf + wi * vpw + i;
        if constexpr (v < NV) field<M, C, S, v>(m) = BufIO<S>::from_word(w, i);
      });
    });
  }
}

// Values [0, LIMIT) of pixel p from the Mix (whole rows and the whole suffix, as load_mix reads
// them). ROWS / SUFFIX select the parts written, so that a caller can store the rows of every
// lane with one instruction per row and the suffix of some lanes only. A lane with `on` false
// writes nothing.
template <int M, int C, typename S, int LIMIT = kNV<M, C, S>, bool ROWS = true, bool SUFFIX = true, int CP = kCached>
__device__ __forceinline__ void store_mix(const Mix<M, C>& m, const StateBlock& b, uint32_t p, bool on) {
  constexpr int es = sizeof(S), vpw = 4 / es;
  using P = Plan<M, C, S>;
  constexpr int nf = static_cast<int>(P::nf), nw = static_cast<int>(P::sb / 4);
  const uint32_t lane = p & 63u;
  const uint32_t base = (p >> 6) * b.tile_rows;
  static_for<0, static_cast<int>(P::nrows)>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    if constexpr (ROWS && static_cast<int>(Plan<M, C, S>::L.first[c]) < LIMIT)
      write_row<M, C, S, c, CP>(m, b, base, lane, on);
  });
  if constexpr (SUFFIX && LIMIT > nf && nw > 0) {
    const uint32_t sbase = at_if(on, b.cold + p * P::sb);
    static_for<0, nw / 4>([&](auto g_) RGBD_BODY {
      constexpr int g = RGBD_I(g_);
      u32x4 w = {0u, 0u, 0u, 0u};
      static_for<0, 4>([&](auto i_) RGBD_BODY {
        constexpr int i = RGBD_I(i_);
        constexpr int v = nf + (4 * g + i) * vpw;
        w[i] = BufIO<S>::word(value_or_pad<M, C, S, v>(m), value_or_pad<M, C, S, v + vpw - 1>(m));
      });
      __builtin_amdgcn_raw_buffer_store_b128(w, b.rsrc, sbase + 16u * g, 0, 0);
    });
    static_for<(nw / 4) * 4, nw>([&](auto w_) RGBD_BODY {
      constexpr int wi = RGBD_I(w_);
      constexpr int v = nf + wi * vpw;
      const uint32_t w = BufIO<S>::word(value_or_pad<M, C, S, v>(m), value_or_pad<M, C, S, v + vpw - 1>(m));
      __builtin_amdgcn_raw_buffer_store_b32(w, b.rsrc, sbase + 4u * wi, 0, 0);
    });
  }
}

// The rows of pixel p starting at or after value FROM, from the Mix: the rows a row store of
// values [0, FROM) leaves out. A lane with `on` false writes nothing.
template <int M, int C, typename S, int FROM, int CP = kCached>
__device__ __forceinline__ void store_rows_from(const Mix<M, C>& m, const StateBlock& b, uint32_t p, bool on) {
  using P = Plan<M, C, S>;
  const uint32_t lane = p & 63u;
  const uint32_t base = (p >> 6) * b.tile_rows;
  static_for<0, static_cast<int>(P::nrows)>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    if constexpr (static_cast<int>(Plan<M, C, S>::L.first[c]) >= FROM) write_row<M, C, S, c, CP>(m, b, base, lane, on);
  });
}

// Whether values [a, e) include one of rank r's (its variance or a mean; in the scaled form also
// its scaled weight).
template <int M, int C, typename S>
__host__ __device__ constexpr bool holds_rank(int a, int e, int r) {
  const int lo = static_cast<int>(rank_first(r, M, C, sizeof(S)));
  const int n = static_cast<int>(rank_values(C, sizeof(S)));
  return lo < e && lo + n > a;
}

// Suffix bytes one lane writes with store_suffix_of when only rank r changed there.
template <int M, int C, typename S>
__host__ __device__ constexpr uint32_t suffix_rank_bytes(int r) {
  constexpr int vpw = 4 / static_cast<int>(sizeof(S));
  using P = Plan<M, C, S>;
  constexpr int nf = static_cast<int>(P::nf), nw = static_cast<int>(P::sb / 4);
  uint32_t n = 0;
  for (int g = 0; g < nw / 4; ++g) n += holds_rank<M, C, S>(nf + 4 * g * vpw, nf + (4 * g + 4) * vpw, r) ? 16u : 0u;
  for (int wi = (nw / 4) * 4; wi < nw; ++wi) n += holds_rank<M, C, S>(nf + wi * vpw, nf + (wi + 1) * vpw, r) ? 4u : 0u;
  return n;
}

// The suffix of pixel p from the Mix, piece by piece as store_mix cuts it (16-byte groups, then
// words): every piece when `all`, else only the pieces holding a value of rank r; nothing when
// `on` is false. After a frame in which the updated component kept its rank r, only the weights
// (in the hot rows) and rank r changed: any other piece would rewrite the bits it holds, and each
// piece is one more write request of a lane.
template <int M, int C, typename S>
__device__ __forceinline__ void store_suffix_of(const Mix<M, C>& m, const StateBlock& b, uint32_t p, bool on, bool all,
                                                int r) {
  constexpr int NV = kNV<M, C, S>, es = sizeof(S), vpw = 4 / es;
  using P = Plan<M, C, S>;
  constexpr int nf = static_cast<int>(P::nf), nw = static_cast<int>(P::sb / 4);
  const uint32_t sbase = b.cold + p * P::sb;
  const int lo = static_cast<int>(rank_first(r, M, C, sizeof(S))), hi = lo + static_cast<int>(rank_values(C, sizeof(S)));
  auto sv = [&](auto v_) RGBD_BODY -> float {
    constexpr int v = RGBD_I(v_);
    if constexpr (v < NV) return field<M, C, S, v>(m);
    else return 0.f;
  };
  static_for<0, nw / 4>([&](auto g_) RGBD_BODY {
    constexpr int g = RGBD_I(g_);
    constexpr int a = nf + 4 * g * vpw, e = nf + (4 * g + 4) * vpw;
    const bool put = on & (all | ((lo < e) & (hi > a)));
    u32x4 w = {0u, 0u, 0u, 0u};
    static_for<0, 4>([&](auto i_) RGBD_BODY {
      constexpr int i = RGBD_I(i_);
      constexpr int v = nf + (4 * g + i) * vpw;
      w[i] = BufIO<S>::word(sv(std::integral_constant<int, v>{}), sv(std::integral_constant<int, v + vpw - 1>{}));
    });
    __builtin_amdgcn_raw_buffer_store_b128(w, b.rsrc, at_if(put, sbase + 16u * g), 0, 0);
  });
  static_for<(nw / 4) * 4, nw>([&](auto w_) RGBD_BODY {
    constexpr int wi = RGBD_I(w_);
    constexpr int v = nf + wi * vpw;
    const bool put = on & (all | ((lo < v + vpw) & (hi > v)));
    const uint32_t w = BufIO<S>::word(sv(std::integral_constant<int, v>{}), sv(std::integral_constant<int, v + vpw - 1>{}));
    __builtin_amdgcn_raw_buffer_store_b32(w, b.rsrc, at_if(put, sbase + 4u * wi), 0, 0);
  });
}

// The smallest scale the scaled form keeps; below it (and at alpha = 1, where the scale becomes
// 0) the scale is folded into the weights and the step renormalises them as plain weights.
constexpr float kMinScale = 2.3283064365386963e-10f;  // 2^-32

// The tile's scale after a frame that starts at scale g: g (1 - alpha), or 1 when that falls
// below kMinScale (the fold). Every pixel of the tile, whatever its path, ends at this value.
__device__ __forceinline__ float next_scale(float g, const ModelConsts& k) {
  const float g1 = g * k.oma;
  return g1 >= kMinScale ? g1 : 1.f;
}

// The matched component's new mean, variance and weight (from the values before the update and
// the squared distance d2j of x to its mean); shared by mix_step and fast_step. Direct weights:
// w <- (1 - alpha) w + alpha. Scaled weights: w' <- w' + inc with inc = alpha / g_new, which
// with g_new = (1 - alpha) g is the same update of g * w'.
template <int C, bool SCALED>
__device__ __forceinline__ void update_matched(float (&mj)[C], float& vj, float& wj, float d2j, const float (&x)[C],
                                               const ModelConsts& k, float inc) {
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
  if constexpr (SCALED) wj = wj + inc;
  else wj = fmaf(k.oma, wj, k.alpha);
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
// paper's reference [6]). Returns the foreground bit; `j_out` is the matched rank (M if none),
// `q_out` the rank the updated (or new) component ends up at, and `all_out` whether every
// stored scaled weight changed (the scaled form's replacement and fold-back; otherwise only rank
// q's weight, and in the direct form the weights, which all sit in the hot rows).
//   match    : first live rank, in stored (w/sigma descending) order, with |x-mu|^2 < k^2 var
//   weights  : w <- (1-alpha) w + alpha [matched]
//   matched  : mu <- (1-rho) mu + rho x ; var <- max(var_min, (1-rho) var + rho |x-mu_new|^2), with
//              rho = alpha, or (variant) rho = alpha * N(x | mu, var I), the isotropic Gaussian
//              density of x under the matched component before its update
//   no match : the last rank becomes (x, sigma0^2, w_init)
//   then     : w <- w / sum(w); re-sort by w/sigma descending; B = min{b : w_0+...+w_{b-1} > T};
//              foreground = no match or new rank >= B
// Scaled weights (SCALED): the decay of every weight is g <- (1-alpha) g, the tile's scale; the
// pixel works with its effective scale d g (d: its hole factor). After a match the weights still
// sum to one, so the renormalisation changes nothing and only the matched w' moves; after a
// replacement every w' is divided by (d g) sum(w'). Keys compare w'/sigma, the same order as
// w/sigma (one positive effective scale per pixel). The tile's new scale is left in s.g, the pixel's hole
// factor in s.d (1 after a fold) and rank 1's key in s.key1.
// Re-sort: the renormalisation scales every unchanged weight by the same factor, so the
// unchanged components keep their order and only the updated one (t) can be out of place. It
// walks up past neighbours with a strictly smaller key and down past neighbours with a strictly
// larger key - the stable sort of the stored order. The walk stops at the first neighbour it may
// not pass, so ranks beyond that neighbour are never consulted.
template <int M, int C, bool SCALED>
__device__ __forceinline__ bool mix_step(Mix<M, C>& s, const float (&x)[C], const ModelConsts& k, int& j_out,
                                         int& q_out, bool& all_out) {
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
  const float wj_old = wj;
  float g1 = 1.f, gt1 = 1.f, inc = 0.f;
  bool fold = false;
  if constexpr (SCALED) {
    gt1 = s.g * k.oma;       // the tile's next scale
    fold = !(gt1 >= kMinScale);
    g1 = gt1 * s.d;          // this pixel's next effective scale
    inc = k.alpha / g1;
  }
  update_matched<C, SCALED>(mj, vj, wj, d2j, x, k, inc);
  // no match: the least probable (last-ranked) component is replaced
  float tmu[C];
  static_for<0, C>([&](auto c_) RGBD_BODY { tmu[RGBD_I(c_)] = pick(matched, mj[RGBD_I(c_)], x[RGBD_I(c_)]); });
  const float tvar = pick(matched, vj, k.var0);
  float tw = pick(matched, wj, SCALED ? k.w_init / g1 : k.w_init);

  // decay of the other weights, renormalisation of all
  float w[M];
  float gn = 1.f;
  if constexpr (SCALED) {
    if (!fold) {
      float sum = 0.f;
      static_for<0, M>([&](auto r_) RGBD_BODY {
#pragma clang fp contract(off)
        constexpr int r = RGBD_I(r_);
        w[r] = pick(r == t, tw, s.w[r]);
        sum += w[r];
      });
      // after a replacement the weights g1 * w' sum to g1 * sum: divide every w' by that
      const float inv = matched ? 1.0f : 1.0f / (g1 * sum);
      static_for<0, M>([&](auto r_) RGBD_BODY { w[RGBD_I(r_)] *= inv; });
      tw = tw * inv;
      gn = g1;
    } else {
      // the weights as plain weights (d g w'), decayed, updated and renormalised; scale 1
      const float ge = s.g * s.d;
      float wt[M];
      static_for<0, M>([&](auto r_) RGBD_BODY { wt[RGBD_I(r_)] = ge * s.w[RGBD_I(r_)]; });
      tw = matched ? fmaf(k.oma, ge * wj_old, k.alpha) : k.w_init;
      renormalise<M>(w, tw, wt, t, k.oma);
    }
  } else {
    renormalise<M>(w, tw, s.w, t, k.oma);
  }

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
  // the tile's new scale, and the pixel's hole factor (a fold leaves plain weights: factor 1)
  o.g = SCALED && !fold ? gt1 : 1.f;
  o.d = SCALED && !fold ? s.d : 1.f;
  if constexpr (SCALED && M > 1) o.key1 = o.w[1] * __builtin_amdgcn_rsqf(o.var[1]);
  s = o;

  // background set: the first B ranks whose cumulative weight exceeds T
  int B = M;
  float run = 0.f;
  static_for<0, M>([&](auto r_) RGBD_BODY {
    constexpr int r = RGBD_I(r_);
    run += SCALED ? gn * s.w[r] : s.w[r];
    B = (B == M && run > k.T) ? r + 1 : B;
  });
  j_out = j;
  q_out = q;
  all_out = SCALED && (fold || !matched);
  return !matched || q >= B;
}

// The frame of a pixel whose rank-0 component does not match x while its rank-1 component
// does and keeps rank 1 (scaled form, the tile's scale not folding): on a mixture's second mode
// most pixels that leave the fast path are such pixels. Computes exactly what mix_step computes
// for them, with the same helpers and expressions (the matched weight moves by the increment and
// no other weight changes, so the re-sort compares the updated key with rank 0's and rank 2's
// only, and the pixel is foreground exactly when rank 0's weight alone passes T), without the
// gather over the ranks and the permutation. Returns whether the pixel is such a pixel; if so,
// `s` holds its new state and `fg` its foreground bit, else `s` is unchanged.
template <int M, int C>
__device__ __forceinline__ bool rank1_step(Mix<M, C>& s, const float (&x)[C], const ModelConsts& k, bool& fg) {
  static_assert(M > 1, "a second rank");
  float d20 = 0.f, d21 = 0.f;
  static_for<0, C>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    const float t0 = x[c] - s.mu[c][0];
    d20 = fmaf(t0, t0, d20);
    const float t1 = x[c] - s.mu[c][1];
    d21 = fmaf(t1, t1, d21);
  });
  const bool hit0 = (s.w[0] > 0.f) & (d20 < k.k2 * s.var[0]);
  const bool hit1 = (s.w[1] > 0.f) & (d21 < k.k2 * s.var[1]);
  const float gt1 = s.g * k.oma;
  const bool fold = !(gt1 >= kMinScale);
  const float g1 = gt1 * s.d;
  const float inc = k.alpha / g1;
  float mj[C], vj = s.var[1], wj = s.w[1];
  static_for<0, C>([&](auto c_) RGBD_BODY { mj[RGBD_I(c_)] = s.mu[RGBD_I(c_)][1]; });
  update_matched<C, true>(mj, vj, wj, d21, x, k, inc);
  const float kt = wj * __builtin_amdgcn_rsqf(vj);
  const bool up = s.w[0] * __builtin_amdgcn_rsqf(s.var[0]) < kt;
  bool down = false;
  if constexpr (M > 2) down = s.w[2] * __builtin_amdgcn_rsqf(s.var[2]) > kt;
  const bool ok = !hit0 & hit1 & !fold & !up & !down;
  if (ok) {
    static_for<0, C>([&](auto c_) RGBD_BODY { s.mu[RGBD_I(c_)][1] = mj[RGBD_I(c_)]; });
    s.var[1] = vj;
    s.w[1] = wj;
    s.key1 = kt;
    s.g = gt1;
    fg = g1 * s.w[0] > k.T;
  }
  return ok;
}

// The frame of a pixel that keeps its state (a depth hole), in the scaled form, when its hole
// count cannot grow (or the tile's scale folds): every w' is rescaled by its effective scale
// d g over the tile's new scale, which keeps each weight, and the hole factor returns to 1.
// Rank 1's key follows its w'.
template <int M, int C>
__device__ __forceinline__ void hold_step(Mix<M, C>& s, const ModelConsts& k) {
  const float gn = next_scale(s.g, k);
  const float f = (s.g * s.d) / gn;
  static_for<0, M>([&](auto r_) RGBD_BODY { s.w[RGBD_I(r_)] *= f; });
  s.g = gn;
  s.d = 1.f;
  if constexpr (M > 1) s.key1 = s.w[1] * __builtin_amdgcn_rsqf(s.var[1]);
}

// The frame of a pixel whose rank-0 component matches x and keeps rank 0, on the values
// load_prefix reads (direct: all weights, rank 0, rank 1's variance; scaled: the tile's scale,
// rank 0 and rank 1's stored key). For such a pixel it computes exactly what mix_step
// computes (same helpers, same order), far more cheaply: no gather over the ranks, no
// permutation, and the pixel is background (rank 0 < B, since B >= 1). Returns whether the pixel
// is such a pixel; if not, `s` holds partial results and the caller runs mix_step on the whole
// state instead. In the scaled form a scale that would fall below kMinScale also sends the pixel
// to mix_step, which folds it into the weights.
template <int M, int C, bool SCALED>
__device__ __forceinline__ bool fast_step(Mix<M, C>& s, const float (&x)[C], const ModelConsts& k) {
  float d2 = 0.f;
  static_for<0, C>([&](auto c_) RGBD_BODY {
    constexpr int c = RGBD_I(c_);
    const float t = x[c] - s.mu[c][0];
    d2 = fmaf(t, t, d2);
  });
  bool hit = (s.w[0] > 0.f) & (d2 < k.k2 * s.var[0]);
  float mj[C], vj = s.var[0], wj = s.w[0];
  static_for<0, C>([&](auto c_) RGBD_BODY { mj[RGBD_I(c_)] = s.mu[RGBD_I(c_)][0]; });
  float gt1 = 1.f, inc = 0.f;
  if constexpr (SCALED) {
    gt1 = s.g * k.oma;                  // the tile's next scale
    hit = hit & (gt1 >= kMinScale);     // a fold sends the pixel to mix_step
    inc = k.alpha / (gt1 * s.d);        // over this pixel's next effective scale
  }
  update_matched<C, SCALED>(mj, vj, wj, d2, x, k, inc);
  // rank 0 keeps its place unless rank 1's key is strictly larger
  bool keeps = true;
  if constexpr (SCALED) {
    // rank 1's key as mix_step computes it (its w' and variance are unchanged after a match of
    // rank 0, and a match leaves the weights unscaled)
    if constexpr (M > 1) keeps = !(s.key1 > wj * __builtin_amdgcn_rsqf(vj));
    s.g = gt1;
  } else {
    float w[M];
    renormalise<M>(w, wj, s.w, 0, k.oma);
    if constexpr (M > 1) keeps = !(w[1] * __builtin_amdgcn_rsqf(s.var[1]) > wj * __builtin_amdgcn_rsqf(vj));
    static_for<1, M>([&](auto r_) RGBD_BODY { s.w[RGBD_I(r_)] = w[RGBD_I(r_)]; });
  }
  static_for<0, C>([&](auto c_) RGBD_BODY { s.mu[RGBD_I(c_)][0] = mj[RGBD_I(c_)]; });
  s.var[0] = vj;
  s.w[0] = wj;
  return hit & keeps;
}

// List 1 (Sec. III.C): one transition of the fused bit I and counter cpt of a pixel.
// Encoded state byte: bits 0-2 hold cpt + 3 (0..6), bit 3 holds I; bits 4-7 (a depth pixel's
// hole count) pass through unchanged.
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
  return static_cast<uint32_t>(c + 3) | (static_cast<uint32_t>(I) << 3) | (st & 0xF0u);
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
