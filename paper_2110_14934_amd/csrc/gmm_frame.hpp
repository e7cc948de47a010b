// The per-pixel body shared by every frame kernel (one stream per launch, or a persistent
// launch over many streams): ingest, colour and/or depth mixture step, List 1 fusion, mask
// ballots. Keeping one body makes the plain and batched paths bit-identical by construction.
#pragma once

#include <hip/hip_runtime.h>

#include "gmm_device.hpp"
#include "gmm_internal.hpp"

namespace rgbd {

// Colour pixel p of the frame, in two halves so that other loads can be issued between them.
// When rows are dense and the whole wave is inside the frame (uniform over the wave), the wave's
// 192 interleaved bytes are fetched as 48 dwords (lanes 48-63 repeat the last one), staged in
// the wave's LDS slice and de-interleaved from there; otherwise each lane reads its own three
// bytes. `p` must be inside the frame.
struct RgbLoad {
  bool staged;
  uint32_t w;           // staged: this lane's dword of the wave's bytes
  uint32_t b0, b1, b2;  // per lane: the pixel's bytes
};

// A bit that a batched launch adds to the mode of a tile whose frames are dense (a.rgb_dense and
// a.depth_dense for the modalities present): such a body reads pixel p of a frame at 3p or 2p
// bytes, with no row arithmetic and no per-stream test.
constexpr int kFramesDense = 16;

template <int CP = kCached, bool DENSE = false>
__device__ __forceinline__ RgbLoad issue_rgb_pixel(const FrameArgs& a, uint32_t p, uint32_t wave_base, int lane) {
  RgbLoad r{};
  r.staged = (DENSE || a.rgb_dense) && (wave_base + kWave <= a.npix);
  if (r.staged) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.rgb + 3 * static_cast<uint64_t>(wave_base));
    if constexpr (CP == kStream) r.w = __builtin_nontemporal_load(&src[lane < 48 ? lane : 47]);
    else r.w = src[lane < 48 ? lane : 47];
  } else {
    const uint8_t* b;
    if constexpr (DENSE) {
      b = a.rgb + 3 * static_cast<uint64_t>(p);
    } else {
      const uint32_t y = p / static_cast<uint32_t>(a.width);
      const uint32_t xx = p - y * static_cast<uint32_t>(a.width);
      b = a.rgb + static_cast<int64_t>(y) * a.rgb_pitch + 3 * xx;
    }
    r.b0 = b[0];
    r.b1 = b[1];
    r.b2 = b[2];
  }
  return r;
}

__device__ __forceinline__ void finish_rgb_pixel(const RgbLoad& r, int lane, uint32_t* lds_wave, float (&x)[3]) {
  if (r.staged) {
    if (lane < 48) lds_wave[lane] = r.w;
    wave_lds_sync();
    const uint8_t* b = reinterpret_cast<const uint8_t*>(lds_wave) + 3 * lane;
    x[0] = b[0];
    x[1] = b[1];
    x[2] = b[2];
    wave_lds_sync();  // the slice is reused by the wave's next pixels
  } else {
    x[0] = static_cast<float>(r.b0);
    x[1] = static_cast<float>(r.b1);
    x[2] = static_cast<float>(r.b2);
  }
}

// Colour pixel p, both halves at once (the four-channel path); lanes past the end read zeros.
template <int CP = kCached>
__device__ __forceinline__ void load_rgb_pixel(const FrameArgs& a, uint32_t p, uint32_t wave_base, int lane,
                                               uint32_t* lds_wave, bool valid, float (&x)[3]) {
  const RgbLoad r = issue_rgb_pixel<CP>(a, valid ? p : a.npix - 1, wave_base, lane);
  finish_rgb_pixel(r, lane, lds_wave, x);
  if (!valid) x[0] = x[1] = x[2] = 0.f;
}

template <int CP = kCached, bool DENSE = false>
__device__ __forceinline__ float load_depth_pixel(const FrameArgs& a, uint32_t p) {
  if (DENSE || a.depth_dense) {
    if constexpr (CP == kStream) return static_cast<float>(__builtin_nontemporal_load(&a.depth[p]));
    else return static_cast<float>(a.depth[p]);
  }
  const uint32_t y = p / static_cast<uint32_t>(a.width);
  const uint32_t xx = p - y * static_cast<uint32_t>(a.width);
  const uint16_t* row = reinterpret_cast<const uint16_t*>(
      reinterpret_cast<const uint8_t*>(a.depth) + static_cast<int64_t>(y) * a.depth_pitch);
  return static_cast<float>(row[xx]);
}

// The values a frame needs when the pixel matches its rank-0 component and that component keeps
// its rank (the fast-path prefix, in the hot rows): all weights, rank 0 and rank 1's variance
// (direct weights), or rank 0 and rank 1's key (scaled), and in the scaled form the tile's scale.
template <int M, int C, typename S, int CP = kCached>
__device__ __forceinline__ void load_prefix(Mix<M, C>& m, const StateBlock& blk, uint32_t p, bool valid) {
  load_mix<M, C, S, kFastLoad<M, C, S>, CP>(m, blk, p, valid);
  if constexpr (kScaled<S>) m.g = load_scale(blk, p);
}

// One modality of pixel p, with lazy state traffic decided lane by lane, on the prefix in `m`.
// fast_step is the step specialised to the case above; a lane for which that case holds writes
// back only the values that case changes (the weights and rank 0, or rank 0 alone). Any other
// lane keeps the prefix as read, loads the rest of its state, runs the full step from the
// original values and writes back what changed: the hot rows, and the whole suffix when the
// ranks were reordered (or every scaled weight changed), else only the suffix pieces of the rank
// the updated component kept. fast_step computes exactly what the full step
// computes for such a pixel, so results never depend on which path ran. `valid` lanes hold a
// pixel; `active` lanes update it (a depth hole is valid but not active: in the direct form it
// writes back what it read; in the scaled form it rescales its weights to the tile's new scale,
// hold_step). In the scaled form the tile's first lane then writes the new scale.
// In three parts, and every load and store is issued by every lane (a lane with nothing to move
// uses an offset outside the block), so no branch hides a memory instruction from the count the
// compiler keeps for its waits: step_begin runs fast_step and issues the loads of the rest of
// the state (their results are used only by lanes that take the general path); step_compute
// runs the general step on those lanes; step_store writes back. The caller issues the other
// modality's step_begin before this one's step_store, so that a wait for one modality's loads
// never waits for the other's stores.
template <int M, int C, typename S>
struct StepState {
  Mix<M, C> full;  // the whole state as read (general-path lanes)
  bool slow;       // this lane takes the general path
  bool fold;       // the tile's scale folds this frame (scaled form; uniform over the wave)
  bool fg;         // its foreground bit
  int kept;        // the rank its updated component kept, or -1 when the ranks were reordered
  uint32_t kout;   // the pixel's hole count after the frame (scaled form)
  float gnext;     // the tile's scale after the frame (scaled form)
};

// `kin`: the pixel's hole count (scaled form; 0 where the caller keeps none). With `defer`, a lane
// that keeps its state (valid, not active) only counts the frame while its count can grow and the
// tile's scale does not fold; otherwise it takes hold_step.
template <int M, int C, typename S, int CP = kCached>
__device__ __forceinline__ void step_begin(Mix<M, C>& m, StepState<M, C, S>& st, const StateBlock& blk, uint32_t p,
                                           bool valid, bool active, const float (&x)[C], const ModelConsts& k,
                                           uint32_t kin, bool defer) {
  constexpr bool SC = kScaled<S>;
  bool held = false;
  st.fold = false;
  if constexpr (SC) {
    m.d = hole_factor(kin, k.dk);
    // the same for every lane (one scale per tile): kept in a scalar register
    st.gnext = __builtin_bit_cast(
        float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, next_scale(m.g, k))));
    st.fold = !(m.g * k.oma >= kMinScale);
    held = defer && valid && !active && kin < kHoleMax && !st.fold;
  }
  st.full = m;  // the prefix as read (fast_step updates m in place)
  const bool fast = active && fast_step<M, C, SC>(m, x, k);
  st.slow = SC ? valid && !fast && !held : active && !fast;
  st.kout = held ? kin + 1 : kin;
  load_rest<M, C, S, kFastLoad<M, C, S>, CP>(st.full, blk, p, st.slow);
}

template <int M, int C, typename S>
__device__ __forceinline__ void step_compute(Mix<M, C>& m, StepState<M, C, S>& st, bool active, const float (&x)[C],
                                             const ModelConsts& k) {
  constexpr bool SC = kScaled<S>;
  st.fg = false;
  st.kept = -1;
  if (st.slow) {  // no memory access in here
    int j = M, q = M;
    bool all = true;
    if (SC && !active) {
      if constexpr (SC) hold_step<M, C>(st.full, k);
    } else {
      // a match of rank 1 that keeps its rank takes the short step; mix_step runs only for the
      // lanes it does not cover (and not at all in a wave with none)
      bool done = false;
      if constexpr (SC && M > 1) done = rank1_step<M, C>(st.full, x, k, st.fg);
      if (done) {
        j = q = 1;
        all = false;
      } else {
        st.fg = mix_step<M, C, SC>(st.full, x, k, j, q, all);
      }
    }
    st.kept = !all && (j < M ? j : M - 1) == q ? q : -1;
    // hold_step and a fold leave the weights relative to the tile's scale alone
    if (!active || st.fold) st.kout = 0;
    m = st.full;
  }
}

// The write-back; adds the state bytes the wave's lanes read and wrote to `wave_bytes`.
template <int M, int C, typename S, int CP = kCached>
__device__ __forceinline__ void step_store(const Mix<M, C>& m, const StepState<M, C, S>& st, const StateBlock& blk,
                                           uint32_t p, bool valid, uint32_t& wave_bytes) {
  constexpr int NV = kNV<M, C, S>;
  constexpr int LF = kFastLoad<M, C, S>;
  constexpr int SF = kFastStore<M, C, S>;
  static_assert(stores_only_read<M, C, LF, SF, S>(), "the fast path writes back a value it did not read");
  using P = Plan<M, C, S>;
  constexpr int NR = static_cast<int>(P::nf);  // values held by the hot rows
  constexpr bool SC = kScaled<S>;
  const bool slow = st.slow;
  const int kept = st.kept;
  // Write-back: every piece both paths write goes out in one store for all the lanes that write
  // it (a hot row then leaves the wave as one write, not as one per path). Both paths write the
  // rows the fast store covers; when the fast store reaches into the suffix (the rows cannot
  // hold the prefix), both write the suffix too. Rows past the fast store, and
  // otherwise the suffix, are the general path's alone; of the suffix, a lane whose updated
  // component kept its rank writes only the pieces holding that rank.
  constexpr bool kSuffixShared = SF > NR;
  store_mix<M, C, S, SF, true, kSuffixShared, CP>(m, blk, p, valid);
  if constexpr (rows_from_exist<M, C, SF, S>()) store_rows_from<M, C, S, SF, CP>(m, blk, p, slow);
  if constexpr (!kSuffixShared) store_suffix_of<M, C, S>(m, blk, p, slow, kept < 0, kept);
  if constexpr (SC) {  // the tile's new scale, from its first lane
    store_scale(st.gnext, blk, p, valid && (p & 63u) == 0);
    wave_bytes += 8u;
  }
  const uint32_t n_slow = __popcll(__ballot(slow)), n_valid = __popcll(__ballot(valid));
  constexpr uint32_t kFull = prefix_bytes<M, C, NV, S>() / kWave;  // a lane's whole state
  wave_bytes += (n_valid - n_slow) * ((prefix_bytes<M, C, LF, S>() + prefix_bytes<M, C, SF, S>()) / kWave);
  if constexpr (kSuffixShared) {
    wave_bytes += n_slow * 2u * kFull;
  } else {
    // read everything; write the rows, and the whole suffix or rank `kept`'s pieces of it
    wave_bytes += n_slow * (kFull + P::hot) + __popcll(__ballot(slow && kept < 0)) * P::sb;
    static_for<0, M>([&](auto r_) RGBD_BODY {
      constexpr int r = RGBD_I(r_);
      wave_bytes += __popcll(__ballot(slow && kept == r)) * suffix_rank_bytes<M, C, S>(r);
    });
  }
}

// The three parts in one, for a single modality; returns the foreground bit.
template <int M, int C, typename S, int CP = kCached>
__device__ __forceinline__ bool step_modality(Mix<M, C>& m, const StateBlock& blk, uint32_t p, bool valid,
                                              bool active, const float (&x)[C], const ModelConsts& k,
                                              uint32_t& wave_bytes) {
  StepState<M, C, S> st;
  step_begin<M, C, S, CP>(m, st, blk, p, valid, active, x, k, 0u, false);
  step_compute<M, C, S>(m, st, active, x, k);
  step_store<M, C, S, CP>(m, st, blk, p, valid, wave_bytes);
  return st.fg;
}

// The depth step's constants. The mixture parameters both modalities share (alpha, k, T, the
// new component's weight, the rate variant and the hole factors) are the same numbers in a.kc and
// a.kd (one configuration makes both); they are read from a.kc alone, so that a kernel keeps one
// copy of them in scalar registers. Only sigma0, the variance floor, the hole policy and the
// density factor are depth's own.
__device__ __forceinline__ ModelConsts depth_consts(const FrameArgs& a) {
  ModelConsts k = a.kc;
  k.var0 = a.kd.var0;
  k.var_min = a.kd.var_min;
  k.hole_skip = a.kd.hole_skip;
  k.rho_scale = a.kd.rho_scale;
  return k;
}

// Pixel p of stream `a` (p may lie past the end: such lanes only take part in the ballots).
// MODE (a compile-time combination of kModeRGB, kModeDepth, kModeFuse and kFramesDense, or kModeAug
// alone) selects the steps, so that no branch on it stands between the memory instructions. kModeAug is the
// four-channel variant:
// one mixture over (R, G, B, D8) with D8 = min(255, depth >> 4), the augmentation the paper
// describes and rejects in Sec. III.B; its mask goes to fg_rgb.
// MEASURE: the body adds the wave's state bytes to a.wave_bytes when the stream has a traffic
// record; without it the byte count is never formed (the batched launches take that body unless a
// stream of the batch records).
template <int M, typename S, int MODE, int CP, bool MEASURE = true>
__device__ __forceinline__ void process_pixel(const FrameArgs& a, uint32_t p, int lane, uint32_t* lds_wave) {
  const uint32_t wave_base = p - lane;
  const bool valid = p < a.npix;
  bool fgc = false, fgd = false;
  uint32_t wave_bytes = 0;
  if constexpr ((MODE & kModeAug) != 0) {
    const StateBlock blk = make_block<M, 4, S>(a.st_rgb, a.tiles64);
    Mix<M, 4> m;
    load_prefix<M, 4, S, CP>(m, blk, p, valid);
    const uint32_t d = valid ? static_cast<uint32_t>(load_depth_pixel<CP>(a, p)) : 0u;
    float x3[3];
    load_rgb_pixel<CP>(a, p, wave_base, lane, lds_wave, valid, x3);
    const bool active = valid && !(a.kc.hole_skip && d == 0u);
    const float x[4] = {x3[0], x3[1], x3[2], static_cast<float>(min(d >> 4, 255u))};
    const bool fg = step_modality<M, 4, S, CP>(m, blk, p, valid, active, x, a.kc, wave_bytes);
    const uint64_t bits = __ballot(fg);
    if (lane == 0 && valid) a.fg_rgb[wave_base >> 6] = bits;
  }
  constexpr bool do_c = (MODE & kModeRGB) != 0, do_d = (MODE & kModeDepth) != 0, do_f = (MODE & kModeFuse) != 0;
  const StateBlock blk_c = make_block<M, 3, S>(a.st_rgb, a.tiles64);
  const StateBlock blk_d = make_block<M, 1, S>(a.st_depth, a.tiles64);
  Mix<M, 3> mc;
  Mix<M, 1> md;
  // Every load of the pixel is issued before any result is used (the state blocks, the fusion
  // bytes and the frames do not overlap), so a wave waits for memory once, not once per step.
  // The frame bytes and the fusion byte go first and none of them sits behind a per-lane branch
  // (a lane past the end reads the last pixel instead, and writes nothing): memory results
  // count down in issue order, so the wait for the colour bytes, which the LDS staging needs at
  // once, covers only them while the state prefixes stay in flight.
  const uint32_t pc = valid ? p : a.npix - 1;
  constexpr bool dense = (MODE & kFramesDense) != 0;
  RgbLoad rl{};
  if (do_c) rl = issue_rgb_pixel<CP, dense>(a, pc, wave_base, lane);
  const float xd = do_d ? load_depth_pixel<CP, dense>(a, pc) : 0.f;
  // the flags byte: List 1 state (bits 0-3) and, in the scaled form, the depth hole count
  constexpr bool do_flags = do_f || (kScaled<S> && do_d);
  const uint32_t fst = do_flags ? a.fstate[pc] : 0u;
  if (do_c) load_prefix<M, 3, S, CP>(mc, blk_c, pc, true);
  if (do_d) load_prefix<M, 1, S, CP>(md, blk_d, pc, true);
  float x[3] = {0.f, 0.f, 0.f};
  if (do_c) finish_rgb_pixel(rl, lane, lds_wave, x);
  const ModelConsts kd = depth_consts(a);
  const bool active_d = valid && !(kd.hole_skip && xd == 0.f);
  const float x1[1] = {xd};
  // colour computed before depth's loads go out, colour written back after them
  StepState<M, 3, S> sc;
  StepState<M, 1, S> sd;
  if constexpr (do_c) {
    step_begin<M, 3, S, CP>(mc, sc, blk_c, p, valid, valid, x, a.kc, 0u, false);
    step_compute<M, 3, S>(mc, sc, valid, x, a.kc);
    fgc = sc.fg;
  }
  if constexpr (do_d) step_begin<M, 1, S, CP>(md, sd, blk_d, p, valid, active_d, x1, kd, fst >> kHoleShift, true);
  if constexpr (do_c) step_store<M, 3, S, CP>(mc, sc, blk_c, p, valid, wave_bytes);
  if constexpr (do_d) {
    step_compute<M, 1, S>(md, sd, active_d, x1, kd);
    fgd = sd.fg;
    step_store<M, 1, S, CP>(md, sd, blk_d, p, valid, wave_bytes);
  }
  // the List 1 step and the mask words last: their stores sit behind lane conditions
  bool fgf = false;
  if (do_flags && valid) {
    uint32_t st = do_f ? fuse_transition(fst, fgc, fgd) : fst;
    if constexpr (kScaled<S> && do_d) st = (st & 0x0Fu) | (sd.kout << kHoleShift);
    a.fstate[p] = static_cast<uint8_t>(st);
    fgf = do_f && ((st >> 3) & 1u);
  }
  const uint64_t bc = __ballot(fgc), bd = __ballot(fgd), bf = __ballot(fgf);
  if (lane == 0 && valid) {
    if (do_c) a.fg_rgb[wave_base >> 6] = bc;
    if (do_d) a.fg_depth[wave_base >> 6] = bd;
    if (do_f) a.fused[wave_base >> 6] = bf;
  }
  // one wave owns each entry, and launches on a handle are ordered: a plain add is exact
  if constexpr (MEASURE)
    if (a.wave_bytes != nullptr && lane == 0 && valid) a.wave_bytes[wave_base >> 6] += wave_bytes;
}

// Pixels [t0, t0 + tile_px) of stream `a` (tile_px a multiple of BLOCK; the part past the
// stream's end is skipped), BLOCK at a time, the stream's mode resolved once for the tile. A
// batched launch serves many streams, whose state together far exceeds the caches: its rows and
// frames stream (kStream).
template <int M, typename S, int MODE, int BLOCK, bool MEASURE>
__device__ __forceinline__ void process_tile_mode(const FrameArgs& a, uint32_t t0, uint32_t tile_px, int lane,
                                                  uint32_t* lds_wave) {
  for (uint32_t sub = 0; sub < tile_px; sub += BLOCK) {
    const uint32_t base = t0 + sub;
    if (base >= a.npix) break;  // uniform: the rest of the tile is past the stream's end
    process_pixel<M, S, MODE, kStream, MEASURE>(a, base + threadIdx.x, lane, lds_wave);
  }
}

template <int M, typename S, int BLOCK, bool MEASURE>
__device__ __forceinline__ void process_tile(const FrameArgs& a, uint32_t t0, uint32_t tile_px, int lane,
                                             uint32_t* lds_wave) {
  constexpr int RGBD = kModeRGB | kModeDepth, FUSED = RGBD | kModeFuse, DN = kFramesDense;
  const bool dense = ((a.mode & kModeRGB) == 0 || a.rgb_dense) && ((a.mode & kModeDepth) == 0 || a.depth_dense);
  switch (a.mode | (dense ? DN : 0)) {  // the modes a batch accepts
    case FUSED | DN: process_tile_mode<M, S, FUSED | DN, BLOCK, MEASURE>(a, t0, tile_px, lane, lds_wave); break;
    case FUSED: process_tile_mode<M, S, FUSED, BLOCK, MEASURE>(a, t0, tile_px, lane, lds_wave); break;
    case RGBD | DN: process_tile_mode<M, S, RGBD | DN, BLOCK, MEASURE>(a, t0, tile_px, lane, lds_wave); break;
    case RGBD: process_tile_mode<M, S, RGBD, BLOCK, MEASURE>(a, t0, tile_px, lane, lds_wave); break;
    case kModeRGB | DN: process_tile_mode<M, S, kModeRGB | DN, BLOCK, MEASURE>(a, t0, tile_px, lane, lds_wave); break;
    case kModeRGB: process_tile_mode<M, S, kModeRGB, BLOCK, MEASURE>(a, t0, tile_px, lane, lds_wave); break;
    case kModeDepth | DN: process_tile_mode<M, S, kModeDepth | DN, BLOCK, MEASURE>(a, t0, tile_px, lane, lds_wave); break;
    case kModeDepth: process_tile_mode<M, S, kModeDepth, BLOCK, MEASURE>(a, t0, tile_px, lane, lds_wave); break;
    default: break;
  }
}

}  // namespace rgbd
