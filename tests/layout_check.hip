// Host-side check of the two-plane state layout (no GPU needed): for every compiled (M, C,
// value size) and a block of a few tiles, every value of every pixel has its own aligned bytes
// inside the block, the hot rows of all tiles come first (row c of tile t at t*64*hot + off[c],
// lane L at + L*width[c]), rows are 16, 8 or 4 bytes per lane and end exactly at the fast path's
// store and load counts (to the 32-bit word), the suffix of each pixel is contiguous at
// cold + p*sb, the scaled form's tile scales follow the cold plane one 32-bit word per tile and
// share no byte with a value, and the fast path's stores cover only values its loads read.
#include <cstdio>
#include <vector>

#include "gmm_device.hpp"

using namespace rgbd;

static uint32_t round_words(uint32_t values, uint32_t es) { return (values * es + 3u) / 4u * 4u; }

template <int M, int C, typename S>
static int check() {
  constexpr uint32_t es = sizeof(S), nv = value_count(M, C, es);
  constexpr TileLayout L = tile_layout(M, C, es);
  constexpr uint64_t tiles = 3;
  const uint64_t block = tiles * L.bytes, cold = tiles * 64u * L.hot;
  int bad = 0;
  std::vector<int64_t> owner(block, -1);
  for (uint64_t p = 0; p < tiles * 64; ++p)
    for (uint32_t v = 0; v < nv; ++v) {
      const uint64_t off = state_value_offset(v, p, tiles, M, C, es);
      if (off % es || off + es > block) {
        std::printf("M=%d C=%d es=%u: value %u pixel %llu at %llu out of the block (%llu bytes)\n", M, C, es, v,
                    (unsigned long long)p, (unsigned long long)off, (unsigned long long)block);
        ++bad;
        continue;
      }
      for (uint32_t b = 0; b < es; ++b) {
        if (owner[off + b] != -1) {
          std::printf("M=%d C=%d es=%u: byte %llu shared\n", M, C, es, (unsigned long long)(off + b));
          ++bad;
        }
        owner[off + b] = static_cast<int64_t>(p * nv + v);
      }
      if (value_offset<M, C, S>(v, p, tiles) != off) ++bad;  // the device code's offset agrees
      if (v >= L.nf && off != cold + p * L.sb + (v - L.nf) * es) ++bad;
      if (v < L.nf) {
        uint32_t c = 0;
        while (L.first[c + 1] <= v) ++c;
        if (off != (p / 64) * 64u * L.hot + L.off[c] + (p % 64) * L.width[c] + (v - L.first[c]) * es) ++bad;
      }
    }
  // the tile scales: one aligned word per tile right after the cold plane, inside the block
  if (L.scale != (scaled_weights(es) ? 4u : 0u)) ++bad;
  for (uint64_t t = 0; L.scale && t < tiles; ++t) {
    const uint64_t off = state_scale_offset(t, tiles, M, C, es);
    if (off % 4 || off != tiles * 64u * (L.hot + L.sb) + 4u * t || off + 4 > block) {
      ++bad;
      continue;
    }
    for (uint32_t b = 0; b < 4; ++b) {
      if (owner[off + b] != -1) ++bad;
      owner[off + b] = -2;
    }
  }
  uint32_t hot = 0;
  for (uint32_t c = 0; c < L.nrows; ++c) {
    if (L.width[c] != 16 && L.width[c] != 8 && L.width[c] != 4) ++bad;
    if (L.off[c] != 64u * hot || (L.first[c + 1] - L.first[c]) * es > L.width[c]) ++bad;
    hot += L.width[c];
  }
  if (hot != L.hot || L.sb % 4 || 64u * (L.hot + L.sb) + L.scale != L.bytes || L.rest * es > L.sb ||
      L.nf + L.rest != nv)
    ++bad;
  // the rows end where the fast path's stores end and where its loads end (whole words)
  const uint32_t sf = fast_store_count(M, C, es), lf = fast_load_count(M, C, es);
  bool store_end = false, load_end = false;
  for (uint32_t c = 0; c <= L.nrows; ++c) {
    if (64u * round_words(sf, es) == L.off[c]) store_end = true;
    if (64u * round_words(lf, es) == L.off[c]) load_end = true;
  }
  if (!store_end || !load_end) {
    std::printf("M=%d C=%d es=%u: rows do not end at the fast store (%u) and load (%u) counts\n", M, C, es, sf, lf);
    ++bad;
  }
  if (!stores_only_read<M, C, kFastLoad<M, C, S>, kFastStore<M, C, S>, S>()) ++bad;
  // every (parameter, rank) has its own value, and the scaled form's key of rank 1 one more
  std::vector<int> seen(nv, 0);
  for (uint32_t param = 0; param < C + 2; ++param)
    for (uint32_t r = 0; r < M; ++r) {
      const uint32_t v = value_index(param, r, M, C, es);
      ++seen[v];
      // a rank's values lie in [rank_first, rank_first + rank_values)
      if (v < rank_first(r, M, C, es) || v >= rank_first(r, M, C, es) + rank_values(C, es)) {
        if (param != C + 1 || scaled_weights(es)) ++bad;  // direct weights sit apart
      }
    }
  if (scaled_weights(es) && M > 1) ++seen[key_index(C)];
  for (uint32_t v = 0; v < nv; ++v)
    if (seen[v] != 1) ++bad;
  return bad;
}

template <int C, typename S>
static int check_all_m() {
  return check<1, C, S>() + check<2, C, S>() + check<3, C, S>() + check<4, C, S>() + check<5, C, S>();
}

int main() {
  const int bad = check_all_m<1, float>() + check_all_m<3, float>() + check_all_m<4, float>() +
                  check_all_m<1, f16s>() + check_all_m<3, f16s>() + check_all_m<4, f16s>();
  std::printf(bad ? "FAILED %d\n" : "layout ok\n", bad);
  return bad ? 1 : 0;
}
