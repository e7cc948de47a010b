// Host-side check of the tiled state layout (no GPU needed): for every compiled (M, C, value
// size), every value of every lane of a tile has its own aligned bytes inside the tile, the
// fast-path prefix lies in the chunk rows whenever whole chunks can hold it, the suffix of each
// lane is contiguous, and the fast path's stores cover only values its loads read.
#include <cstdio>
#include <vector>

#include "gmm_device.hpp"

using namespace rgbd;

template <int M, int C, typename S>
static int check() {
  constexpr uint32_t es = sizeof(S), nv = (C + 2) * M;
  constexpr TileLayout L = tile_layout(M, C, es);
  int bad = 0;
  std::vector<int> owner(L.bytes, -1);
  for (uint32_t lane = 0; lane < 64; ++lane)
    for (uint32_t v = 0; v < nv; ++v) {
      const uint32_t off = tile_value_offset(v, lane, M, C, es);
      if (off % es || off + es > L.bytes) {
        std::printf("M=%d C=%d es=%u: value %u lane %u at %u out of tile (%u bytes)\n", M, C, es, v, lane, off, L.bytes);
        ++bad;
        continue;
      }
      for (uint32_t b = 0; b < es; ++b) {
        if (owner[off + b] != -1) {
          std::printf("M=%d C=%d es=%u: byte %u shared\n", M, C, es, off + b);
          ++bad;
        }
        owner[off + b] = static_cast<int>(lane * nv + v);
      }
      if (v >= L.npc * L.vpc && off != L.npc * kRowBytes + lane * L.sb + (v - L.npc * L.vpc) * es) ++bad;
    }
  if (L.sb % 4 || L.npc * kRowBytes + 64 * L.sb != L.bytes || L.rest * es > L.sb) ++bad;
  const uint32_t lf = fast_load_count(M, C);
  if (L.npc * L.vpc < lf && L.npc != nv / L.vpc) ++bad;   // prefix in rows whenever it fits
  if (!stores_only_read<M, C, kFastLoad<M, C>, kFastStore<M, C>, S>()) ++bad;
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
