// Host-side check of the two-plane state layout (no GPU needed): for every compiled (M, C,
// value size) and a block of a few tiles, every value of every pixel has its own aligned bytes
// inside the block, the chunk rows of all tiles come first (row c of tile t at t*npc KB + c KB),
// the suffix of each pixel is contiguous at cold + p*sb, the fast-path prefix lies in the chunk
// rows whenever whole chunks can hold it, and the fast path's stores cover only values its loads
// read.
#include <cstdio>
#include <vector>

#include "gmm_device.hpp"

using namespace rgbd;

template <int M, int C, typename S>
static int check() {
  constexpr uint32_t es = sizeof(S), nv = (C + 2) * M;
  constexpr TileLayout L = tile_layout(M, C, es);
  constexpr uint64_t tiles = 3;
  const uint64_t block = tiles * L.bytes, cold = tiles * L.npc * kRowBytes;
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
      const uint32_t nf = L.npc * L.vpc;
      if (v >= nf && off != cold + p * L.sb + (v - nf) * es) ++bad;
      if (v < nf && off != (p / 64) * L.npc * kRowBytes + (v / L.vpc) * kRowBytes + (p % 64) * kChunkBytes +
                               (v % L.vpc) * es)
        ++bad;
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
