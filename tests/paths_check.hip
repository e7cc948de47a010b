// The short steps against the general step, on the GPU: fast_step and rank1_step must compute
// bit for bit what mix_step computes for every pixel they take (and rank1_step must take nearly
// every pixel whose rank-1 component matches and keeps its rank). Random mixtures (keys sorted,
// some empty ranks, scales over six decades, hole counts 0..15, inputs near rank 0 or rank 1),
// for M in {2, 3, 5} and C in {1, 3, 4}, with rho = alpha and the density rate, in the scaled
// form (fp32 state), and fast_step against mix_step in the direct form. Built by the package's
// build step; prints one line per case and "paths ok" when every case holds.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "gmm_device.hpp"

using namespace rgbd;

#define CK(x)                                                                     \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 2;                                                                   \
    }                                                                             \
  } while (0)

__device__ __forceinline__ uint32_t mixbits(uint32_t x) {  // a 32-bit integer hash (lowbias32)
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ float u01(uint32_t& s) {
  s = mixbits(s + 0x9e3779b9u);
  return static_cast<float>(s >> 8) * (1.0f / 16777216.0f);
}
__device__ __forceinline__ bool same(float a, float b) { return __float_as_uint(a) == __float_as_uint(b); }

template <int M, int C>
__device__ bool same_mix(const Mix<M, C>& a, const Mix<M, C>& b, bool scaled) {
  bool ok = true;
  for (int r = 0; r < M; ++r) {
    ok = ok && same(a.w[r], b.w[r]) && same(a.var[r], b.var[r]);
    for (int c = 0; c < C; ++c) ok = ok && same(a.mu[c][r], b.mu[c][r]);
  }
  if (scaled) ok = ok && same(a.g, b.g) && same(a.d, b.d) && (M < 2 || same(a.key1, b.key1));
  return ok;
}

// counts: 0 fast claims, 1 fast mismatches, 2 rank1 claims, 3 rank1 mismatches,
// 4 general steps that matched rank 1 and kept it (no fold)
template <int M, int C, bool SCALED>
__global__ void __launch_bounds__(256) check_kernel(ModelConsts k, uint32_t seed, uint32_t n,
                                                    unsigned long long* counts) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  uint32_t s = mixbits(seed ^ (i * 2654435761u));
  Mix<M, C> m{};
  float sum = 0.f;
  for (int r = 0; r < M; ++r) {
    m.w[r] = (r > 0 && u01(s) < 0.1f) ? 0.f : 0.02f + 2.f * u01(s);
    m.var[r] = 4.f + 396.f * u01(s);
    for (int c = 0; c < C; ++c) m.mu[c][r] = 255.f * u01(s);
    sum += m.w[r];
  }
  if (!SCALED)
    for (int r = 0; r < M; ++r) m.w[r] /= sum;
  // ranks in key order (w / sigma descending), empty ranks last
  for (int a = 1; a < M; ++a)
    for (int b = a; b > 0; --b) {
      const float kb = m.w[b] * __builtin_amdgcn_rsqf(m.var[b]), ka = m.w[b - 1] * __builtin_amdgcn_rsqf(m.var[b - 1]);
      if (!(kb > ka)) break;
      float t = m.w[b]; m.w[b] = m.w[b - 1]; m.w[b - 1] = t;
      t = m.var[b]; m.var[b] = m.var[b - 1]; m.var[b - 1] = t;
      for (int c = 0; c < C; ++c) { t = m.mu[c][b]; m.mu[c][b] = m.mu[c][b - 1]; m.mu[c][b - 1] = t; }
    }
  m.g = SCALED ? exp2f(-20.f * u01(s)) : 1.f;
  m.g = (SCALED && u01(s) < 0.02f) ? 1e-10f : m.g;  // a tile about to fold
  const uint32_t kk = u01(s) < 0.3f ? (mixbits(s) & 15u) : 0u;
  m.d = SCALED ? hole_factor(kk, k.dk) : 1.f;
  if (M > 1) m.key1 = m.w[1] * __builtin_amdgcn_rsqf(m.var[1]);
  // an input near rank 0 or rank 1 (up to about 2.6 sigma away per channel)
  const int rr = (M > 1 && u01(s) < 0.5f) ? 1 : 0;
  float x[C];
  for (int c = 0; c < C; ++c) x[c] = m.mu[c][rr] + sqrtf(m.var[rr]) * (u01(s) * 2.6f - 1.3f);

  Mix<M, C> ref = m;
  int j = M, q = M;
  bool all = false;
  const bool fg_ref = mix_step<M, C, SCALED>(ref, x, k, j, q, all);
  const bool fold = SCALED && !(m.g * k.oma >= kMinScale);

  Mix<M, C> f = m;
  if (fast_step<M, C, SCALED>(f, x, k)) {
    atomicAdd(&counts[0], 1ull);
    // the fast path writes rank 0 (and the weights, direct form); the rest stays as read
    Mix<M, C> expect = f;
    if (SCALED) expect.key1 = m.key1;
    const bool ok = j == 0 && q == 0 && !fg_ref && same_mix(expect, ref, SCALED);
    if (!ok) atomicAdd(&counts[1], 1ull);
  }
  if constexpr (SCALED && M > 1) {
    Mix<M, C> r1 = m;
    bool fg1 = false;
    if (rank1_step<M, C>(r1, x, k, fg1)) {
      atomicAdd(&counts[2], 1ull);
      const bool ok = j == 1 && q == 1 && fg1 == fg_ref && same_mix(r1, ref, true);
      if (!ok) atomicAdd(&counts[3], 1ull);
    }
    if (j == 1 && q == 1 && !fold) atomicAdd(&counts[4], 1ull);
  }
}

static ModelConsts consts(float alpha, int C, bool density) {
  ModelConsts k{};
  k.alpha = alpha;
  k.oma = 1.0f - alpha;
  k.k2 = 2.5f * 2.5f;
  k.T = 0.7f;
  k.var0 = 900.f;
  k.var_min = 4.f;
  k.w_init = 0.05f;
  k.hole_skip = 1;
  k.rho_density = density ? 1 : 0;
  k.rho_scale = static_cast<float>(alpha * std::pow(2.0 * M_PI, -0.5 * C));
  k.dk[0] = 1.0f / k.oma;
  k.dk[1] = k.dk[0] * k.dk[0];
  k.dk[2] = k.dk[1] * k.dk[1];
  k.dk[3] = k.dk[2] * k.dk[2];
  return k;
}

template <int M, int C, bool SCALED>
static int run(unsigned long long* d_counts, float alpha, bool density, uint32_t seed) {
  const uint32_t n = 1u << 20;
  CK(hipMemset(d_counts, 0, 8 * sizeof(unsigned long long)));
  check_kernel<M, C, SCALED><<<dim3(n / 256), dim3(256)>>>(consts(alpha, C, density), seed, n, d_counts);
  CK(hipGetLastError());
  unsigned long long h[8];
  CK(hipMemcpy(h, d_counts, sizeof(h), hipMemcpyDeviceToHost));
  const bool cover = !(SCALED && M > 1) || h[2] >= h[4] - h[4] / 100;  // at least 99% of the rank-1 cases
  const bool ok = h[1] == 0 && h[3] == 0 && cover && h[0] > 0 && (!(SCALED && M > 1) || h[2] > 0);
  std::printf("M=%d C=%d %s alpha=%g rho=%s: fast %llu (bad %llu), rank1 %llu (bad %llu) of %llu rank-1 cases: %s\n",
              M, C, SCALED ? "scaled" : "direct", alpha, density ? "density" : "alpha", h[0], h[1], h[2], h[3], h[4],
              ok ? "ok" : "FAILED");
  return ok ? 0 : 1;
}

int main() {
  unsigned long long* d = nullptr;
  CK(hipMalloc(&d, 8 * sizeof(unsigned long long)));
  int bad = 0;
  bad += run<2, 1, true>(d, 0.01f, false, 11u);
  bad += run<3, 3, true>(d, 0.05f, false, 12u);
  bad += run<5, 3, true>(d, 0.01f, false, 13u);
  bad += run<5, 1, true>(d, 0.01f, false, 14u);
  bad += run<5, 4, true>(d, 0.02f, false, 15u);
  bad += run<5, 3, true>(d, 0.01f, true, 16u);
  bad += run<5, 1, true>(d, 0.05f, true, 17u);
  bad += run<5, 3, false>(d, 0.01f, false, 18u);
  bad += run<3, 1, false>(d, 0.05f, false, 19u);
  CK(hipFree(d));
  std::printf(bad ? "paths FAILED (%d cases)\n" : "paths ok\n", bad);
  return bad ? 1 : 0;
}
