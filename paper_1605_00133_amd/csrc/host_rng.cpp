// Host-side index generators for the sub-sampling operators (Sec. 3.1.1: random
// single points; Sec. 3.1.2 and 4.3: scrambled Hadamard patterns).
//
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) drives a Durstenfeld
// Fisher-Yates shuffle of [0, n) with unbiased bounded draws by rejection:
//   bounded(m): repeat x = next(); r = x mod m; until x - r <= 2^64 - m.
//   shuffle(n, seed): for i = n-1 down to 1: j = bounded(i+1); swap a[i], a[j].
// rSP keeps the first mc entries of shuffle(n_pix, seed), sorted; sHd takes
// shuffle(n_pix, seed) as the column scramble and the first mc entries of
// shuffle(n_pix, seed + 1), sorted, as the selected Hadamard rows.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "pat_internal.hpp"

namespace pat {

namespace {

struct SplitMix64 {
  uint64_t state;
  explicit SplitMix64(uint64_t s) : state(s) {}
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // uniform in [0, m), m >= 1
  uint64_t bounded(uint64_t m) {
    const uint64_t limit = 0ull - m;   // 2^64 - m
    for (;;) {
      const uint64_t x = next();
      const uint64_t r = x % m;
      if (x - r <= limit) return r;
    }
  }
};

std::vector<int32_t> shuffle(int32_t n, uint64_t seed) {
  std::vector<int32_t> a(n);
  for (int32_t i = 0; i < n; ++i) a[i] = i;
  SplitMix64 g(seed);
  for (int32_t i = n - 1; i >= 1; --i) {
    const int32_t j = (int32_t)g.bounded((uint64_t)i + 1);
    std::swap(a[i], a[j]);
  }
  return a;
}

}  // namespace

pat_status make_rsp_mask(int32_t n_pix, int32_t mc, uint64_t seed, int32_t* idx_out) {
  if (n_pix <= 0 || mc <= 0 || mc > n_pix || idx_out == nullptr)
    return set_error(PAT_ERR_INVALID, "pat_make_rsp_mask: need 0 < mc <= n_pix and a non-null output");
  std::vector<int32_t> a = shuffle(n_pix, seed);
  std::sort(a.begin(), a.begin() + mc);
  std::copy(a.begin(), a.begin() + mc, idx_out);
  return PAT_OK;
}

pat_status make_shd_pattern(int32_t n_pix, int32_t mc, uint64_t seed, int32_t* perm_out, int32_t* rows_out) {
  if (n_pix <= 0 || mc <= 0 || mc > n_pix || perm_out == nullptr || rows_out == nullptr)
    return set_error(PAT_ERR_INVALID, "pat_make_shd_pattern: need 0 < mc <= n_pix and non-null outputs");
  if ((n_pix & (n_pix - 1)) != 0)
    return set_error(PAT_ERR_UNSUPPORTED, "pat_make_shd_pattern: n_pix must be a power of two");
  std::vector<int32_t> perm = shuffle(n_pix, seed);
  std::copy(perm.begin(), perm.end(), perm_out);
  std::vector<int32_t> rows = shuffle(n_pix, seed + 1);
  std::sort(rows.begin(), rows.begin() + mc);
  std::copy(rows.begin(), rows.begin() + mc, rows_out);
  return PAT_OK;
}

}  // namespace pat
