// Sanitizer driver for the oracle (test infrastructure, like the oracle):
// built with g++ -fsanitize=address,undefined by tests/test_sanitize.py and
// run there.  It calls every exported oracle function on random inputs of
// several shapes and sizes (including 0 and 1 records, digits wider than the
// remaining key bits, and rejected arguments) and checks the results against
// each other, so that an out-of-bounds access or undefined behaviour anywhere
// in them stops the run with a sanitizer report.
#include "oracle.cpp"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

namespace {

int g_fail = 0;

void expect(bool ok, const char* what, uint32_t R, uint32_t K, uint64_t n) {
  if (!ok) {
    std::fprintf(stderr, "FAIL %s R=%u K=%u n=%llu\n", what, R, K,
                 static_cast<unsigned long long>(n));
    g_fail = 1;
  }
}

}  // namespace

int main() {
  std::mt19937_64 rng(12345);
  const uint32_t shapes[][2] = {{8, 8}, {8, 1}, {16, 8}, {16, 5}, {16, 16}, {24, 16}, {32, 9}, {64, 64}};
  const uint64_t sizes[] = {0, 1, 2, 3, 17, 64, 257, 2000};
  for (const auto& sh : shapes) {
    const uint32_t R = sh[0], K = sh[1];
    for (const uint64_t n : sizes) {
      // records with few distinct keys, so that ties and equal runs occur
      std::vector<uint8_t> in(n * R), pool(16 * K);
      for (auto& b : pool) b = uint8_t(rng());
      for (uint64_t i = 0; i < n; ++i) {
        const uint64_t k = rng() % 16;
        for (uint32_t q = 0; q < R; ++q)
          in[i * R + q] = q < K ? pool[k * K + q] : uint8_t(rng());
      }
      std::vector<uint8_t> a(n * R), b(n * R), c(n * R);
      expect(oracle_sort(in.data(), a.data(), n, R, K) == ST_OK, "sort", R, K, n);
      int used = 0;
      expect(oracle_sort_parallel(in.data(), b.data(), n, R, K, 2, &used) == ST_OK, "sort_parallel",
             R, K, n);
      expect(a == b, "parallel sort differs", R, K, n);
      expect(oracle_first_unsorted(a.data(), n, R, K) == n, "first_unsorted", R, K, n);
      for (const uint32_t width : {1u, 3u, 8u, 11u}) {
        expect(oracle_msd_sort(in.data(), c.data(), n, R, K, width, width == 3 ? 2 : 32) == ST_OK,
               "msd_sort", R, K, n);
        expect(a == c, "msd_sort differs", R, K, n);
        for (const uint32_t bits : {8 * K, 8 * K - 1, width, 1u}) {
          if (bits == 0 || bits > 8 * K) continue;
          const uint32_t w = std::min(width, bits);
          std::vector<uint64_t> counts(uint64_t(1) << w), offs(uint64_t(1) << w);
          expect(oracle_histogram(in.data(), n, R, K, bits, width, counts.data()) == ST_OK,
                 "histogram", R, K, n);
          oracle_exclusive_scan(counts.data(), counts.size(), 7, offs.data());
          expect(offs[0] == 7, "scan base", R, K, n);
          expect(oracle_partition(in.data(), c.data(), n, R, K, bits, width) == ST_OK, "partition",
                 R, K, n);
        }
        for (uint32_t levels = 0; levels <= 3; ++levels) {
          const uint64_t need =
              oracle_bins_at_level(a.data(), n, R, K, width, levels, nullptr, nullptr, 0);
          std::vector<uint64_t> st(need + 1), sz(need + 1);
          const uint64_t got =
              oracle_bins_at_level(a.data(), n, R, K, width, levels, st.data(), sz.data(), need);
          expect(got == need, "bins_at_level", R, K, n);
          uint64_t total = 0;
          for (uint64_t i = 0; i < got; ++i) total += sz[i];
          expect(total == n, "bins cover the array", R, K, n);
        }
      }
      if (n <= 257) {
        expect(oracle_enum_sort(in.data(), c.data(), n, R, K) == ST_OK, "enum_sort", R, K, n);
        expect(a == c, "enum_sort differs", R, K, n);
      }
    }
  }
  // rejected arguments return an error and touch nothing
  std::vector<uint8_t> tiny(64);
  uint64_t cnt[4] = {};
  expect(oracle_validate(10, 12, 8) != ST_OK, "R not a multiple of 8", 12, 8, 10);
  expect(oracle_validate(10, 16, 0) != ST_OK, "K = 0", 16, 0, 10);
  expect(oracle_validate(10, 16, 17) != ST_OK, "K > R", 16, 17, 10);
  expect(oracle_histogram(tiny.data(), 4, 16, 8, 0, 2, cnt) != ST_OK, "bits = 0", 16, 8, 4);
  expect(oracle_histogram(tiny.data(), 4, 16, 8, 65, 2, cnt) != ST_OK, "bits > 8K", 16, 8, 4);
  expect(oracle_partition(tiny.data(), tiny.data(), 4, 16, 8, 8, 0) != ST_OK, "width = 0", 16, 8, 4);
  expect(oracle_msd_sort(tiny.data(), tiny.data(), 4, 16, 8, 17, 4) != ST_OK, "width > 16", 16, 8, 4);
  if (g_fail) return 1;
  std::puts("oracle sanitize run: ok");
  return 0;
}
