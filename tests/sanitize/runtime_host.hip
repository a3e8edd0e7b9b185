// Host-side sanitizer driver for libraduls's runtime (test infrastructure):
// tests/test_sanitize.py compiles it with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side only and runs it on the CPU;
// it launches nothing.  It includes the runtime's source and stands in for
// the kernel launchers, then drives the size queries, the workspace layout
// for many shapes and tunings (every region inside the workspace, in order,
// and each region's last element written through the layout's pointers into
// a host buffer of exactly the planned size), and the argument checks of
// every entry point.
#include "raduls_runtime.hip"

#include <cstdio>
#include <vector>

namespace raduls {
#define RADULS_STUB(N)                                                                     \
  hipError_t run_rw##N(const Params&, uint32_t, hipStream_t) { return hipErrorInvalidValue; } \
  hipError_t serve_rw##N(const Params&, uint32_t, uint32_t, hipStream_t) {                  \
    return hipErrorInvalidValue;                                                            \
  }
RADULS_STUB(1)
RADULS_STUB(2)
RADULS_STUB(3)
RADULS_STUB(4)
RADULS_STUB(5)
RADULS_STUB(6)
RADULS_STUB(7)
RADULS_STUB(8)
#undef RADULS_STUB
}  // namespace raduls

namespace {
int g_fail = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL %s\n", what);
    g_fail = 1;
  }
}
template <class T>
void touch_last(T* p, uint64_t count) {
  if (count) std::memset(static_cast<void*>(p + (count - 1)), 0xA5, sizeof(T));
}
}  // namespace

int main() {
  using namespace raduls;
  const uint64_t ns[] = {0, 1, 2, 63, 5000, 5121, 40000, 1ull << 20, 1ull << 24};
  raduls_tuning tunings[6] = {};
  tunings[1].digit_bits = 3;
  tunings[2].mid_max = 64;
  tunings[2].tiny_max = 256;
  tunings[3].lookback = 1;
  tunings[3].tile_items = 2;
  tunings[4].digit_bits = 8;
  tunings[4].pair_hist = 2;
  tunings[4].wave_job_max = 1;
  tunings[5].es_job_max = 256;
  tunings[5].wave_job_max = 64;
  for (uint32_t R = 8; R <= 64; R += 8) {
    for (uint32_t K : {1u, 5u, 8u, 9u, 16u, 64u}) {
      if (K > R) continue;
      for (const auto& t : tunings) {
        expect(raduls_set_tuning(&t) == RADULS_OK, "set_tuning");
        const Eff e = effective(current_tuning(), R, K);
        expect(e.mid_max >= 64 && e.mid_max <= mid_capacity(R / 8, (K + 7) / 8), "mid_max range");
        for (uint64_t n : ns) {
          uint64_t bytes = 0;
          expect(raduls_tmp_bytes(n, R, K, &bytes) == RADULS_OK, "tmp_bytes");
          expect(bytes >= n * R, "tmp covers the records");
          for (int variant = 0; variant < 4; ++variant) {
            const bool step = variant == 1, pair = variant == 2;
            const uint32_t count = variant == 3 ? 7u : 1u;
            const Shape s = plan_shape(n, count, R, K, e, step, pair);
            const uint64_t offs[] = {s.off_ctrl,  s.off_arrays, s.off_large[0], s.off_large[1],
                                     s.off_hist[0], s.off_hist[1], s.off_diff[0], s.off_diff[1],
                                     s.off_eqkey[0], s.off_eqkey[1], s.off_tp, s.off_tb,
                                     s.off_status, s.off_tail, s.off_carry, s.off_flag,
                                     s.off_mid, s.off_tiny, s.off_pair_part,
                                     s.off_pair_hist, s.off_pair_d1, s.bytes};
            for (size_t i = 1; i < sizeof(offs) / sizeof(offs[0]); ++i)
              expect(offs[i - 1] <= offs[i] && offs[i] % 256 == 0, "regions in order, aligned");
            if (s.bytes > (256ull << 20)) continue;
            std::vector<uint8_t> aux(s.bytes);
            const Layout L = make_layout(aux.data(), s);
            touch_last(L.ctrl, 1);
            touch_last(L.arrays, count);
            for (int i = 0; i < 2; ++i) {
              touch_last(L.large[i], s.cap_large);
              touch_last(L.hist[i], uint64_t(s.cap_large) * kRadix);
              touch_last(L.diff[i], uint64_t(s.cap_large) * 8);
              if (s.eq_split) touch_last(L.eqkey[i], uint64_t(s.cap_large) * 8);
            }
            touch_last(L.tile_prefix, uint64_t(s.cap_large) + 1);
            touch_last(L.tile_bin, s.cap_tiles);
            touch_last(L.status, uint64_t(e.lookback ? s.cap_tiles : 1) * kRadix);
            touch_last(L.wg_tail, uint64_t(s.cap_ranges) * kRadix);
            touch_last(L.wg_carry, uint64_t(s.cap_ranges) * kRadix);
            touch_last(L.wg_flag, s.cap_ranges);
            touch_last(L.mid, s.cap_mid);
            touch_last(L.tiny, s.cap_mid);
            if (pair) {
              touch_last(L.pair_part,
                         std::min<uint64_t>(s.cap_ranges, kPairRanges) * kPairWords);
              touch_last(L.pair_hist, 2ull * kPairWords);
              touch_last(L.pair_d1, kRadix);
            }
          }
        }
      }
    }
  }
  raduls_tuning none = {};
  expect(raduls_set_tuning(&none) == RADULS_OK, "reset tuning");
  // argument checks that return before any device work
  uint64_t b = 0;
  expect(raduls_tmp_bytes(1ull << 32, 16, 8, &b) == RADULS_E_UNSUPPORTED, "n >= 2^32");
  expect(raduls_tmp_bytes(10, 12, 8, &b) == RADULS_E_UNSUPPORTED, "R not a multiple of 8");
  expect(raduls_tmp_bytes(10, 16, 0, &b) == RADULS_E_INVALID, "K = 0");
  expect(raduls_sort(nullptr, nullptr, 100, 16, 8, nullptr) == RADULS_E_INVALID, "null recs");
  expect(raduls_sort(reinterpret_cast<void*>(4096 + 8), reinterpret_cast<void*>(1 << 30), 100, 16,
                     8, nullptr) == RADULS_E_ALIGN,
         "misaligned recs");
  expect(raduls_sort(reinterpret_cast<void*>(1 << 20), reinterpret_cast<void*>((1 << 20) + 256), 100,
                     16, 8, nullptr) == RADULS_E_INVALID,
         "overlapping tmp");
  expect(raduls_sort(nullptr, nullptr, 1, 16, 8, nullptr) == RADULS_OK, "n = 1 is a no-op");
  expect(raduls_batch_ws_bytes(0, 0, 16, 8, &b) == RADULS_OK, "empty batch size");
  expect(raduls_sort_batch(nullptr, 5, 100, 16, 8, nullptr, 0, nullptr) == RADULS_E_INVALID,
         "batch without descriptors");
  expect(raduls_step_ws_bytes(1000, 16, 8, &b) == RADULS_OK, "step size");
  expect(raduls_histogram(nullptr, 10, 16, 8, 8, 9, nullptr, nullptr, 0, nullptr) ==
             RADULS_E_INVALID,
         "digit width 9");
  raduls_tuning bad = {};
  bad.wave_job_max = 1000;
  expect(raduls_set_tuning(&bad) == RADULS_E_INVALID, "wave_job_max too large");
  uint64_t cap = 0;
  expect(raduls_server_max_records(16, 8, &cap) == RADULS_OK && cap == 5120, "server capacity");
  raduls_server* srv = nullptr;
  expect(raduls_server_create(16, 8, 0, 1, 10, 0, &srv) == RADULS_E_INVALID && !srv, "server slots 0");
  expect(raduls_server_destroy(nullptr) == RADULS_E_INVALID, "destroy null");
  for (int st = 0; st >= -10; --st)
    expect(std::strcmp(raduls_strerror(st), "unknown status") != 0, "strerror");
  if (g_fail) return 1;
  std::puts("runtime host sanitize run: ok");
  return 0;
}
