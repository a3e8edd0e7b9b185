// Host runtime and C ABI of libraduls: argument validation, workspace
// layout, tuning, launch shapes.  Never allocates, frees or synchronizes in
// the sort calls.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <cstring>
#include <mutex>
#include <vector>

#include "raduls.h"
#include "raduls_common.hpp"

namespace raduls {
struct ProfileEvents {
  hipEvent_t ev[2 * kProfileSlots];
  uint32_t count;
};
ProfileEvents g_profile = {};

hipError_t run_rw1(const Params&, uint32_t, hipStream_t);
hipError_t run_rw2(const Params&, uint32_t, hipStream_t);
hipError_t run_rw3(const Params&, uint32_t, hipStream_t);
hipError_t run_rw4(const Params&, uint32_t, hipStream_t);
hipError_t run_rw5(const Params&, uint32_t, hipStream_t);
hipError_t run_rw6(const Params&, uint32_t, hipStream_t);
hipError_t run_rw7(const Params&, uint32_t, hipStream_t);
hipError_t run_rw8(const Params&, uint32_t, hipStream_t);
hipError_t serve_rw1(const Params&, uint32_t, uint32_t, hipStream_t);
hipError_t serve_rw2(const Params&, uint32_t, uint32_t, hipStream_t);
hipError_t serve_rw3(const Params&, uint32_t, uint32_t, hipStream_t);
hipError_t serve_rw4(const Params&, uint32_t, uint32_t, hipStream_t);
hipError_t serve_rw5(const Params&, uint32_t, uint32_t, hipStream_t);
hipError_t serve_rw6(const Params&, uint32_t, uint32_t, hipStream_t);
hipError_t serve_rw7(const Params&, uint32_t, uint32_t, hipStream_t);
hipError_t serve_rw8(const Params&, uint32_t, uint32_t, hipStream_t);

namespace {

raduls_tuning g_tuning = {};
std::mutex g_tuning_mu;

raduls_tuning current_tuning() {
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  return g_tuning;
}

uint32_t mid_capacity(uint32_t rw, uint32_t kw) { return mid_cap(int(rw), int(kw)); }

struct Eff {  // tuning after defaults and clamps, for one record width
  uint32_t digit_bits, tiny_max, mid_max, tile, nontemporal, grid_blocks, lookback, pair_hist;
  uint32_t wave_job, es_job;
};

Eff effective(const raduls_tuning& t, uint32_t R, uint32_t K) {
  const uint32_t rw = R / 8;
  Eff e;
  e.digit_bits = t.digit_bits ? std::min<uint32_t>(std::max<uint32_t>(t.digit_bits, 1), 8) : 8;
  const uint32_t cap = mid_capacity(rw, (K + 7) / 8);
  e.mid_max = t.mid_max ? std::min(t.mid_max, cap) : cap;
  e.tiny_max = t.tiny_max ? std::min<uint32_t>(std::max<uint32_t>(t.tiny_max, 1), 256) : 64;
  // ranges waiting for an LDS pass are disjoint and larger than tiny_max
  // (wave passes) or than one wave's capacity (workgroup passes), so these
  // bound their number by the LDS list capacities
  e.tiny_max = std::max<uint32_t>(e.tiny_max, (e.mid_max + kMidListCap - 1) / kMidListCap);
  const uint32_t items = uint32_t(scatter_items(int(rw)));
  e.tile = uint32_t(kScatterBlock) * (t.tile_items ? std::min(t.tile_items, items) : items);
  e.nontemporal = t.nontemporal ? t.nontemporal : 1;
  e.grid_blocks = t.grid_blocks;
  e.lookback = t.lookback ? 1 : 0;
  e.pair_hist = t.pair_hist == 2 ? 0 : 1;
  const uint32_t wmax = tiny_job_max(int(rw), int((K + 7) / 8));
  e.wave_job = t.wave_job_max ? std::min(t.wave_job_max, wmax) : wmax;
  if (e.wave_job == 1) e.wave_job = 0;  // off: every job goes to the LDS sorter
  e.es_job = std::min(t.es_job_max ? t.es_job_max : kMidDirectEs, e.tiny_max);
  return e;
}

// Whether a single-array sort of n records counts digit pairs at the top
// level: 8-bit digits, at least two key bytes, the carry-scan scatter, and
// enough records that the second round's bins are likely large.
bool use_pair(const Eff& e, uint64_t n, uint32_t K) {
  return e.pair_hist && e.digit_bits == 8 && K >= 2 && !e.lookback &&
         n > 256ull * uint64_t(e.mid_max);
}

struct Shape {
  uint32_t cap_large, cap_tiles, cap_mid, cap_ranges, rounds, pair;
  uint32_t eq_split;
  uint64_t off_ctrl, off_arrays, off_large[2], off_hist[2], off_diff[2], off_eqkey[2], off_tp, off_tb,
      off_status,
      off_tail, off_carry, off_flag, off_mid, off_tiny, off_pair_part, off_pair_hist, off_pair_d1,
      bytes;
};

// Capacities of the device lists.  Large bins of one round are disjoint and
// hold more than mid_max records each; every round consumes at least one key
// bit per bin, so there are at most ceil(8K / digit_bits) rounds.  LDS jobs:
// a parent's greedy packing yields at most 2*small/mid_max + (large children)
// + 2 jobs; copy jobs (finished runs left in tmp, on the same list): every
// record is copied at most once, each run in pieces of at most mid_max.
Shape plan_shape(uint64_t n_total, uint32_t count, uint32_t R, uint32_t K, const Eff& e,
                 bool step, bool pair = false) {
  Shape s{};
  s.pair = pair ? 1 : 0;
  const uint64_t T = e.mid_max;
  s.rounds = step ? 1 : (8 * K + e.digit_bits - 1) / e.digit_bits;
  // many records: dominated bins may be split on an equality key, which
  // takes a round but no key bit.  Below 256 * mid_max records the top
  // level alone leaves bins of about mid_max records, and a heavy key's run
  // is cheap to isolate by digits, so those sorts launch no rounds for it.
  s.eq_split = !step && n_total > 256ull * T ? 1u : 0u;
  if (s.eq_split) s.rounds += kEqRounds;
  const uint64_t large = step ? 1 : n_total / (T + 1) + 1;
  const uint64_t tiles = n_total / e.tile + large + 1;
  // (plus copy jobs: finished runs left in tmp, at most mid_max records each)
  const uint64_t mid = step ? 1
                            : 3 * (n_total / std::max<uint64_t>(T, 1) + 1) + 4ull * s.rounds * large +
                                  count + 32;
  s.cap_large = uint32_t(std::min<uint64_t>(large, 0xFFFFFFFFull));
  s.cap_tiles = uint32_t(std::min<uint64_t>(tiles, 0xFFFFFFFFull));
  s.cap_mid = uint32_t(std::min<uint64_t>(mid, 0xFFFFFFFFull));
  s.cap_ranges = uint32_t(std::min<uint64_t>(tiles, kMaxRanges));
  // look-back status rows are needed only when that scatter is selected
  const uint64_t status_rows = e.lookback ? s.cap_tiles : 1;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  s.off_ctrl = take(sizeof(Ctrl));
  s.off_arrays = take(uint64_t(std::max<uint32_t>(count, 1)) * sizeof(ArrayDesc));
  for (int i = 0; i < 2; ++i) s.off_large[i] = take(uint64_t(s.cap_large) * sizeof(Bin));
  for (int i = 0; i < 2; ++i) s.off_hist[i] = take(uint64_t(s.cap_large) * kRadix * 4);
  for (int i = 0; i < 2; ++i) s.off_diff[i] = take(uint64_t(s.cap_large) * 8 * 8);
  for (int i = 0; i < 2; ++i) s.off_eqkey[i] = take(s.eq_split ? uint64_t(s.cap_large) * 8 * 8 : 0);
  s.off_tp = take((uint64_t(s.cap_large) + 1) * 4);
  s.off_tb = take(uint64_t(s.cap_tiles) * 4);
  s.off_status = take(status_rows * kRadix * 8);
  s.off_tail = take(uint64_t(s.cap_ranges) * kRadix * 4);
  s.off_carry = take(uint64_t(s.cap_ranges) * kRadix * 4);
  s.off_flag = take(uint64_t(s.cap_ranges) * 4);
  s.off_mid = take(uint64_t(s.cap_mid) * sizeof(MidJob));
  s.off_tiny = take(uint64_t(s.cap_mid) * sizeof(MidJob));
  // per-range pair counts, one row per histogram workgroup (at most
  // kPairRanges of them when pairs are counted), and their sum
  const uint64_t pair_rows = pair ? std::min<uint64_t>(s.cap_ranges, kPairRanges) : 0;
  s.off_pair_part = take(pair_rows * kPairWords * 4);
  s.off_pair_hist = take(pair ? 2ull * kPairWords * 4 : 0);
  s.off_pair_d1 = take(pair ? kRadix * 4 : 0);
  s.bytes = o;
  return s;
}

Layout make_layout(uint8_t* aux, const Shape& s) {
  Layout L;
  L.ctrl = reinterpret_cast<Ctrl*>(aux + s.off_ctrl);
  L.arrays = reinterpret_cast<ArrayDesc*>(aux + s.off_arrays);
  for (int i = 0; i < 2; ++i) {
    L.large[i] = reinterpret_cast<Bin*>(aux + s.off_large[i]);
    L.hist[i] = reinterpret_cast<uint32_t*>(aux + s.off_hist[i]);
    L.diff[i] = reinterpret_cast<uint64_t*>(aux + s.off_diff[i]);
    L.eqkey[i] = reinterpret_cast<uint64_t*>(aux + s.off_eqkey[i]);
  }
  L.tile_prefix = reinterpret_cast<uint32_t*>(aux + s.off_tp);
  L.tile_bin = reinterpret_cast<uint32_t*>(aux + s.off_tb);
  L.status = reinterpret_cast<uint64_t*>(aux + s.off_status);
  L.wg_tail = reinterpret_cast<uint32_t*>(aux + s.off_tail);
  L.wg_carry = reinterpret_cast<uint32_t*>(aux + s.off_carry);
  L.wg_flag = reinterpret_cast<uint32_t*>(aux + s.off_flag);
  L.cap_ranges = s.cap_ranges;
  L.mid = reinterpret_cast<MidJob*>(aux + s.off_mid);
  L.tiny = reinterpret_cast<MidJob*>(aux + s.off_tiny);
  L.pair_part = reinterpret_cast<uint32_t*>(aux + s.off_pair_part);
  L.pair_hist = reinterpret_cast<uint32_t*>(aux + s.off_pair_hist);
  L.pair_d1 = reinterpret_cast<uint32_t*>(aux + s.off_pair_d1);
  L.cap_large = s.cap_large;
  L.cap_tiles = s.cap_tiles;
  L.cap_mid = s.cap_mid;
  return L;
}

int check_shape(uint32_t R, uint32_t K) {
  if (R < 8 || R > 64 || (R % 8) != 0) return RADULS_E_UNSUPPORTED;
  if (K == 0 || K > R) return RADULS_E_INVALID;
  return RADULS_OK;
}

bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) != 0; }

bool overlap(const void* a, uint64_t an, const void* b, uint64_t bn) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return an && bn && x < y + bn && y < x + an;
}

// Size check against the allocation that holds `p`, when HIP can tell.
int check_room(const void* p, uint64_t need) {
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
    (void)hipGetLastError();
    return RADULS_OK;
  }
  const uintptr_t end = reinterpret_cast<uintptr_t>(base) + size;
  if (reinterpret_cast<uintptr_t>(p) + need > end) return RADULS_E_TMP_SMALL;
  return RADULS_OK;
}

struct DevInfo {
  int cus = 0;
};

DevInfo device_info() {
  static std::mutex mu;
  static DevInfo cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  std::lock_guard<std::mutex> lk(mu);
  if (cache[dev].cus == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cache[dev].cus = cus;
  }
  return cache[dev];
}

void fill_params(Params& P, const Eff& e, const Shape& s, uint8_t* aux, uint32_t R, uint32_t K,
                 uint32_t mode, uint32_t count) {
  P = Params{};
  P.L = make_layout(aux, s);
  P.R = R;
  P.K = K;
  const uint32_t top = K - 8 * ((K - 1) / 8);  // key bytes in the top word, 1..8
  P.kmask = top == 8 ? ~0ull : ((1ull << (8 * top)) - 1);
  P.digit_bits = e.digit_bits;
  P.tiny_job = e.wave_job;
  P.es_job = e.es_job;
  P.tiny_max = e.tiny_max;
  P.mid_max = e.mid_max;
  P.tile = e.tile;
  P.nontemporal = e.nontemporal;
  P.lookback = e.lookback;
  P.rounds = s.rounds;
  P.round_budget = s.rounds;
  P.eq_split = s.eq_split;
  // a single array large enough to keep rounds for equality splits guesses
  // its root's top bit from a sample: a wrong guess costs one of those rounds
  P.spec = mode == kModeSort && s.eq_split ? 1u : 0u;
  P.mode = mode;
  P.count = count;
  const DevInfo d = device_info();
  const uint32_t cus = uint32_t(d.cus);
  P.grid_hist = std::max<uint32_t>(1, std::min<uint32_t>(s.cap_ranges, 4 * cus));
  if (s.pair) {
    P.pair = 1;
    P.grid_hist = std::min<uint32_t>(P.grid_hist, kPairRanges);
    P.pair_min_bins = std::max<uint32_t>(1, cus * 3 / 4);
  }
  P.grid_scatter = e.grid_blocks ? e.grid_blocks
                                 : std::max<uint32_t>(1, std::min<uint32_t>(s.cap_tiles, 2 * cus));
  P.grid_classify = std::max<uint32_t>(1, std::min<uint32_t>(s.cap_large, 4 * cus));
  P.scatter_lds_bytes = scatter_lds_bytes(int(R / 8));
  P.mid_lds_bytes = mid_dynamic_lds(mid_capacity(R / 8, (K + 7) / 8), int(R / 8));
  P.grid_mid = std::max<uint32_t>(1, std::min<uint32_t>(s.cap_mid, cus));
  P.grid_tiny = std::max<uint32_t>(1, std::min<uint32_t>(s.cap_mid / kMidWaves + 1, 4 * cus));
}

int launch(const Params& P, uint32_t R, uint32_t K, hipStream_t stream) {
  const uint32_t kw = (K + 7) / 8;
  hipError_t err;
  switch (R / 8) {
    case 1: err = run_rw1(P, kw, stream); break;
    case 2: err = run_rw2(P, kw, stream); break;
    case 3: err = run_rw3(P, kw, stream); break;
    case 4: err = run_rw4(P, kw, stream); break;
    case 5: err = run_rw5(P, kw, stream); break;
    case 6: err = run_rw6(P, kw, stream); break;
    case 7: err = run_rw7(P, kw, stream); break;
    case 8: err = run_rw8(P, kw, stream); break;
    default: return RADULS_E_UNSUPPORTED;
  }
  return err == hipSuccess ? RADULS_OK : RADULS_E_HIP;
}

uint64_t aux_offset(uint64_t n, uint32_t R) { return align_up(n * R, 256); }

// The auxiliary workspace of raduls_sort_static: a device array of fixed
// size that every GPU the library runs on holds until the process ends.  In
// host code its name stands for a host-side shadow, not a device address:
// kernels get the address hipGetSymbolAddress returns for the current
// device, taken once per device.
constexpr uint64_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

int static_scratch(void** out) {
  static std::mutex mu;
  static void* ptr[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return RADULS_E_HIP;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return RADULS_E_HIP;
    }
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return RADULS_OK;
}

hipError_t serve_launch_rw(const Params& P, uint32_t R, uint32_t K, uint32_t wgs, hipStream_t s) {
  const uint32_t kw = (K + 7) / 8;
  switch (R / 8) {
    case 1: return serve_rw1(P, kw, wgs, s);
    case 2: return serve_rw2(P, kw, wgs, s);
    case 3: return serve_rw3(P, kw, wgs, s);
    case 4: return serve_rw4(P, kw, wgs, s);
    case 5: return serve_rw5(P, kw, wgs, s);
    case 6: return serve_rw6(P, kw, wgs, s);
    case 7: return serve_rw7(P, kw, wgs, s);
    case 8: return serve_rw8(P, kw, wgs, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace raduls

// A resident server: its ring (host-pinned), device state, own stream and
// the kernel running there.
struct raduls_server {
  uint32_t R = 0, K = 0, slots = 0, wgs = 0;
  uint64_t cap = 0;                          // records per request
  raduls::ServeRing* ring = nullptr;         // host address
  void* dmem = nullptr;                      // ServeState + Ctrl[wgs]
  hipStream_t stream = nullptr;
  std::atomic<uint64_t> next{0};             // next ticket
  uint64_t through = 0;                      // tickets below it have all completed (under mu_done)
  std::mutex mu_done;
  // launches of the kernel so far, and the last launch seen to have left
  // (a stale observation never hides a later launch)
  std::atomic<uint64_t> launched{0}, exited{0};
  std::mutex mu;                             // submitters, relaunches
  raduls::Params P{};                        // the kernel's launch parameters
};

namespace raduls {
namespace {

bool server_running(raduls_server* s) {
  const uint64_t g = s->launched.load(std::memory_order_acquire);
  if (s->exited.load(std::memory_order_acquire) >= g) return false;
  const hipError_t q = hipStreamQuery(s->stream);
  if (q == hipErrorNotReady) return true;
  if (q != hipSuccess) (void)hipGetLastError();
  // launch g (and every one before it) has left; a relaunch since the
  // query has a larger number and is not covered
  uint64_t e = s->exited.load(std::memory_order_relaxed);
  while (e < g && !s->exited.compare_exchange_weak(e, g, std::memory_order_acq_rel)) {
  }
  return false;
}

// The server's kernel, relaunched (same stream, same ring and device state)
// if it left idle or at the end of its lease: requests still in the device
// queue, or published after its last look at the ring, are then picked up.  False if the host stopped it or the launch
// failed.  The caller holds s->mu.
bool server_ensure(raduls_server* s) {
  if (server_running(s)) return true;
  if (__atomic_load_n(&s->ring->stop, __ATOMIC_ACQUIRE)) return false;
  __atomic_store_n(&s->ring->reason, 0u, __ATOMIC_RELEASE);
  if (serve_launch_rw(s->P, s->R, s->K, s->wgs, s->stream) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  s->launched.fetch_add(1, std::memory_order_acq_rel);
  return true;
}

void server_free(raduls_server* s) {
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->dmem) (void)hipFree(s->dmem);
  if (s->ring) (void)hipHostFree(s->ring);
  delete s;
}

}  // namespace
}  // namespace raduls

using namespace raduls;

extern "C" {

int raduls_tmp_bytes(uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, uint64_t* out_bytes) {
  int st = check_shape(rec_bytes, key_bytes);
  if (st) return st;
  if (!out_bytes) return RADULS_E_INVALID;
  if (n >= (1ull << 32)) return RADULS_E_UNSUPPORTED;
  const Eff e = effective(current_tuning(), rec_bytes, key_bytes);
  const Shape s = plan_shape(n, 1, rec_bytes, key_bytes, e, false, use_pair(e, n, key_bytes));
  *out_bytes = aux_offset(n, rec_bytes) + s.bytes;
  return RADULS_OK;
}

int raduls_sort(void* recs, void* tmp, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                hipStream_t stream) {
  int st = check_shape(rec_bytes, key_bytes);
  if (st) return st;
  if (n >= (1ull << 32)) return RADULS_E_UNSUPPORTED;
  if (n <= 1) return RADULS_OK;
  if (!recs || !tmp) return RADULS_E_INVALID;
  if (misaligned(recs) || misaligned(tmp)) return RADULS_E_ALIGN;
  const Eff e = effective(current_tuning(), rec_bytes, key_bytes);
  const Shape s = plan_shape(n, 1, rec_bytes, key_bytes, e, false, use_pair(e, n, key_bytes));
  const uint64_t need = aux_offset(n, rec_bytes) + s.bytes;
  if (overlap(recs, n * rec_bytes, tmp, need)) return RADULS_E_INVALID;
  st = check_room(tmp, need);
  if (st) return st;
  Params P;
  fill_params(P, e, s, static_cast<uint8_t*>(tmp) + aux_offset(n, rec_bytes), rec_bytes,
              key_bytes, kModeSort, 1);
  P.recs = static_cast<uint8_t*>(recs);
  P.tmp = static_cast<uint8_t*>(tmp);
  P.n = n;
  if (n <= e.mid_max) P.rounds = 0;
  return launch(P, rec_bytes, key_bytes, stream);
}

int raduls_sort_static(void* recs, void* tmp, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                       hipStream_t stream) {
  int st = check_shape(rec_bytes, key_bytes);
  if (st) return st;
  if (n >= (1ull << 32)) return RADULS_E_UNSUPPORTED;
  if (n <= 1) return RADULS_OK;
  if (!recs || !tmp) return RADULS_E_INVALID;
  if (misaligned(recs) || misaligned(tmp)) return RADULS_E_ALIGN;
  const Eff e = effective(current_tuning(), rec_bytes, key_bytes);
  // (the top-level digit-pair counts, a speed option, are not used: their
  // rows alone would take as much room as the rest of the workspace)
  const Shape s = plan_shape(n, 1, rec_bytes, key_bytes, e, false, false);
  if (s.bytes > kStaticScratchBytes) return RADULS_E_SCRATCH;
  if (overlap(recs, n * rec_bytes, tmp, n * rec_bytes)) return RADULS_E_INVALID;
  st = check_room(tmp, n * rec_bytes);
  if (st) return st;
  void* aux = nullptr;
  st = static_scratch(&aux);
  if (st) return st;
  Params P;
  fill_params(P, e, s, static_cast<uint8_t*>(aux), rec_bytes, key_bytes, kModeSort, 1);
  P.recs = static_cast<uint8_t*>(recs);
  P.tmp = static_cast<uint8_t*>(tmp);
  P.n = n;
  if (n <= e.mid_max) P.rounds = 0;
  return launch(P, rec_bytes, key_bytes, stream);
}

int raduls_inspect_rounds(void* recs, void* tmp, uint64_t n, uint32_t rec_bytes,
                          uint32_t key_bytes, uint32_t rounds, raduls_bin* bins, uint32_t cap,
                          uint32_t* count, hipStream_t stream) {
  int st = check_shape(rec_bytes, key_bytes);
  if (st) return st;
  if (!count || (cap && !bins)) return RADULS_E_INVALID;
  *count = 0;
  if (n >= (1ull << 32)) return RADULS_E_UNSUPPORTED;
  if (rounds == 0) return RADULS_E_INVALID;
  if (!recs || !tmp) return RADULS_E_INVALID;
  if (misaligned(recs) || misaligned(tmp)) return RADULS_E_ALIGN;
  const Eff e = effective(current_tuning(), rec_bytes, key_bytes);
  const Shape s = plan_shape(n, 1, rec_bytes, key_bytes, e, false, use_pair(e, n, key_bytes));
  const uint64_t need = aux_offset(n, rec_bytes) + s.bytes;
  if (overlap(recs, n * rec_bytes, tmp, need)) return RADULS_E_INVALID;
  st = check_room(tmp, need);
  if (st) return st;
  if (n <= e.mid_max) return RADULS_OK;  // no round: the whole array is one LDS job
  Params P;
  uint8_t* aux = static_cast<uint8_t*>(tmp) + aux_offset(n, rec_bytes);
  fill_params(P, e, s, aux, rec_bytes, key_bytes, kModeSort, 1);
  P.recs = static_cast<uint8_t*>(recs);
  P.tmp = static_cast<uint8_t*>(tmp);
  P.n = n;
  P.rounds = std::min(rounds, s.rounds);
  P.inspect = 1;
  st = launch(P, rec_bytes, key_bytes, stream);
  if (st) return st;
  if (hipStreamSynchronize(stream) != hipSuccess) return RADULS_E_HIP;
  Ctrl c;
  if (hipMemcpy(&c, P.L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost) != hipSuccess) return RADULS_E_HIP;
  const uint32_t side = P.rounds & 1;
  const uint32_t nb = std::min(c.large_count[side], P.L.cap_large);
  *count = nb;
  const uint32_t take = std::min(nb, cap);
  if (take) {
    std::vector<Bin> host(take);
    if (hipMemcpy(host.data(), P.L.large[side], take * sizeof(Bin), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return RADULS_E_HIP;
    for (uint32_t i = 0; i < take; ++i) {
      bins[i].start = host[i].start;
      bins[i].size = host[i].size;
      bins[i].bits = host[i].bits;
      bins[i].side = host[i].side;
      bins[i].flags = host[i].flags;
    }
  }
  return c.error ? RADULS_E_DEVICE : RADULS_OK;
}

int raduls_batch_ws_bytes(uint32_t count, uint64_t total_n, uint32_t rec_bytes,
                          uint32_t key_bytes, uint64_t* out_bytes) {
  int st = check_shape(rec_bytes, key_bytes);
  if (st) return st;
  if (!out_bytes) return RADULS_E_INVALID;
  const Eff e = effective(current_tuning(), rec_bytes, key_bytes);
  *out_bytes = plan_shape(total_n, count, rec_bytes, key_bytes, e, false).bytes;
  return RADULS_OK;
}

int raduls_sort_batch(const raduls_array* d_arrays, uint32_t count, uint64_t total_n,
                      uint32_t rec_bytes, uint32_t key_bytes, void* ws, uint64_t ws_bytes,
                      hipStream_t stream) {
  int st = check_shape(rec_bytes, key_bytes);
  if (st) return st;
  if (count == 0) return RADULS_OK;
  if (!d_arrays || !ws) return RADULS_E_INVALID;
  if (misaligned(d_arrays) || misaligned(ws)) return RADULS_E_ALIGN;
  const Eff e = effective(current_tuning(), rec_bytes, key_bytes);
  const Shape s = plan_shape(total_n, count, rec_bytes, key_bytes, e, false);
  if (ws_bytes < s.bytes) return RADULS_E_TMP_SMALL;
  if (overlap(d_arrays, uint64_t(count) * sizeof(raduls_array), ws, s.bytes))
    return RADULS_E_INVALID;
  Params P;
  fill_params(P, e, s, static_cast<uint8_t*>(ws), rec_bytes, key_bytes, kModeBatch, count);
  P.d_arrays_in = reinterpret_cast<const ArrayDesc*>(d_arrays);
  P.total_cap = total_n;
  return launch(P, rec_bytes, key_bytes, stream);
}

int raduls_step_ws_bytes(uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, uint64_t* out_bytes) {
  int st = check_shape(rec_bytes, key_bytes);
  if (st) return st;
  if (!out_bytes) return RADULS_E_INVALID;
  if (n >= (1ull << 32)) return RADULS_E_UNSUPPORTED;
  const Eff e = effective(current_tuning(), rec_bytes, key_bytes);
  *out_bytes = plan_shape(n, 1, rec_bytes, key_bytes, e, true).bytes;
  return RADULS_OK;
}

static int step_common(const void* src, void* dst, uint64_t n, uint32_t R, uint32_t K,
                       uint32_t bits, uint32_t width, uint32_t* d_counts, uint32_t* d_offsets,
                       void* ws, uint64_t ws_bytes, uint32_t mode, hipStream_t stream) {
  int st = check_shape(R, K);
  if (st) return st;
  if (n >= (1ull << 32)) return RADULS_E_UNSUPPORTED;
  if (width < 1 || width > 8 || bits < 1 || bits > 8 * K) return RADULS_E_INVALID;
  if (!src || !ws || (mode == kModePartition && !dst) || (mode == kModeHist && !d_counts))
    return RADULS_E_INVALID;
  if (misaligned(src) || misaligned(ws) || (dst && misaligned(dst))) return RADULS_E_ALIGN;
  const Eff e = effective(current_tuning(), R, K);
  const Shape s = plan_shape(n, 1, R, K, e, true);
  if (ws_bytes < s.bytes) return RADULS_E_TMP_SMALL;
  if (mode == kModePartition && overlap(src, n * R, dst, n * R)) return RADULS_E_INVALID;
  if (overlap(src, n * R, ws, s.bytes) || (dst && overlap(dst, n * R, ws, s.bytes)))
    return RADULS_E_INVALID;
  Params P;
  fill_params(P, e, s, static_cast<uint8_t*>(ws), R, K, mode, 1);
  P.recs = static_cast<uint8_t*>(const_cast<void*>(src));
  P.tmp = static_cast<uint8_t*>(dst);
  P.n = n;
  P.step_bits = bits;
  P.step_width = width;
  P.digit_bits = width;
  P.d_counts_out = d_counts;
  P.d_offsets_out = d_offsets;
  return launch(P, R, K, stream);
}

int raduls_histogram(const void* recs, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                     uint32_t bits, uint32_t width, uint32_t* d_counts, void* ws,
                     uint64_t ws_bytes, hipStream_t stream) {
  return step_common(recs, nullptr, n, rec_bytes, key_bytes, bits, width, d_counts, nullptr, ws,
                     ws_bytes, kModeHist, stream);
}

int raduls_partition(const void* src, void* dst, uint64_t n, uint32_t rec_bytes,
                     uint32_t key_bytes, uint32_t bits, uint32_t width, uint32_t* d_offsets,
                     void* ws, uint64_t ws_bytes, hipStream_t stream) {
  return step_common(src, dst, n, rec_bytes, key_bytes, bits, width, nullptr, d_offsets, ws,
                     ws_bytes, kModePartition, stream);
}

int raduls_check(const void* tmp_or_ws, uint64_t n, uint32_t rec_bytes, int ws_only,
                 raduls_stats* stats, hipStream_t stream) {
  if (!tmp_or_ws || !stats) return RADULS_E_INVALID;
  if (!ws_only && (rec_bytes < 8 || rec_bytes > 64 || rec_bytes % 8)) return RADULS_E_UNSUPPORTED;
  const uint8_t* base = static_cast<const uint8_t*>(tmp_or_ws) + (ws_only ? 0 : aux_offset(n, rec_bytes));
  if (hipStreamSynchronize(stream) != hipSuccess) return RADULS_E_HIP;
  Ctrl c;
  if (hipMemcpy(&c, base, sizeof(Ctrl), hipMemcpyDeviceToHost) != hipSuccess) return RADULS_E_HIP;
  std::memset(stats, 0, sizeof(*stats));
  stats->error = c.error;
  stats->rounds = c.rounds;
  stats->large_bins = c.large_bins;
  stats->scattered_bins = c.scattered_bins;
  stats->mid_jobs = c.mid_count + c.tiny_count - c.copy_count;
  stats->copy_jobs = c.copy_count;
  stats->moved_records = c.moved_records;
  stats->large_records = c.large_records;
  stats->pair_rounds = c.pair_rounds;
  stats->eq_bins = c.eq_bins;
  return c.error ? RADULS_E_DEVICE : RADULS_OK;
}

int raduls_set_tuning(const raduls_tuning* tuning) {
  if (!tuning) return RADULS_E_INVALID;
  if (tuning->digit_bits > 8 || tuning->tiny_max > 256 || tuning->nontemporal > 2 ||
      tuning->wave_job_max > kTinyJob || tuning->es_job_max > 256 || tuning->tile_items > 8)
    return RADULS_E_INVALID;
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  g_tuning = *tuning;
  return RADULS_OK;
}

int raduls_get_tuning(raduls_tuning* tuning) {
  if (!tuning) return RADULS_E_INVALID;
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  *tuning = g_tuning;
  return RADULS_OK;
}

int raduls_set_profile_events(hipEvent_t* events, uint32_t count) {
  if (count > 2 * kProfileSlots || (count && !events)) return RADULS_E_INVALID;
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  for (uint32_t i = 0; i < 2 * kProfileSlots; ++i) g_profile.ev[i] = i < count ? events[i] : nullptr;
  g_profile.count = count;
  return RADULS_OK;
}

uint32_t raduls_mid_capacity(uint32_t rec_bytes, uint32_t key_bytes) {
  if (check_shape(rec_bytes, key_bytes) != RADULS_OK) return 0;
  return mid_capacity(rec_bytes / 8, (key_bytes + 7) / 8);
}

int raduls_server_max_records(uint32_t rec_bytes, uint32_t key_bytes, uint64_t* out_records) {
  int st = check_shape(rec_bytes, key_bytes);
  if (st) return st;
  if (!out_records) return RADULS_E_INVALID;
  *out_records = effective(current_tuning(), rec_bytes, key_bytes).mid_max;
  return RADULS_OK;
}

int raduls_server_create(uint32_t rec_bytes, uint32_t key_bytes, uint32_t slots,
                         uint32_t workgroups, uint32_t idle_ms, uint32_t lease_ms,
                         raduls_server** out) {
  int st = check_shape(rec_bytes, key_bytes);
  if (st) return st;
  if (!out || slots == 0 || slots > kServeMaxSlots || idle_ms > kServeMaxIdleMs ||
      lease_ms > kServeMaxLeaseMs)
    return RADULS_E_INVALID;
  *out = nullptr;
  const uint32_t cus = uint32_t(device_info().cus);
  const uint32_t wgs = std::min(workgroups ? workgroups : std::max(1u, cus / 8), cus);
  const Eff e = effective(current_tuning(), rec_bytes, key_bytes);
  raduls_server* s = new raduls_server;
  s->R = rec_bytes;
  s->K = key_bytes;
  s->slots = slots;
  s->wgs = wgs;
  s->cap = e.mid_max;
  const size_t ring_bytes = sizeof(ServeRing) + size_t(slots - 1) * sizeof(ServeSlot);
  const size_t dev_bytes =
      sizeof(ServeState) + size_t(wgs) * sizeof(Ctrl) + size_t(slots) * sizeof(ServeJob);
  void* dring = nullptr;
  if (hipHostMalloc(reinterpret_cast<void**>(&s->ring), ring_bytes,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer(&dring, s->ring, 0) != hipSuccess ||
      hipMalloc(&s->dmem, dev_bytes) != hipSuccess ||
      hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    server_free(s);
    return RADULS_E_HIP;
  }
  std::memset(s->ring, 0, ring_bytes);
  if (hipMemsetAsync(s->dmem, 0, dev_bytes, s->stream) != hipSuccess) {
    (void)hipGetLastError();
    server_free(s);
    return RADULS_E_HIP;
  }
  Params P{};
  P.R = rec_bytes;
  P.K = key_bytes;
  const uint32_t top = key_bytes - 8 * ((key_bytes - 1) / 8);
  P.kmask = top == 8 ? ~0ull : ((1ull << (8 * top)) - 1);
  P.tiny_job = e.wave_job;
  P.es_job = e.es_job;
  P.tiny_max = e.tiny_max;
  P.mid_max = e.mid_max;
  P.mid_lds_bytes = mid_dynamic_lds(mid_capacity(rec_bytes / 8, (key_bytes + 7) / 8),
                                    int(rec_bytes / 8));
  P.ring = static_cast<ServeRing*>(dring);
  P.serve = static_cast<ServeState*>(s->dmem);
  P.serve_ctrl = reinterpret_cast<Ctrl*>(static_cast<uint8_t*>(s->dmem) + sizeof(ServeState));
  P.serve_queue = reinterpret_cast<ServeJob*>(P.serve_ctrl + wgs);
  P.serve_slots = slots;
  P.serve_idle = uint64_t(idle_ms ? idle_ms : kServeDefaultIdleMs) * 100000ull;  // 100 MHz ticks
  P.serve_lease = uint64_t(lease_ms) * 100000ull;
  s->P = P;
  if (serve_launch_rw(P, rec_bytes, key_bytes, wgs, s->stream) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s->stream);
    server_free(s);
    return RADULS_E_HIP;
  }
  s->launched.store(1, std::memory_order_release);
  *out = s;
  return RADULS_OK;
}

int raduls_server_submit(raduls_server* s, void* recs, uint64_t n, uint64_t* ticket) {
  if (!s || !ticket || (n && !recs)) return RADULS_E_INVALID;
  if (n > s->cap) return RADULS_E_UNSUPPORTED;
  if (recs && misaligned(recs)) return RADULS_E_ALIGN;
  std::lock_guard<std::mutex> lk(s->mu);
  if (!server_ensure(s)) return RADULS_E_STOPPED;
  const uint64_t t = s->next.load(std::memory_order_relaxed);
  ServeSlot& sl = s->ring->slot[t % s->slots];
  // the slot's previous request must have completed
  if (t >= s->slots && __atomic_load_n(&sl.done, __ATOMIC_ACQUIRE) != t - s->slots + 1)
    return RADULS_E_BUSY;
  sl.recs = reinterpret_cast<uint64_t>(recs);
  sl.n = n;
  sl.status = 0;
  __atomic_store_n(&sl.seq, t + 1, __ATOMIC_RELEASE);  // publish
  s->next.store(t + 1, std::memory_order_release);
  *ticket = t;
  (void)server_ensure(s);  // (it may have left since the check above)
  return RADULS_OK;
}

int raduls_server_submit_many(raduls_server* s, void* const* recs, const uint64_t* n,
                              uint32_t count, uint64_t* first_ticket, uint32_t* accepted) {
  if (!s || !first_ticket || !accepted || (count && (!recs || !n))) return RADULS_E_INVALID;
  *accepted = 0;
  for (uint32_t i = 0; i < count; ++i) {
    if (n[i] > s->cap) return RADULS_E_UNSUPPORTED;
    if ((n[i] && !recs[i])) return RADULS_E_INVALID;
    if (recs[i] && misaligned(recs[i])) return RADULS_E_ALIGN;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (!server_ensure(s)) return RADULS_E_STOPPED;
  const uint64_t t0 = s->next.load(std::memory_order_relaxed);
  *first_ticket = t0;
  uint32_t i = 0;
  for (; i < count; ++i) {
    const uint64_t t = t0 + i;
    ServeSlot& sl = s->ring->slot[t % s->slots];
    if (t >= s->slots && __atomic_load_n(&sl.done, __ATOMIC_ACQUIRE) != t - s->slots + 1) break;
    sl.recs = reinterpret_cast<uint64_t>(recs[i]);
    sl.n = n[i];
    sl.status = 0;
    __atomic_store_n(&sl.seq, t + 1, __ATOMIC_RELEASE);
  }
  s->next.store(t0 + i, std::memory_order_release);
  *accepted = i;
  if (i) (void)server_ensure(s);
  return RADULS_OK;
}

int raduls_server_poll(raduls_server* s, uint64_t ticket, uint32_t* status) {
  if (!s || ticket >= s->next.load(std::memory_order_acquire)) return RADULS_E_INVALID;
  const ServeSlot& sl = s->ring->slot[ticket % s->slots];
  const uint64_t d = __atomic_load_n(&sl.done, __ATOMIC_ACQUIRE);
  if (d >= ticket + 1) {  // (larger: the slot has served a later request since)
    if (status) *status = d == ticket + 1 ? __atomic_load_n(&sl.status, __ATOMIC_RELAXED) : 0u;
    return 1;
  }
  if (!server_running(s)) {
    // the kernel may have completed the request just before leaving;
    // otherwise it left idle before seeing it and is relaunched
    if (__atomic_load_n(&sl.done, __ATOMIC_ACQUIRE) >= ticket + 1) return raduls_server_poll(s, ticket, status);
    std::lock_guard<std::mutex> lk(s->mu);
    if (!server_ensure(s)) return RADULS_E_STOPPED;
  }
  return 0;
}

int raduls_server_wait(raduls_server* s, uint64_t ticket, uint32_t timeout_ms, uint32_t* status) {
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t k = 0;; ++k) {
    const int r = raduls_server_poll(s, ticket, status);
    if (r != 0) return r;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms))
      return RADULS_E_TIMEOUT;
    if (k > 64) std::this_thread::yield();
  }
}

int raduls_server_wait_range(raduls_server* s, uint64_t first, uint64_t count,
                             uint32_t timeout_ms, uint32_t* status_or) {
  if (!s) return RADULS_E_INVALID;
  if (count && first + count > s->next.load(std::memory_order_acquire)) return RADULS_E_INVALID;
  const auto t0 = std::chrono::steady_clock::now();
  uint32_t acc = 0;
  for (uint64_t t = first; t < first + count; ++t) {
    for (uint32_t k = 0;; ++k) {
      uint32_t st = 0;
      const int r = raduls_server_poll(s, t, &st);
      if (r < 0) return r;
      if (r == 1) {
        acc |= st;
        break;
      }
      if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms))
        return RADULS_E_TIMEOUT;
      if (k > 64) std::this_thread::yield();
    }
  }
  if (status_or) *status_or = acc;
  return RADULS_OK;
}

int raduls_server_completed(raduls_server* s, uint64_t* through, uint32_t* status_or) {
  if (!s || !through) return RADULS_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu_done);
  const uint64_t next = s->next.load(std::memory_order_acquire);
  uint64_t t = s->through;
  uint32_t acc = 0;
  while (t < next) {
    const ServeSlot& sl = s->ring->slot[t % s->slots];
    if (__atomic_load_n(&sl.done, __ATOMIC_ACQUIRE) != t + 1) break;
    acc |= __atomic_load_n(&sl.status, __ATOMIC_RELAXED);
    ++t;
  }
  s->through = t;
  *through = t;
  if (status_or) *status_or = acc;
  if (t < next && !server_running(s)) {
    std::lock_guard<std::mutex> lk2(s->mu);
    if (!server_ensure(s)) return RADULS_E_STOPPED;
  }
  return RADULS_OK;
}

int raduls_server_info(raduls_server* s, uint64_t* max_records, uint32_t* workgroups,
                       uint32_t* running, uint32_t* reason) {
  if (!s) return RADULS_E_INVALID;
  if (max_records) *max_records = s->cap;
  if (workgroups) *workgroups = s->wgs;
  if (running) *running = server_running(s) ? 1u : 0u;
  if (reason) *reason = __atomic_load_n(&s->ring->reason, __ATOMIC_ACQUIRE);
  return RADULS_OK;
}

int raduls_server_destroy(raduls_server* s) {
  if (!s) return RADULS_E_INVALID;
  __atomic_store_n(&s->ring->stop, 1ull, __ATOMIC_RELEASE);
  // every wait of the kernel checks the stop word, so it leaves after the
  // requests it is sorting
  const hipError_t e = hipStreamSynchronize(s->stream);
  server_free(s);
  return e == hipSuccess ? RADULS_OK : RADULS_E_HIP;
}

const char* raduls_strerror(int status) {
  switch (status) {
    case RADULS_OK: return "ok";
    case RADULS_E_INVALID: return "invalid argument";
    case RADULS_E_ALIGN: return "device pointer not 16-byte aligned";
    case RADULS_E_TMP_SMALL: return "scratch buffer or workspace too small";
    case RADULS_E_UNSUPPORTED: return "unsupported record size or record count";
    case RADULS_E_HIP: return "HIP runtime error";
    case RADULS_E_DEVICE: return "device reported an error";
    case RADULS_E_SCRATCH: return "the static workspace is too small for this many records";
    case RADULS_E_BUSY: return "the server's ring slot for the next request is still in use";
    case RADULS_E_STOPPED: return "the resident server has stopped";
    case RADULS_E_TIMEOUT: return "the request did not complete in time";
    default: return "unknown status";
  }
}

}  // extern "C"
