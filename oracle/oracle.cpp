// CPU oracle for the RADULS2 record sort (Kokot, Deorowicz, Dlugosz,
// "Even faster sorting of (not only) integers", arXiv 1703.00687).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the sorting library links, loads or
// calls this file; only the tests, the package smoke check and the CPU
// baseline leg of the benchmark do.  It shares no code with the HIP path.
//
// Everything here is plain and slow on purpose: byte-by-byte key arithmetic,
// a library stable sort for the definition of the result, and the textbook
// form of each step of an MSD radix sort.
//
// Record model (paper: abstract; Sec. 4.2 "16 B records (8 B key and 8 B
// data)"; Sec. 4.2 record-size experiment).  A record is R contiguous bytes;
// its key is the first K bytes read as an unsigned little-endian integer
// (byte K-1 is the most significant).  The paper does not fix the byte order;
// this reading makes a uint64 key at offset 0 sort numerically.
//
// Digits (Sec. 1 radix-sort description; Sec. 3.1 "MSD radix sort with 1 B
// digits").  Key bits are numbered 0 .. 8K-1 from the least significant bit
// of byte 0.  A digit is named by (bits, width): it is the bit field
// [bits - w, bits) of the key with w = min(width, bits).  MSD processing
// starts at bits = 8K and moves towards 0.  With width 8 and bits a multiple
// of 8 the digit is one key byte, as in the paper.

#include <omp.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <parallel/algorithm>
#include <vector>

namespace {

// Status codes mirror the ones the sorting library documents so the error
// paths can be compared; the values are restated here, not shared.
constexpr int ST_OK = 0;
constexpr int ST_INVALID = -1;
constexpr int ST_UNSUPPORTED = -4;

int validate(uint64_t n, uint32_t R, uint32_t K) {
  if (R < 8 || R > 64 || (R % 8) != 0) return ST_UNSUPPORTED;
  if (K == 0 || K > R) return ST_INVALID;
  if (n >= (uint64_t(1) << 32)) return ST_UNSUPPORTED;
  return ST_OK;
}

// key(a) < key(b): compare key bytes from the most significant (K-1) down to
// byte 0; the first differing byte decides.
bool key_less(const uint8_t* a, const uint8_t* b, uint32_t K) {
  for (uint32_t i = K; i-- > 0;) {
    if (a[i] != b[i]) return a[i] < b[i];
  }
  return false;
}

bool key_equal(const uint8_t* a, const uint8_t* b, uint32_t K) {
  return std::memcmp(a, b, K) == 0;
}

// Bit p of the key (bit 0 = least significant bit of byte 0).
unsigned key_bit(const uint8_t* rec, uint32_t p) { return (rec[p / 8] >> (p % 8)) & 1u; }

// The digit (bits, width) of one record, assembled one bit at a time.
uint32_t digit_of(const uint8_t* rec, uint32_t bits, uint32_t width) {
  uint32_t w = std::min(width, bits);
  uint32_t lo = bits - w;
  uint32_t d = 0;
  for (uint32_t j = 0; j < w; ++j) d |= key_bit(rec, lo + j) << j;
  return d;
}

void gather(const uint8_t* in, uint8_t* out, const std::vector<uint64_t>& order, uint32_t R) {
  for (uint64_t i = 0; i < order.size(); ++i) std::memcpy(out + i * R, in + order[i] * R, R);
}

// Counting-sort partition of records [0, n) of `in` on one digit, written to
// `out` (Sec. 1: one radix phase is a counting sort on the current digit).
// Steps in textbook order: histogram, exclusive prefix sum, stable placement.
void counting_partition(const uint8_t* in, uint8_t* out, uint64_t n, uint32_t R, uint32_t bits,
                        uint32_t width, std::vector<uint64_t>* counts_out) {
  uint32_t w = std::min(width, bits);
  uint64_t buckets = uint64_t(1) << w;
  std::vector<uint64_t> count(buckets, 0);
  for (uint64_t i = 0; i < n; ++i) count[digit_of(in + i * R, bits, width)]++;
  std::vector<uint64_t> next(buckets, 0);
  uint64_t run = 0;
  for (uint64_t b = 0; b < buckets; ++b) {
    next[b] = run;
    run += count[b];
  }
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t d = digit_of(in + i * R, bits, width);
    std::memcpy(out + next[d] * R, in + i * R, R);
    next[d]++;
  }
  if (counts_out) *counts_out = count;
}

// Enumeration sort (Sec. 2.2): the final position of each record is found by
// comparing it with every other record.  Equal keys are ranked by their input
// index so the ranks form a permutation (the paper does not say how ties are
// broken; without a tie rule equal keys would collide).
void enum_sort(const uint8_t* in, uint8_t* out, uint64_t n, uint32_t R, uint32_t K) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t rank = 0;
    for (uint64_t j = 0; j < n; ++j) {
      if (key_less(in + j * R, in + i * R, K)) ++rank;
      else if (j < i && key_equal(in + j * R, in + i * R, K)) ++rank;
    }
    std::memcpy(out + rank * R, in + i * R, R);
  }
}

// Plain MSD radix sort (Sec. 1 and Sec. 3.1): partition the bin on the current
// digit, then recurse into every resulting bin on the next digit; a bin is
// finished when it holds at most one record or no key bits remain; bins of at
// most `tiny_max` records go to the tiny-bin sorter (Sec. 3.3; enumeration
// sort here).  `buf` is scratch of the same size as the bin.
void msd_rec(uint8_t* a, uint8_t* buf, uint64_t n, uint32_t R, uint32_t K, uint32_t bits,
             uint32_t width, uint64_t tiny_max) {
  if (n <= 1 || bits == 0) return;
  if (n <= tiny_max) {
    enum_sort(a, buf, n, R, K);
    std::memcpy(a, buf, n * R);
    return;
  }
  std::vector<uint64_t> count;
  counting_partition(a, buf, n, R, bits, width, &count);
  std::memcpy(a, buf, n * R);
  uint32_t w = std::min(width, bits);
  uint64_t start = 0;
  for (uint64_t b = 0; b < count.size(); ++b) {
    msd_rec(a + start * R, buf + start * R, count[b], R, K, bits - w, width, tiny_max);
    start += count[b];
  }
}

}  // namespace

extern "C" {

int oracle_validate(uint64_t n, uint32_t R, uint32_t K) { return validate(n, R, K); }

// The sorted result by definition: a stable permutation of the records with
// non-decreasing keys.  Radix MSD reaches exactly this key sequence (Sec. 1,
// Sec. 3.1); stability fixes the order of equal keys so the output is unique.
int oracle_sort(const uint8_t* in, uint8_t* out, uint64_t n, uint32_t R, uint32_t K) {
  int st = validate(n, R, K);
  if (st != ST_OK) return st;
  std::vector<uint64_t> order(n);
  std::iota(order.begin(), order.end(), uint64_t(0));
  std::stable_sort(order.begin(), order.end(), [&](uint64_t x, uint64_t y) {
    return key_less(in + x * R, in + y * R, K);
  });
  gather(in, out, order, R);
  return ST_OK;
}

// The same definition computed on several cores, used only as the CPU
// baseline of the benchmark (the paper's comparison includes a parallel
// library sort, Sec. 4.2): the same stable sort by the same comparator, run
// as libstdc++'s parallel-mode stable sort (a multiway mergesort) over
// `threads` OpenMP threads (0: all available), and a parallel gather.  Both
// sorts are stable, so the output is identical to oracle_sort's.  `used`
// receives the number of threads.
int oracle_sort_parallel(const uint8_t* in, uint8_t* out, uint64_t n, uint32_t R, uint32_t K,
                         int threads, int* used) {
  int st = validate(n, R, K);
  if (st != ST_OK) return st;
  const int nt = threads > 0 ? threads : omp_get_max_threads();
  if (used) *used = nt;
  std::vector<uint64_t> order(n);
  std::iota(order.begin(), order.end(), uint64_t(0));
  __gnu_parallel::stable_sort(
      order.begin(), order.end(),
      [&](uint64_t x, uint64_t y) { return key_less(in + x * R, in + y * R, K); },
      __gnu_parallel::multiway_mergesort_tag(nt));
#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t i = 0; i < int64_t(n); ++i) std::memcpy(out + i * R, in + order[i] * R, R);
  return ST_OK;
}

// Digit histogram (step one of a counting sort, Sec. 1; per-bin counters of
// Sec. 3.2/3.3).  `counts` receives 2^min(width,bits) entries.
int oracle_histogram(const uint8_t* in, uint64_t n, uint32_t R, uint32_t K, uint32_t bits,
                     uint32_t width, uint64_t* counts) {
  int st = validate(n, R, K);
  if (st != ST_OK) return st;
  if (bits == 0 || bits > 8 * K || width == 0 || width > 16) return ST_INVALID;
  uint32_t w = std::min(width, bits);
  for (uint64_t b = 0; b < (uint64_t(1) << w); ++b) counts[b] = 0;
  for (uint64_t i = 0; i < n; ++i) counts[digit_of(in + i * R, bits, width)]++;
  return ST_OK;
}

// Exclusive prefix sum: offsets[b] = base + sum of counts[c] for c < b.
void oracle_exclusive_scan(const uint64_t* counts, uint64_t m, uint64_t base, uint64_t* offsets) {
  uint64_t run = base;
  for (uint64_t b = 0; b < m; ++b) {
    offsets[b] = run;
    run += counts[b];
  }
}

// One stable counting-sort pass on digit (bits, width) from `in` to `out`.
int oracle_partition(const uint8_t* in, uint8_t* out, uint64_t n, uint32_t R, uint32_t K,
                     uint32_t bits, uint32_t width) {
  int st = validate(n, R, K);
  if (st != ST_OK) return st;
  if (bits == 0 || bits > 8 * K || width == 0 || width > 16) return ST_INVALID;
  counting_partition(in, out, n, R, bits, width, nullptr);
  return ST_OK;
}

// Enumeration sort of the whole input (the tiny-bin sorter's rule, Sec. 2.2,
// Sec. 3.3).  O(n^2): small inputs only.
int oracle_enum_sort(const uint8_t* in, uint8_t* out, uint64_t n, uint32_t R, uint32_t K) {
  int st = validate(n, R, K);
  if (st != ST_OK) return st;
  enum_sort(in, out, n, R, K);
  return ST_OK;
}

// The MSD radix sort itself, in the paper's order of steps.
int oracle_msd_sort(const uint8_t* in, uint8_t* out, uint64_t n, uint32_t R, uint32_t K,
                    uint32_t width, uint64_t tiny_max) {
  int st = validate(n, R, K);
  if (st != ST_OK) return st;
  if (width == 0 || width > 16) return ST_INVALID;
  if (n) std::memcpy(out, in, n * R);  // (memcpy with a null pointer is undefined even for 0 bytes)
  std::vector<uint8_t> buf(n * R + 1);
  msd_rec(out, buf.data(), n, R, K, 8 * K, width, tiny_max);
  return ST_OK;
}

// Bins after `levels` MSD phases of `width`-bit digits over an already sorted
// array: the maximal runs of records whose top min(8K, levels*width) key bits
// are equal (Sec. 1: after each phase the data is split into bins that are
// processed independently).  Writes run start/size pairs; returns the count
// (or, if `cap` is too small, the count needed).
uint64_t oracle_bins_at_level(const uint8_t* sorted, uint64_t n, uint32_t R, uint32_t K,
                              uint32_t width, uint32_t levels, uint64_t* starts, uint64_t* sizes,
                              uint64_t cap) {
  uint32_t total = 8 * K;
  uint32_t top = std::min<uint64_t>(total, uint64_t(levels) * width);
  uint64_t nb = 0;
  uint64_t i = 0;
  while (i < n) {
    uint64_t j = i + 1;
    while (j < n) {
      bool same = true;
      for (uint32_t p = total - top; p < total; ++p) {
        if (key_bit(sorted + i * R, p) != key_bit(sorted + j * R, p)) {
          same = false;
          break;
        }
      }
      if (!same) break;
      ++j;
    }
    if (nb < cap) {
      starts[nb] = i;
      sizes[nb] = j - i;
    }
    ++nb;
    i = j;
  }
  return nb;
}

// Independent checkers (sortedness; permutation by payload index).
// Returns the first index i with key(i) > key(i+1), or n when sorted.
uint64_t oracle_first_unsorted(const uint8_t* recs, uint64_t n, uint32_t R, uint32_t K) {
  for (uint64_t i = 0; i + 1 < n; ++i) {
    if (key_less(recs + (i + 1) * R, recs + i * R, K)) return i;
  }
  return n;
}

}  // extern "C"
