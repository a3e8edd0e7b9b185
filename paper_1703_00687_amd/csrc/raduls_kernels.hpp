// Device kernels of libraduls (gfx950, wave64).  Included by one translation
// unit per record width; each instantiates the kernels for its R = 8*RW and
// every key width KW = ceil(K/8) <= RW.
//
// The sort is an MSD radix sort of fixed-size records (RADULS2, Sec. 3):
//   round r (large bins):  k_prep     tile counts of the round's bins
//                          k_hist     per-bin digit histogram (+ key spread);
//                                     at the top level optionally also the
//                                     (top, second) digit pair counts, which
//                                     can stand in for round 1's histograms
//                          k_carry    per-range carries (blocked scan)
//                          k_scatter_carry / k_scatter (look-back variant)
//                                     stable scatter into the child bins
//                          k_classify child bins -> next round / LDS jobs
//   then                   k_tiny     jobs of at most 64 records, one wave each
//                          k_mid      bins that fit in LDS, sorted there; tiny
//                                     sub-bins by enumeration sort; finished
//                                     runs left in tmp back to recs
#pragma once

#include "raduls_common.hpp"

namespace raduls {

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// Record buffers are reached through pointers stored in descriptors, so the
// compiler cannot infer their address space and would emit FLAT accesses,
// which also count against the LDS wait counter and stall every LDS wait
// behind outstanding HBM traffic.  These casts make them global accesses.
#define RADULS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const RADULS_GLOBAL T* gmem(const T* p) {
  return (const RADULS_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ RADULS_GLOBAL T* gmem(T* p) {
  return (RADULS_GLOBAL T*)p;
}

// ------------------------------------------------------------ small helpers

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

// A value the same in every lane, made a scalar (wave-uniform) one.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup barrier for LDS hand-offs.  __syncthreads() also orders global
// memory, which makes every wave wait for all of its outstanding global loads
// and stores (vmcnt 0) at each barrier; no barrier in these kernels publishes
// global data to other threads, so waiting for LDS operations (lgkmcnt 0) is
// enough and keeps prefetched loads and write-out stores in flight.  The empty
// asm statements keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // gfx9 encoding: lgkmcnt(0), vmcnt/expcnt not waited
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <int RW>
__device__ __forceinline__ void load_rec(const uint8_t* base, uint64_t idx, uint64_t (&w)[RW]) {
  const RADULS_GLOBAL uint64_t* p = gmem(reinterpret_cast<const uint64_t*>(base)) + idx * RW;
  if constexpr (RW % 2 == 0) {
    const RADULS_GLOBAL u64x2* q = reinterpret_cast<const RADULS_GLOBAL u64x2*>(p);
#pragma unroll
    for (int i = 0; i < RW / 2; ++i) {
      u64x2 v = q[i];
      w[2 * i] = v.x;
      w[2 * i + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < RW; ++i) w[i] = p[i];
  }
}

template <int RW>
__device__ __forceinline__ void store_rec(uint8_t* base, uint64_t idx, const uint64_t* w, bool nt) {
  RADULS_GLOBAL uint64_t* p = gmem(reinterpret_cast<uint64_t*>(base)) + idx * RW;
  if constexpr (RW % 2 == 0) {
    RADULS_GLOBAL u64x2* q = reinterpret_cast<RADULS_GLOBAL u64x2*>(p);
#pragma unroll
    for (int i = 0; i < RW / 2; ++i) {
      u64x2 v;
      v.x = w[2 * i];
      v.y = w[2 * i + 1];
      if (nt) __builtin_nontemporal_store(v, q + i);
      else q[i] = v;
    }
  } else {
#pragma unroll
    for (int i = 0; i < RW; ++i) {
      if (nt) __builtin_nontemporal_store((unsigned long long)w[i], (RADULS_GLOBAL unsigned long long*)p + i);
      else p[i] = w[i];
    }
  }
}

// Key words of a record (word KW-1 most significant), top word masked to the
// key bytes it holds.
template <int KW, class Ptr>
__device__ __forceinline__ void key_of(Ptr w, uint64_t kmask, uint64_t (&k)[KW]) {
#pragma unroll
  for (int i = 0; i < KW; ++i) k[i] = w[i];
  k[KW - 1] &= kmask;
}

// Bits [lo, lo + w) of a multi-word key, 1 <= w <= 16.
template <int KW>
__device__ __forceinline__ uint32_t digit_of(const uint64_t (&k)[KW], uint32_t lo, uint32_t w) {
  const uint32_t wi = lo >> 6, sh = lo & 63;
  uint64_t a = 0, b = 0;
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    a = (uint32_t(j) == wi) ? k[j] : a;
    b = (uint32_t(j) == wi + 1) ? k[j] : b;
  }
  uint64_t v = a >> sh;
  if (sh + w > 64) v |= b << (64 - sh);
  return uint32_t(v) & ((1u << w) - 1u);
}

template <int KW>
__device__ __forceinline__ bool key_lt(const uint64_t (&a)[KW], const uint64_t (&b)[KW]) {
  bool lt = false, decided = false;
#pragma unroll
  for (int i = KW - 1; i >= 0; --i) {
    const bool ne = a[i] != b[i];
    lt = (!decided && ne) ? (a[i] < b[i]) : lt;
    decided = decided || ne;
  }
  return lt;
}

template <int KW>
__device__ __forceinline__ bool key_eq(const uint64_t (&a)[KW], const uint64_t (&b)[KW]) {
  bool eq = true;
#pragma unroll
  for (int i = 0; i < KW; ++i) eq = eq && (a[i] == b[i]);
  return eq;
}

// Index of the highest set bit of a multi-word value, -1 if it is zero.
template <int KW>
__device__ __forceinline__ int top_bit(const uint64_t (&d)[KW]) {
  int r = -1;
#pragma unroll
  for (int i = 0; i < KW; ++i)
    if (d[i]) r = 64 * i + 63 - __clzll((long long)d[i]);
  return r;
}

// Whether a key spread has a bit at or above `bits`: the keys of a bin then
// differ where the bin says they agree (only a root whose first split was
// guessed from a sample can be such a bin; see k_seed_single).
template <int KW>
__device__ __forceinline__ bool spread_above(const uint64_t (&d)[KW], uint32_t bits) {
  bool a = false;
#pragma unroll
  for (int i = 0; i < KW; ++i) {
    const uint32_t b0 = 64u * uint32_t(i);
    const uint64_t m = bits <= b0 ? ~0ull : (bits >= b0 + 64 ? 0ull : ~((1ull << (bits - b0)) - 1ull));
    a = a || (d[i] & m) != 0;
  }
  return a;
}

// How a large bin's records are bucketed in a round: by the digit
// [lob, lob + w) of the key (Sec. 1), or, for a bin marked for an equality
// split (kBinEq), into 0: keys below its equality key, 1: that key, 2: keys
// above it (the key bits stay to be sorted in both ranges).
// The digit width a large bin is split on (its own narrower width, if set).
__device__ __forceinline__ uint32_t bin_width(const Params& P, const Bin& bin) {
  const uint32_t bw = (uint32_t(bin.flags) & kBinWidthMask) >> kBinWidthShift;
  return bw ? bw : P.digit_bits;
}

template <int KW>
struct Bucketing {
  uint32_t lob, w, nb;
  bool eq;
  uint64_t k[KW];
  __device__ __forceinline__ uint32_t of(const uint64_t (&key)[KW]) const {
    if (eq) return key_eq<KW>(key, k) ? 1u : (key_lt<KW>(key, k) ? 0u : 2u);
    return digit_of<KW>(key, lob, w);
  }
};
// The bucketing of bin b of large list `list` (its equality key, if any, is
// read from that list's key table).
template <int KW>
__device__ __forceinline__ Bucketing<KW> bucketing(const Params& P, const Bin& bin, uint32_t list,
                                                   uint32_t b) {
  Bucketing<KW> d;
  d.eq = (bin.flags & kBinEq) != 0;
  d.w = d.eq ? 2u : min(bin_width(P, bin), uint32_t(bin.bits));
  d.lob = d.eq ? uint32_t(bin.bits) : uint32_t(bin.bits) - d.w;
  d.nb = 1u << d.w;
#pragma unroll
  for (int q = 0; q < KW; ++q) d.k[q] = d.eq ? P.L.eqkey[list][uint64_t(b) * 8 + q] : 0ull;
  return d;
}

// Wave-wide OR, returned to every lane: DPP reductions inside each row of 16
// lanes, then the rows combined through the broadcasts of lanes 15 and 31,
// after which lane 63 holds the total.
__device__ __forceinline__ uint32_t wave_or32(uint32_t v) {
  v |= uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v |= uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v |= uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x124, 0xF, 0xF, false));  // row_ror:4
  v |= uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x128, 0xF, 0xF, false));  // row_ror:8
  v |= uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xA, 0xF, false));  // row_bcast:15
  v |= uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xC, 0xF, false));  // row_bcast:31
  return uint32_t(__builtin_amdgcn_readlane(int(v), 63));
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
  return (uint64_t(wave_or32(uint32_t(v >> 32))) << 32) | wave_or32(uint32_t(v));
}

// Inclusive prefix sum over the wave's lanes: DPP shifts inside each row of
// 16 lanes (lanes shifted in from outside the row add 0), then each row adds
// the totals of the rows before it through the broadcasts of lanes 15 and 31.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x111, 0xF, 0xF, false));  // row_shr:1
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x112, 0xF, 0xF, false));  // row_shr:2
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x114, 0xF, 0xF, false));  // row_shr:4
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x118, 0xF, 0xF, false));  // row_shr:8
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xA, 0xF, false));  // row_bcast:15
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xC, 0xF, false));  // row_bcast:31
  return v;
}

// Exclusive prefix sum of one value per thread over threads [0, 256).  Every
// thread of the block must call it (it holds barriers).  scratch: 4 words.
__device__ __forceinline__ void block_exclusive_scan256(uint32_t v, uint32_t* out,
                                                        uint32_t* scratch) {
  const uint32_t t = threadIdx.x;
  uint32_t inc = 0;
  if (t < 256) {
    inc = wave_inclusive_scan(v);
    if ((t & 63) == 63) scratch[t >> 6] = inc;
  }
  lds_barrier();
  if (t < 256) {
    uint32_t add = 0;
    for (uint32_t w = 0; w < (t >> 6); ++w) add += scratch[w];
    out[t] = inc - v + add;
  }
  lds_barrier();
}

// Peers of each lane: the valid lanes of this wave holding the same digit,
// found with one ballot per digit bit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, uint32_t nbits) {
  uint64_t peers = __ballot(valid);
  for (uint32_t b = 0; b < nbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    peers &= bit ? bal : ~bal;
  }
  return peers;
}

// Stable rank of each item among the items of this wave with the same digit,
// counting earlier items first: items are processed in order j, and inside an
// item by lane.  wcnt: this wave's 256 counters in LDS, advanced by the
// number of items per digit.  Only one lane per distinct digit touches wcnt
// in each step, so no atomics are needed.
template <int ITEMS>
__device__ __forceinline__ void wave_rank(const uint32_t (&d)[ITEMS], const bool (&valid)[ITEMS],
                                          uint32_t nbits, uint16_t* wcnt,
                                          uint32_t (&rank)[ITEMS]) {
  const uint64_t lt = lanemask_lt();
  const uint32_t lane = lane_id();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint64_t peers = match_digit(d[j], valid[j], nbits);
    const uint32_t below = __popcll(peers & lt);
    uint32_t old = 0;
    if (valid[j] && below == 0) {
      old = wcnt[d[j]];
      wcnt[d[j]] = uint16_t(old + __popcll(peers));
    }
    const int leader = peers ? (__ffsll((long long)peers) - 1) : int(lane);
    old = __shfl(old, leader);
    rank[j] = old + below;
  }
}

// After wave_rank in all waves and a barrier: turn the per-wave counters into
// exclusive prefixes over waves, write per-digit totals and the exclusive
// prefix over digits.  Contains barriers.
template <int WAVES>
__device__ __forceinline__ void block_digit_scan(uint16_t* cnt, uint32_t* tot, uint32_t* off,
                                                 uint32_t* scratch) {
  const uint32_t t = threadIdx.x;
  uint32_t run = 0;
  if (t < kRadix) {
#pragma unroll 4
    for (int w = 0; w < WAVES; ++w) {
      const uint32_t c = cnt[w * kRadix + t];
      cnt[w * kRadix + t] = uint16_t(run);
      run += c;
    }
    tot[t] = run;
  }
  block_exclusive_scan256(run, off, scratch);
}

__device__ __forceinline__ bool push_bin(Bin* list, uint32_t* count, uint32_t cap, const Bin& b,
                                         uint32_t* err, uint32_t* out_index = nullptr) {
  const uint32_t i = atomicAdd(count, 1u);
  if (i >= cap) {
    atomicOr(err, kErrCapacity);
    return false;
  }
  list[i] = b;
  if (out_index) *out_index = i;
  return true;
}

// Append a bin to the next large list and clear its histogram and key-spread
// rows (they are accumulated with atomics by the next round's k_hist).
// Pushes a large bin for the next round (with its equality key when it is
// marked kBinEq) and clears its histogram row and key spread.
template <int KW>
__device__ __forceinline__ void push_large(const Params& P, uint32_t nxt, const Bin& b,
                                           const uint64_t (&eqk)[KW]) {
  uint32_t i;
  if (!push_bin(P.L.large[nxt], &P.L.ctrl->large_count[nxt], P.L.cap_large, b, &P.L.ctrl->error, &i))
    return;
  uint4* h = reinterpret_cast<uint4*>(P.L.hist[nxt] + uint64_t(i) * kRadix);
  for (int q = 0; q < kRadix / 4; ++q) h[q] = make_uint4(0, 0, 0, 0);
  uint64_t* df = P.L.diff[nxt] + uint64_t(i) * 8;
  for (int q = 0; q < 8; ++q) df[q] = 0;
  if (b.flags & kBinEq) {
#pragma unroll
    for (int q = 0; q < KW; ++q) P.L.eqkey[nxt][uint64_t(i) * 8 + q] = eqk[q];
  }
}

// Whether a large bin about to be pushed is dominated by one key: the
// Boyer-Moore majority candidate of kEqSamples evenly spaced records, kept
// when at least kEqDominant of the samples equal it.  `base` is the bin's
// first record; R the record size.
template <int KW>
__device__ bool dominant_key(const uint8_t* base, uint32_t size, uint32_t R, uint64_t kmask,
                             uint64_t (&cand)[KW]) {
  const RADULS_GLOBAL uint8_t* b8 = gmem(base);
  uint32_t votes = 0;
  for (uint32_t i = 0; i < kEqSamples; ++i) {
    const uint64_t pos = (uint64_t(2 * i + 1) * size) / (2 * kEqSamples);
    uint64_t k[KW];
    key_of<KW>(reinterpret_cast<const RADULS_GLOBAL uint64_t*>(b8 + pos * R), kmask, k);
    if (votes == 0) {
#pragma unroll
      for (int q = 0; q < KW; ++q) cand[q] = k[q];
      votes = 1;
    } else {
      votes += key_eq<KW>(k, cand) ? 1u : uint32_t(-1);
    }
  }
  uint32_t same = 0;
  for (uint32_t i = 0; i < kEqSamples; ++i) {
    const uint64_t pos = (uint64_t(2 * i + 1) * size) / (2 * kEqSamples);
    uint64_t k[KW];
    key_of<KW>(reinterpret_cast<const RADULS_GLOBAL uint64_t*>(b8 + pos * R), kmask, k);
    same += key_eq<KW>(k, cand) ? 1u : 0u;
  }
  return same >= kEqDominant;
}

// Slot in a list for every active lane with `want`: one atomic per wave on
// the list's counter (many thousands of arrays push jobs at once; per-lane
// atomics on one address would serialize).  All active lanes call.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t* counter, bool want) {
  const uint64_t mask = __ballot(want);
  const uint32_t before = uint32_t(__popcll(mask & lanemask_lt()));
  const int leader = mask ? __ffsll((long long)mask) - 1 : 0;
  uint32_t base = 0;
  if (want && int(lane_id()) == leader) base = atomicAdd(counter, uint32_t(__popcll(mask)));
  base = uint32_t(__shfl(int(base), leader));
  return base + before;
}

// Append a sort job for bin b of array a: to the tiny-job list if one wave
// can hold it, else to the LDS-sort list.
__device__ __forceinline__ void push_mid(const Params& P, const Bin& b, const ArrayDesc& a) {
  const bool tiny = b.size <= P.tiny_job;
  const uint32_t it = wave_reserve(&P.L.ctrl->tiny_count, tiny);
  const uint32_t im = wave_reserve(&P.L.ctrl->mid_count, !tiny);
  const uint32_t i = tiny ? it : im;
  if (i >= P.L.cap_mid) {
    atomicOr(&P.L.ctrl->error, kErrCapacity);
    return;
  }
  MidJob j;
  j.src = (b.side ? a.tmp : a.recs) + uint64_t(b.start) * P.R;
  j.dst = a.recs + uint64_t(b.start) * P.R;
  j.size = b.size;
  j.pad[0] = j.pad[1] = j.pad[2] = 0;
  (tiny ? P.L.tiny : P.L.mid)[i] = j;
}

// A finished run of records that sits in tmp, [start, start + size) of array
// `array`, goes back to recs as LDS-sort jobs of at most mid_max records:
// a run whose keys are all equal (or already in order, as an exhausted key's
// buckets are) is its own stable sort, and the sorter moves such a job
// through LDS unchanged without a pass.  So the copies interleave with the
// sort jobs of the same launch, which are bound by their instructions
// rather than by HBM, instead of following them in a launch of their own.
// All threads of the workgroup call (the callers' conditions are uniform);
// the one thread with `want` set supplies the run, and the workgroup writes
// the pieces' descriptors together.
__device__ void push_copy_jobs(const Params& P, bool want, uint32_t array, uint32_t start,
                               uint32_t size) {
  __shared__ uint32_t s_cp[4];  // first list index, start, size, array
  if (!__syncthreads_or(want && size > 0)) return;
  const uint32_t T = P.mid_max;
  if (want && size > 0) {
    const uint32_t pieces = (size + T - 1) / T;
    s_cp[0] = atomicAdd(&P.L.ctrl->mid_count, pieces);
    s_cp[1] = start;
    s_cp[2] = size;
    s_cp[3] = array;
    atomicAdd(&P.L.ctrl->copy_count, pieces);
  }
  __syncthreads();
  const uint32_t base = s_cp[0], st = s_cp[1], sz = s_cp[2];
  const ArrayDesc a = P.L.arrays[s_cp[3]];
  const uint32_t pieces = (sz + T - 1) / T;
  for (uint32_t k = threadIdx.x; k < pieces; k += blockDim.x) {
    if (base + k >= P.L.cap_mid) {
      atomicOr(&P.L.ctrl->error, kErrCapacity);
      break;
    }
    const uint64_t at = uint64_t(st) + uint64_t(k) * T;
    MidJob jb;
    jb.src = a.tmp + at * P.R;
    jb.dst = a.recs + at * P.R;
    jb.size = min(T, sz - k * T);
    jb.pad[0] = jb.pad[1] = jb.pad[2] = 0;
    P.L.mid[base + k] = jb;
  }
  __syncthreads();  // s_cp is written again by the next call
}

// ------------------------------------------------------------ seeding

// Clears the control block and installs the root bin of a single-array call.
//
// With P.spec, the root's first digit is not the key's top byte but the one
// just below the highest key bit in which kSpecSamples evenly spaced records
// differ from the first record (key bits above it are then constant in the
// sample, as when keys are narrower than their field): the top-level pass
// would only find them constant and move nothing.  Round 0's histogram pass
// measures the true spread of the keys; if a record differs above the guess,
// that round moves nothing and the root is pushed again from its true top
// bit, as for a constant digit (the sort then uses one of the rounds that it
// keeps for equality splits).
static __global__ void __launch_bounds__(64) k_seed_single(Params P) {
  Ctrl* c = P.L.ctrl;
  uint32_t top = 8 * P.K;  // the root's bits
  if (P.spec && P.mode == kModeSort && P.n > P.mid_max) {
    const uint32_t kw = (P.K + 7) / 8, lane = threadIdx.x;
    const RADULS_GLOBAL uint64_t* base = gmem(reinterpret_cast<const uint64_t*>(P.recs));
    const uint32_t rw = P.R / 8;
    int tb = -1;
    for (uint32_t q = kw; q-- > 0;) {
      const uint64_t m = q == kw - 1 ? P.kmask : ~0ull;
      const uint64_t k0 = base[q] & m;
      uint64_t d = 0;
      for (uint32_t i = lane; i < kSpecSamples; i += 64) {
        const uint64_t pos = (uint64_t(2 * i + 1) * P.n) / (2 * kSpecSamples);
        d |= (base[pos * rw + q] & m) ^ k0;
      }
      d = wave_or(d);
      if (d) {
        tb = int(64 * q) + 63 - __clzll(static_cast<long long>(d));
        break;
      }
    }
    // (the top-level pair counts take the digit below the first: 16 bits)
    if (tb >= 0) top = max(uint32_t(tb + 1), P.pair ? 16u : 8u);
  }
  if (threadIdx.x == 0) {
    *c = Ctrl{};
    ArrayDesc a;
    a.recs = P.recs;
    a.tmp = P.tmp;
    a.n = P.n;
    P.L.arrays[0] = a;
    Bin b;
    b.start = 0;
    b.size = uint32_t(P.n);
    b.array = 0;
    b.side = 0;
    b.flags = 0;
    if (P.mode == kModeHist || P.mode == kModePartition) {
      b.bits = uint16_t(P.step_bits);
      P.L.large[0][0] = b;
      c->large_count[0] = P.n ? 1 : 0;
    } else {
      b.bits = uint16_t(top);
      if (P.n > P.mid_max) {
        P.L.large[0][0] = b;
        c->large_count[0] = 1;
      } else if (P.n >= 2) {
        push_mid(P, b, a);
      }
    }
  }
  __syncthreads();
  if (P.mode != kModeSort || P.n > P.mid_max) {
    uint32_t* h = P.L.hist[0];
    for (int q = threadIdx.x; q < kRadix; q += 64) h[q] = 0;
    if (threadIdx.x < 8) P.L.diff[0][threadIdx.x] = 0;
  }
}

static __global__ void __launch_bounds__(64) k_zero_ctrl(Params P) {
  if (threadIdx.x == 0) *P.L.ctrl = Ctrl{};
}

// Every array of a batch becomes a root bin: large roots start round 0, small
// ones become LDS jobs directly.
static __global__ void __launch_bounds__(256) k_seed_batch(Params P) {
  Ctrl* c = P.L.ctrl;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < P.count; a += stride) {
    ArrayDesc d = P.d_arrays_in[a];
    bool ok = d.n < (1ull << 32);
    if (ok) {
      const unsigned long long before = atomicAdd(&c->batch_total, (unsigned long long)d.n);
      ok = before + d.n <= P.total_cap;
    }
    if (!ok) {
      atomicOr(&c->error, kErrBatchTotal);
      d.n = 0;
    }
    P.L.arrays[a] = d;
    Bin b;
    b.start = 0;
    b.size = uint32_t(d.n);
    b.array = a;
    b.bits = uint16_t(8 * P.K);
    b.side = 0;
    b.flags = 0;
    if (d.n > P.mid_max) {
      const uint64_t none[1] = {};
      push_large<1>(P, 0, b, none);
    }
    else if (d.n >= 2) push_mid(P, b, d);
  }
}

// ------------------------------------------------------------ round: prep

// Second round of a sort whose top level counted digit pairs (one workgroup
// of 1024 threads; all threads call).  The round's bins are the large
// children of the root, in recs order of their top digit d1, each to be split
// on the second digit, whose counts per d1 are row d1 of pair_hist.  Those
// rows replace this round's histogram pass when
//   - no 16-bit pair counter wrapped: for every d1 the row sums to the root's
//     exact count of d1;
//   - every bin is a child of the root split on the byte below the top one;
//   - the bins are many (>= pair_min_bins, at most one per scatter
//     workgroup) and of even size (largest <= 5/4 of the mean, in tiles),
//     since the scatter then gives each bin one workgroup;
//   - no bin is constant in the second digit (such a bin would jump digits).
// Then every bin's top digit goes to pair_d1, where the scatter and classify
// of this round find the bin's row of pair_hist (and take every key bit
// below the bin's digit as possibly differing).  Returns 1 if so.
__device__ uint32_t pair_decide(const Params& P, uint32_t cur, uint32_t nb, uint32_t tiles,
                                uint32_t max_tiles_thread) {
  __shared__ uint32_t s_pre[kRadix], s_scan[8], s_d1[kRadix], s_nz[kRadix], s_ok, s_max;
  const uint32_t t = threadIdx.x;
  const uint32_t* root = P.L.hist[0];  // the root was bin 0 of round 0
  if (t == 0) {
    s_ok = 1;
    s_max = 0;
  }
  __syncthreads();
  atomicMax(&s_max, max_tiles_thread);
  const uint32_t h0 = t < kRadix ? root[t] : 0u;
  block_exclusive_scan256(h0, s_pre, s_scan);  // all threads; ends with a barrier
  // (children of the root, split on the digit below its first)
  const uint32_t bits = uint32_t(P.L.large[0][0].bits) - 8u;
  if (t == 0 && !(nb >= P.pair_min_bins && nb <= kRadix && nb <= P.grid_hist &&
                  4ull * s_max * nb <= 5ull * tiles))
    s_ok = 0;
  // row d1 = t / 4 of the pair counts, a quarter per thread: its sum must be
  // the root's exact count of d1 (no counter wrapped), and its non-zero
  // entries say whether the second digit is constant in that bin
  {
    const uint32_t d1 = t >> 2, qq = t & 3;
    const uint4* rowp = reinterpret_cast<const uint4*>(P.L.pair_hist + d1 * kRadix + qq * 64);
    uint32_t sum = 0, nz = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint4 v = rowp[k];
      sum += v.x + v.y + v.z + v.w;
      nz += (v.x != 0u) + (v.y != 0u) + (v.z != 0u) + (v.w != 0u);
    }
    sum += __shfl_xor(sum, 1);
    sum += __shfl_xor(sum, 2);
    nz += __shfl_xor(nz, 1);
    nz += __shfl_xor(nz, 2);
    if (qq == 0) {
      s_nz[d1] = nz;
      if (sum != root[d1]) atomicAnd(&s_ok, 0u);
    }
  }
  __syncthreads();
  // bin t: its top digit (the last d with s_pre[d] <= start), and checks
  if (t < nb && t < kRadix) {
    const Bin bn = P.L.large[cur][t];
    uint32_t lo = 0, hi = kRadix;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_pre[mid] <= bn.start) lo = mid;
      else hi = mid;
    }
    s_d1[t] = lo;
    if (bn.bits != bits || bn.side != 1 || bn.array != 0 || bn.flags != 0 || s_pre[lo] != bn.start ||
        root[lo] != bn.size || s_nz[lo] < 2)
      atomicAnd(&s_ok, 0u);
  }
  __syncthreads();
  if (!s_ok) return 0;
  if (t < nb) P.L.pair_d1[t] = s_d1[t];
  return 1;
}

// Tile prefix over the round's large bins (one workgroup).  In the second
// round of a sort whose top level counted digit pairs, also decides whether
// this round takes its histograms from those counts (see pair_decide).
static __global__ void __launch_bounds__(1024) k_prep(Params P, uint32_t cur, uint32_t round) {
  __shared__ uint32_t s_part[16];
  __shared__ unsigned long long s_sz[16];
  Ctrl* c = P.L.ctrl;
  const uint32_t nb = min(c->large_count[cur], P.L.cap_large);
  const Bin* bins = P.L.large[cur];
  const uint32_t t = threadIdx.x, wave = t >> 6, lane = t & 63;
  uint32_t running = 0, max_tiles = 0;
  unsigned long long records = 0;
  for (uint32_t base = 0; base < nb; base += 1024) {
    const uint32_t i = base + t;
    uint32_t v = 0;
    uint32_t sz = 0;
    if (i < nb) {
      sz = bins[i].size;
      v = (sz + P.tile - 1) / P.tile;
    }
    max_tiles = max(max_tiles, v);
    const uint32_t inc = wave_inclusive_scan(v);
    unsigned long long s64 = sz;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s64 += __shfl_xor(s64, o);
    if (lane == 63) s_part[wave] = inc;
    if (lane == 0) s_sz[wave] = s64;
    __syncthreads();
    uint32_t add = 0, tot = 0;
    for (uint32_t w = 0; w < 16; ++w) {
      add += (w < wave) ? s_part[w] : 0;
      tot += s_part[w];
    }
    unsigned long long chunk_rec = 0;
    for (uint32_t w = 0; w < 16; ++w) chunk_rec += s_sz[w];
    if (i < nb) P.L.tile_prefix[i] = running + add + inc - v;
    running += tot;
    records += chunk_rec;
    __syncthreads();
  }
  uint32_t fused = 0;
  if (t == 0) P.L.tile_prefix[nb] = running;
  if (P.pair && round == 1) fused = pair_decide(P, cur, nb, running, max_tiles);
  if (t == 0) {
    c->round_tiles = running;
    c->ticket = 0;
    c->large_count[cur ^ 1] = 0;
    c->fused = fused;
    c->pair_rounds += fused;
    if (nb) {
      c->rounds += 1;
      c->large_bins += nb;
      c->large_records += records;
    }
  }
}

// ------------------------------------------------------------ round: histogram

// Digit histogram of every large bin of the round, and the OR over the bin of
// (key xor first key), which shows whether the digit or the whole key is
// constant.  Workgroups take contiguous tile ranges and accumulate in LDS,
// flushing to the bin's global row when the range crosses into the next bin.
// Also clears the look-back status rows of its tiles and records their bin.
// TOP: 0 for later rounds, 1 for the top level, 2 for the top level of a
// single-array sort with 8-bit digits that also counts the pairs (top digit,
// second digit) of each range in 16-bit LDS counters and stores them to the
// range's row of pair_part (a counter that wraps is caught later because the
// pair counts of a top digit then fall short of its exact count).  Those
// counters fill the LDS, so that variant runs one workgroup per CU.
template <int RW, int KW, int TOP>
__global__ void __launch_bounds__(kScatterBlock, TOP == 2 ? 1 : 8) k_hist(Params P, uint32_t cur) {
  constexpr int ITEMS = scatter_items(RW);
  constexpr int W = kScatterWaves;
  constexpr uint32_t TILE = kScatterBlock * ITEMS;
  constexpr bool pair = TOP == 2;
  __shared__ uint32_t s_cnt[W * kRadix];
  __shared__ unsigned long long s_diff[W][KW];
  extern __shared__ __align__(16) uint32_t s_pair[];  // [kPairWords] when pair

  const Ctrl* c = P.L.ctrl;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (pair) {  // the pair totals are summed into here after this kernel
    for (uint32_t q = blockIdx.x * kScatterBlock + tid; q < 2 * kPairWords;
         q += gridDim.x * kScatterBlock)
      P.L.pair_hist[q] = 0;
  }
  if (!TOP && c->fused) return;  // histograms already taken from the pair counts
  const uint32_t total = c->round_tiles;
  const uint32_t nbins = min(c->large_count[cur], P.L.cap_large);
  if (total == 0) return;
  const uint32_t t0 = uint32_t(uint64_t(total) * blockIdx.x / gridDim.x);
  const uint32_t t1 = uint32_t(uint64_t(total) * (blockIdx.x + 1) / gridDim.x);
  if (t0 >= t1) return;
  if (pair) {
    for (uint32_t q = tid; q < kPairWords; q += kScatterBlock) s_pair[q] = 0;
  }

  // clear look-back rows of this range (only that scatter uses them)
  if (P.lookback) {
    uint4* st = reinterpret_cast<uint4*>(P.L.status + uint64_t(t0) * kRadix);
    const uint64_t nq = uint64_t(t1 - t0) * kRadix / 2;
    for (uint64_t q = tid; q < nq; q += kScatterBlock) st[q] = make_uint4(0, 0, 0, 0);
  }
  for (int q = lane; q < kRadix; q += kWave) s_cnt[wave * kRadix + q] = 0;

  const uint32_t* tp = P.L.tile_prefix;
  uint32_t lo = 0, hi = nbins;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tp[mid] <= t0) lo = mid;
    else hi = mid;
  }
  uint32_t b = lo;
  const uint32_t b_first = lo;

  uint64_t dacc[KW];
#pragma unroll
  for (int i = 0; i < KW; ++i) dacc[i] = 0;

  auto flush = [&](uint32_t bb, bool last) {
#pragma unroll
    for (int i = 0; i < KW; ++i) {
      const uint64_t v = wave_or(dacc[i]);
      if (lane == 0) s_diff[wave][i] = v;
      dacc[i] = 0;
    }
    __syncthreads();
    if (tid < kRadix) {
      uint32_t s = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        s += s_cnt[w * kRadix + tid];
        s_cnt[w * kRadix + tid] = 0;
      }
      if (s) atomicAdd(P.L.hist[cur] + uint64_t(bb) * kRadix + tid, s);
      // counts of the range's last bin segment, for the carry scan
      if (last) P.L.wg_tail[uint64_t(blockIdx.x) * kRadix + tid] = s;
    }
    if (tid < KW) {
      unsigned long long v = 0;
      for (int w = 0; w < W; ++w) v |= s_diff[w][tid];
      if (v) atomicOr((unsigned long long*)(P.L.diff[cur] + uint64_t(bb) * 8 + tid), v);
    }
    __syncthreads();
  };

  // Tiles are software-pipelined: the keys of tile t+1 are loaded while tile
  // t is counted.  Counting needs no order, so every lane adds its items to
  // its wave's counters with LDS atomics.
  Bin bin = P.L.large[cur][b];
  ArrayDesc arr = P.L.arrays[bin.array];
  const uint8_t* src = bin.side ? arr.tmp : arr.recs;
  uint64_t key0[KW];
  key_of<KW>(gmem(reinterpret_cast<const uint64_t*>(src)) + uint64_t(bin.start) * RW, P.kmask, key0);
  Bucketing<KW> bk = bucketing<KW>(P, bin, cur, b);

  // the tile to load: its bin (bl) and that bin's tiles, records and source,
  // kept in registers so that the loads of a tile wait for nothing (a load of
  // a descriptor would wait for every key load still in flight); they are
  // reread only when the tiles cross into the next bin
  uint32_t bl = b;
  uint32_t bl_first = tp[b], bl_end = b + 1 < nbins ? tp[b + 1] : 0xFFFFFFFFu;
  uint32_t bl_start = bin.start, bl_size = bin.size;
  const uint8_t* bl_src = src;
  auto load_tile = [&](uint32_t t, uint64_t (&kt)[ITEMS][KW], uint32_t& tn_out) {
    if (t >= bl_end) {
      while (bl + 1 < nbins && t >= tp[bl + 1]) ++bl;
      bl_first = tp[bl];
      bl_end = bl + 1 < nbins ? tp[bl + 1] : 0xFFFFFFFFu;
      const Bin bb = P.L.large[cur][bl];
      const ArrayDesc aa = P.L.arrays[bb.array];
      bl_src = bb.side ? aa.tmp : aa.recs;
      bl_start = bb.start;
      bl_size = bb.size;
    }
    const RADULS_GLOBAL uint64_t* sw = gmem(reinterpret_cast<const uint64_t*>(bl_src));
    const uint32_t k = t - bl_first;
    const uint32_t tbeg = bl_start + k * P.tile;
    const uint32_t tn = min(P.tile, bl_size - k * P.tile);
    const uint32_t ipw = (tn + kWave * W - 1) / (kWave * W);
    tn_out = tn;
    // Raw, unconditional loads (lanes past the tile reread its last record,
    // which is not counted): a load under a branch, or masking the top word
    // here, would make the loads wait at once instead of when the tile is
    // counted.
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t i = wave * ipw * kWave + j * kWave + lane;
      const uint32_t ii = (uint32_t(j) < ipw && i < tn) ? i : tn - 1u;
      const RADULS_GLOBAL uint64_t* kp = sw + uint64_t(tbeg + ii) * RW;
#pragma unroll
      for (int q = 0; q < KW; ++q) kt[j][q] = kp[q];
    }
  };
  uint64_t kt[ITEMS][KW];
  uint32_t tnr = 0;
  load_tile(t0, kt, tnr);
  uint32_t b_end = b + 1 < nbins ? tp[b + 1] : 0xFFFFFFFFu;
  for (uint32_t t = t0; t < t1; ++t) {
    if (t >= b_end) {
      while (b + 1 < nbins && t >= tp[b + 1]) {
        flush(b, false);
        ++b;
        bin = P.L.large[cur][b];
        arr = P.L.arrays[bin.array];
        src = bin.side ? arr.tmp : arr.recs;
        key_of<KW>(gmem(reinterpret_cast<const uint64_t*>(src)) + uint64_t(bin.start) * RW, P.kmask, key0);
        bk = bucketing<KW>(P, bin, cur, b);
      }
      b_end = b + 1 < nbins ? tp[b + 1] : 0xFFFFFFFFu;
    }
    if (tid == 0) P.L.tile_bin[t] = b;
    const uint32_t tn = tnr;
    const uint32_t ipw = (tn + kWave * W - 1) / (kWave * W);
    const uint32_t lob = bk.lob;
    uint32_t dg[ITEMS];
    bool valid[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t i = wave * ipw * kWave + j * kWave + lane;
      valid[j] = (uint32_t(j) < ipw) && (i < tn);
      dg[j] = 0;
      kt[j][KW - 1] &= P.kmask;
      if (valid[j]) {
        dg[j] = bk.of(kt[j]);
#pragma unroll
        for (int q = 0; q < KW; ++q) dacc[q] |= kt[j][q] ^ key0[q];
      }
    }
    uint32_t d2[ITEMS];
    if (pair) {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) d2[j] = valid[j] ? digit_of<KW>(kt[j], lob - 8, 8) : 0u;
    }
    if (t + 1 < t1) load_tile(t + 1, kt, tnr);
    uint32_t* wc = s_cnt + wave * kRadix;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (valid[j]) atomicAdd(&wc[dg[j]], 1u);
    if (pair) {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j)
        if (valid[j]) atomicAdd(&s_pair[(dg[j] << 7) | (d2[j] >> 1)], 1u << ((d2[j] & 1u) << 4));
    }
  }
  flush(b, true);
  if (pair) {  // flush ends with a barrier
    uint4* dstp = reinterpret_cast<uint4*>(P.L.pair_part + uint64_t(blockIdx.x) * kPairWords);
    const uint4* srcp = reinterpret_cast<const uint4*>(s_pair);
    for (uint32_t q = tid; q < kPairWords / 4; q += kScatterBlock) dstp[q] = srcp[q];
  }
  if (tid == 0) {
    // bit 0: the range starts a bin; bit 1: the whole range lies in one bin
    P.L.wg_flag[blockIdx.x] = (t0 == tp[b_first] ? 1u : 0u) | (b_first == b ? 2u : 0u);
  }
}

// Sum of the per-range pair counts of the top-level histogram pass: thread
// (word q, group g) adds word q over the ranges of group g and adds both
// 16-bit halves, the pairs (d1, 2 * (q & 127)) and (d1, 2 * (q & 127) + 1) of
// top digit d1 = q >> 7, into pair_hist.  Ranges without tiles wrote nothing.
constexpr uint32_t kPairGroups = 8;
static __global__ void __launch_bounds__(256) k_pair_reduce(Params P, uint32_t nranges) {
  const Ctrl* c = P.L.ctrl;
  const uint32_t total = c->round_tiles;
  const uint32_t q = (blockIdx.x % (kPairWords / 256)) * 256 + threadIdx.x;
  const uint32_t g = blockIdx.x / (kPairWords / 256);
  const uint32_t h0 = uint32_t(uint64_t(nranges) * g / kPairGroups);
  const uint32_t h1 = uint32_t(uint64_t(nranges) * (g + 1) / kPairGroups);
  uint32_t lo = 0, hi = 0;
#pragma unroll 8
  for (uint32_t h = h0; h < h1; ++h) {
    const uint32_t t0 = uint32_t(uint64_t(total) * h / nranges);
    const uint32_t t1 = uint32_t(uint64_t(total) * (h + 1) / nranges);
    const uint32_t v = t0 < t1 ? P.L.pair_part[uint64_t(h) * kPairWords + q] : 0u;
    lo += v & 0xFFFFu;
    hi += v >> 16;
  }
  if (lo) atomicAdd(&P.L.pair_hist[2 * q], lo);
  if (hi) atomicAdd(&P.L.pair_hist[2 * q + 1], hi);
}

// Carry of every histogram range: the per-digit count of records of the
// range's first bin that lie in earlier ranges (the blocked form of the
// exclusive scan over tiles).  After range h the running count R is the
// range's own tail when h starts a bin or spans more than one bin, else the
// previous R plus that tail; a range that starts a bin carries 0, any other
// carries the R of the range before it.  That is a segmented scan over the
// ranges, done in parallel: one workgroup per digit, kMaxRanges / 1024 ranges
// per thread.
static __global__ void __launch_bounds__(1024) k_carry(Params P, uint32_t nranges) {
  constexpr uint32_t kPer = kMaxRanges / 1024;
  __shared__ uint32_t s_sum[16], s_flag[16];
  const Ctrl* c = P.L.ctrl;
  const uint32_t total = c->round_tiles;
  if (total == 0 || c->fused) return;
  const uint32_t d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t per = (nranges + 1023) / 1024;
  uint32_t tail[kPer];
  bool start[kPer], head[kPer], live[kPer];
  uint32_t run = 0;
  bool any = false;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t g = tid * per + k;
    live[k] = false;
    tail[k] = 0;
    start[k] = head[k] = false;
    if (k < per && g < nranges) {
      const uint32_t t0 = uint32_t(uint64_t(total) * g / nranges);
      const uint32_t t1 = uint32_t(uint64_t(total) * (g + 1) / nranges);
      if (t0 < t1) {  // empty ranges pass the running count through
        const uint32_t f = P.L.wg_flag[g];
        live[k] = true;
        tail[k] = P.L.wg_tail[uint64_t(g) * kRadix + d];
        start[k] = f & 1u;
        head[k] = start[k] || !(f & 2u);
      }
    }
    run = head[k] ? tail[k] : run + tail[k];
    any = any || head[k];
  }
  // exclusive segmented scan of (any, run) over the threads
  uint32_t s = run, f = any;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t s2 = __shfl_up(s, o), f2 = __shfl_up(f, o);
    if (lane >= uint32_t(o)) {
      s = f ? s : s2 + s;
      f = f | f2;
    }
  }
  if (lane == 63) {
    s_sum[wave] = s;
    s_flag[wave] = f;
  }
  uint32_t es = __shfl_up(s, 1), ef = __shfl_up(f, 1);
  if (lane == 0) es = ef = 0;
  __syncthreads();
  uint32_t ps = 0;  // R after everything before this wave
  for (uint32_t w = 0; w < wave; ++w) ps = s_flag[w] ? s_sum[w] : ps + s_sum[w];
  uint32_t r = ef ? es : ps + es;  // R before this thread's first range
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    if (!live[k]) continue;
    const uint32_t g = tid * per + k;
    P.L.wg_carry[uint64_t(g) * kRadix + d] = start[k] ? 0u : r;
    r = head[k] ? tail[k] : r + tail[k];
  }
}

// ------------------------------------------------------------ round: scatter

// Stable scatter of every active large bin (Sec. 3.2 buffered scatter, done
// the GPU way).  Each tile ranks its records by digit inside the wave (ballot
// matching) and across waves (LDS counters), gets the exclusive prefix of its
// digit counts over the earlier tiles of its bin, stages the tile in LDS in
// digit order and writes every digit's run as consecutive, coalesced records.
// The prefix comes either from the carry scan (LOOKBACK = 0: the workgroup
// walks the same contiguous tile range the histogram pass used, starting
// from that range's carry) or from a decoupled look-back over tiles taken in
// ticket order (LOOKBACK = 1).
template <int RW, int KW, int TOP, int LOOKBACK>
__global__ void __launch_bounds__(kScatterBlock) k_scatter(Params P, uint32_t cur) {
  constexpr int ITEMS = scatter_items(RW);
  constexpr int W = kScatterWaves;
  constexpr uint32_t TILE = kScatterBlock * ITEMS;
  extern __shared__ __align__(16) uint8_t smem[];
  uint64_t* s_rec = reinterpret_cast<uint64_t*>(smem);
  uint8_t* s_dig = reinterpret_cast<uint8_t*>(s_rec + TILE * RW);
  uint16_t* s_cnt = reinterpret_cast<uint16_t*>(s_dig + TILE);
  uint32_t* s_tot = reinterpret_cast<uint32_t*>(s_cnt + W * kRadix);
  uint32_t* s_off = s_tot + kRadix;
  uint32_t* s_binoff = s_off + kRadix;
  uint64_t* s_gbase = reinterpret_cast<uint64_t*>(s_binoff + kRadix);
  __shared__ uint32_t s_ticket;
  __shared__ uint32_t s_scan[8];

  Ctrl* c = P.L.ctrl;
  const uint32_t total = c->round_tiles;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const bool nt = P.nontemporal != 2;

  // carry mode: this workgroup's tile range and running prefix (thread d)
  const uint32_t r0 = LOOKBACK ? 0u : uint32_t(uint64_t(total) * blockIdx.x / gridDim.x);
  const uint32_t r1 = LOOKBACK ? 0u : uint32_t(uint64_t(total) * (blockIdx.x + 1) / gridDim.x);
  uint32_t running = 0;
  if (!LOOKBACK && tid < kRadix && r0 < r1)
    running = P.L.wg_carry[uint64_t(blockIdx.x) * kRadix + tid];

  for (uint32_t it = r0;; ++it) {
    uint32_t t;
    if constexpr (LOOKBACK) {
      if (tid == 0) s_ticket = atomicAdd(&c->ticket, 1u);
      __syncthreads();
      t = s_ticket;
      if (t >= total) break;
    } else {
      t = it;
      if (t >= r1) break;
    }
    const uint32_t b = P.L.tile_bin[t];
    const Bin bin = P.L.large[cur][b];
    const uint32_t k = t - P.L.tile_prefix[b];
    const ArrayDesc arr = P.L.arrays[bin.array];
    const uint8_t* src = bin.side ? arr.tmp : arr.recs;
    uint8_t* dst = bin.side ? arr.recs : arr.tmp;
    const Bucketing<KW> bk = bucketing<KW>(P, bin, cur, b);
    const uint32_t nb = bk.nb;

    if (!LOOKBACK && k == 0) running = 0;  // a new bin starts inside the range
    const uint32_t h = tid < nb ? P.L.hist[cur][uint64_t(b) * kRadix + tid] : 0;
    bool active = true;
    if (P.mode != kModePartition) {
      uint64_t any = 0;
#pragma unroll
      for (int i = 0; i < KW; ++i) any |= P.L.diff[cur][uint64_t(b) * 8 + i];
      active = any != 0;
      // a digit shared by the whole bin is skipped without moving it
      active = active && !__syncthreads_or(tid < nb && h == bin.size);
    }
    if (!active) {
      __syncthreads();
      continue;
    }
    block_exclusive_scan256(h, s_binoff, s_scan);

    const uint32_t tbeg = bin.start + k * P.tile;
    const uint32_t tn = min(P.tile, bin.size - k * P.tile);
    const uint32_t ipw = (tn + kWave * W - 1) / (kWave * W);
    uint64_t rec[ITEMS][RW];
    uint32_t dg[ITEMS], rank[ITEMS];
    bool valid[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t i = wave * ipw * kWave + j * kWave + lane;
      valid[j] = (uint32_t(j) < ipw) && (i < tn);
      dg[j] = 0;
      if (valid[j]) {
        load_rec<RW>(src, uint64_t(tbeg) + i, rec[j]);
        uint64_t key[KW];
        key_of<KW>(rec[j], P.kmask, key);
        dg[j] = bk.of(key);
      }
    }
    uint16_t* wc = s_cnt + wave * kRadix;
    for (int q = lane; q < kRadix; q += kWave) wc[q] = 0;
    wave_rank<ITEMS>(dg, valid, bk.w, wc, rank);
    __syncthreads();
    block_digit_scan<W>(s_cnt, s_tot, s_off, s_scan);

    if (!LOOKBACK && tid < nb) {
      s_gbase[tid] = uint64_t(bin.start) + s_binoff[tid] + running - s_off[tid];
      running += s_tot[tid];
    }
    // publish this tile's counts, then look back for the exclusive prefix
    if (LOOKBACK && tid < nb) {
      uint64_t* row = P.L.status + uint64_t(t) * kRadix;
      const uint64_t cnt = s_tot[tid];
      uint64_t excl = 0;
      if (k == 0) {
        __hip_atomic_store(row + tid, kFlagPrefix | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(row + tid, kFlagAggregate | cnt, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        // walk back over earlier tiles of the bin, reading kLookback of them
        // per round trip; stop at the first inclusive prefix
        const uint32_t first = P.L.tile_prefix[b];
        uint32_t j = t - 1;
        const uint64_t t_start = wall_clock64();
        uint32_t spins = 0;
        bool done = false;
        while (!done) {
          const uint32_t nr = min(uint32_t(kLookback), j - first + 1);
          uint64_t v[kLookback];
#pragma unroll
          for (int i = 0; i < kLookback; ++i)
            v[i] = uint32_t(i) < nr ? __hip_atomic_load(P.L.status + uint64_t(j - i) * kRadix + tid,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                    : 0;
          uint32_t used = 0;
#pragma unroll
          for (int i = 0; i < kLookback; ++i) {
            if (done || uint32_t(i) >= nr || used != uint32_t(i)) continue;
            const uint64_t flag = v[i] >> 62;
            if (flag == 0) continue;  // not published yet: re-read from here
            excl += v[i] & kValueMask;
            ++used;
            if (flag == 2) done = true;
          }
          if (done) break;
          j -= used;
          if (used == 0) {
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 255) == 0) {
              // bounded wait: 0.2 s at the 100 MHz constant clock, or another
              // wave already gave up
              if (wall_clock64() - t_start > 20000000ull ||
                  __hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                      kErrSpin) {
                atomicOr(&c->error, kErrSpin);
                break;
              }
            }
          }
        }
        __hip_atomic_store(row + tid, kFlagPrefix | (excl + cnt), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      s_gbase[tid] = uint64_t(bin.start) + s_binoff[tid] + excl - s_off[tid];
    }

    // stage the tile in digit order
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (valid[j]) {
        const uint32_t pos = s_off[dg[j]] + wc[dg[j]] + rank[j];
#pragma unroll
        for (int q = 0; q < RW; ++q) s_rec[pos * RW + q] = rec[j][q];
        s_dig[pos] = uint8_t(dg[j]);
      }
    }
    __syncthreads();
    bool oob = false;
    for (uint32_t p = tid; p < tn; p += kScatterBlock) {
      const uint32_t d = s_dig[p];
      const uint64_t at = s_gbase[d] + p;
      // never write outside the bin, whatever the counts say
      if (at - bin.start < bin.size) store_rec<RW>(dst, at, s_rec + uint64_t(p) * RW, nt);
      else oob = true;
    }
    if (oob) atomicOr(&c->error, kErrBounds);
    __syncthreads();
  }
}

// Stable scatter in carry mode (Sec. 3.2 buffered scatter, done the GPU way).
// The workgroup walks the same contiguous tile range the histogram pass gave
// it, starting from that range's carry.  Each tile ranks its records by digit
// inside the wave (ballot matching) and across waves (LDS counters), stages
// them in LDS in digit order and writes every digit's run as consecutive,
// coalesced records.  The next tile's loads are issued as soon as the current
// tile is staged, so they overlap its write-out.
template <int RW, int KW, int TOP>
__global__ void __launch_bounds__(kScatterBlock) k_scatter_carry(Params P, uint32_t cur) {
  constexpr int ITEMS = scatter_items(RW);
  constexpr int W = kScatterWaves;
  constexpr uint32_t TILE = kScatterBlock * ITEMS;
  extern __shared__ __align__(16) uint8_t smem[];
  uint64_t* s_rec = reinterpret_cast<uint64_t*>(smem);          // tile, input order
  uint16_t* s_perm = reinterpret_cast<uint16_t*>(s_rec + TILE * RW);  // position -> slot
  uint16_t* s_cnt = s_perm + TILE;
  uint32_t* s_tot = reinterpret_cast<uint32_t*>(s_cnt + W * kRadix);
  uint32_t* s_off = s_tot + kRadix;
  uint32_t* s_binoff = s_off + kRadix;
  uint64_t* s_gbase = reinterpret_cast<uint64_t*>(s_binoff + kRadix);
  // line buffers: per digit up to one line of records not yet stored, the
  // limit below which a tile's records are stored now, where the buffer's
  // records start (new and old) and how many old ones are stored now
  constexpr bool LINES = scatter_lines(RW);
  constexpr uint32_t LREC = 16u / RW;  // records per 128-byte line
  uint64_t* s_line = s_gbase + kRadix;
  uint64_t* s_lim = s_line + (LINES ? kRadix * 16 : 0);
  uint64_t* s_ncst = s_lim + kRadix;
  uint32_t* s_fl = reinterpret_cast<uint32_t*>(s_ncst + kRadix);
  __shared__ uint32_t s_scan[8];

  Ctrl* c = P.L.ctrl;
  const uint32_t total = c->round_tiles;
  uint32_t r0 = uint32_t(uint64_t(total) * blockIdx.x / gridDim.x);
  uint32_t r1 = uint32_t(uint64_t(total) * (blockIdx.x + 1) / gridDim.x);
  // histograms from the pair counts: workgroup i sorts the whole bin i
  const bool whole_bin = !TOP && c->fused;
  if (whole_bin) {
    const uint32_t nbins = min(c->large_count[cur], P.L.cap_large);
    r0 = blockIdx.x < nbins ? P.L.tile_prefix[blockIdx.x] : 0u;
    r1 = blockIdx.x < nbins ? P.L.tile_prefix[blockIdx.x + 1] : 0u;
  }
  if (r0 >= r1) return;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const bool nt = P.nontemporal != 2;
  uint32_t running =
      tid < kRadix && !whole_bin ? P.L.wg_carry[uint64_t(blockIdx.x) * kRadix + tid] : 0u;
  uint64_t lcst = 0;   // thread d: global index of the first buffered record of digit d
  uint32_t lcnt = 0;   // thread d: buffered records of digit d
  bool lines_on = false;  // the destination's lines align with records

  // state of the bin the current tile belongs to (uniform), including its
  // tile range [bt0, bt1), kept in registers: a global load inside the tile
  // loop would make it wait for every store still in flight
  uint32_t b = 0, nb = 0, bt0 = 0, bt1 = 0;
  Bucketing<KW> bk{};
  Bin bin{};
  const uint8_t* src = nullptr;
  uint8_t* dst = nullptr;
  bool active = false;
  auto enter_bin = [&](uint32_t t) {
    b = whole_bin ? blockIdx.x : P.L.tile_bin[t];
    bt0 = P.L.tile_prefix[b];
    bt1 = P.L.tile_prefix[b + 1];
    bin = P.L.large[cur][b];
    const ArrayDesc arr = P.L.arrays[bin.array];
    src = bin.side ? arr.tmp : arr.recs;
    dst = bin.side ? arr.recs : arr.tmp;
    lines_on = LINES && (reinterpret_cast<uintptr_t>(dst) & 127u) == 0;
    bk = bucketing<KW>(P, bin, cur, b);
    nb = bk.nb;
    const uint32_t* hrow = whole_bin ? P.L.pair_hist + P.L.pair_d1[b] * kRadix
                                     : P.L.hist[cur] + uint64_t(b) * kRadix;
    const uint32_t h = tid < nb ? hrow[tid] : 0;
    active = true;
    if (P.mode != kModePartition) {
      uint64_t any = whole_bin ? 1u : 0u;  // (a bin of pair counts is never constant)
      uint64_t dw[KW];
#pragma unroll
      for (int i = 0; i < KW; ++i) {
        dw[i] = whole_bin ? 0ull : P.L.diff[cur][uint64_t(b) * 8 + i];
        any |= dw[i];
      }
      // all keys equal, a digit shared by the whole bin, or keys that differ
      // above the bin's bits (a wrong guess of the root's top): nothing moves
      active = any != 0 && !spread_above<KW>(dw, bin.bits) &&
               !__syncthreads_or(tid < nb && h == bin.size);
    }
    if (active) block_exclusive_scan256(h, s_binoff, s_scan);
  };

  uint64_t rec[ITEMS][RW];
  auto tile_span = [&](uint32_t t, uint32_t& tbeg, uint32_t& tn, uint32_t& ipw) {
    const uint32_t k = t - bt0;
    tbeg = bin.start + k * P.tile;
    tn = min(P.tile, bin.size - k * P.tile);
    ipw = (tn + kWave * W - 1) / (kWave * W);
  };
  auto issue_loads = [&](uint32_t t) {
    uint32_t tbeg, tn, ipw;
    tile_span(t, tbeg, tn, ipw);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t i = wave * ipw * kWave + j * kWave + lane;
      if (uint32_t(j) < ipw && i < tn) load_rec<RW>(src, uint64_t(tbeg) + i, rec[j]);
    }
  };

  uint32_t t = r0;
  enter_bin(t);
  if (active) issue_loads(t);
  __builtin_amdgcn_s_waitcnt(0x3F70);
  while (t < r1) {
    if (t == bt0) running = 0;  // a new bin starts inside the range
    uint32_t tbeg, tn, ipw;
    tile_span(t, tbeg, tn, ipw);
    uint32_t dg[ITEMS];
    bool valid[ITEMS];
    const uint32_t next = t + 1;
    const bool same = next < r1 && next < bt1;
    if (active) {
      // the tile into LDS in input order and its digits into registers; the
      // registers are then free for the next tile's loads, which stay in
      // flight through the ranking and the stores of this tile
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = wave * ipw * kWave + j * kWave + lane;
        valid[j] = (uint32_t(j) < ipw) && (i < tn);
        dg[j] = 0;
        if (valid[j]) {
          uint64_t key[KW];
          key_of<KW>(rec[j], P.kmask, key);
          dg[j] = bk.of(key);
#pragma unroll
          for (int q = 0; q < RW; ++q) s_rec[uint64_t(i) * RW + q] = rec[j][q];
        }
      }
      if (same) issue_loads(next);
      uint32_t rank[ITEMS];
      uint16_t* wc = s_cnt + wave * kRadix;
      for (int q = lane; q < kRadix; q += kWave) wc[q] = 0;
      wave_rank<ITEMS>(dg, valid, bk.w, wc, rank);
      lds_barrier();
      block_digit_scan<W>(s_cnt, s_tot, s_off, s_scan);
      if (tid < nb) {
        const uint64_t g0 = uint64_t(bin.start) + s_binoff[tid] + running;  // first record of d
        s_gbase[tid] = g0 - s_off[tid];
        running += s_tot[tid];
        if (LINES && lines_on) {
          // whole lines of [buffered records, this tile's records) are
          // stored now; the tail (less than a line) stays buffered
          const uint64_t A = lcnt ? lcst : g0, E = g0 + s_tot[tid];
          const uint64_t Eal = E & ~uint64_t(LREC - 1);
          if (Eal > A) {
            s_lim[tid] = Eal;
            s_fl[tid] = lcnt;
            lcst = Eal;
            lcnt = uint32_t(E - Eal);
          } else {
            s_lim[tid] = A;
            s_fl[tid] = 0;
            lcst = A;
            lcnt = uint32_t(E - A);
          }
          s_ncst[tid] = lcst;
        }
      }
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        if (valid[j]) {
          const uint32_t pos = s_off[dg[j]] + wc[dg[j]] + rank[j];
          s_perm[pos] = uint16_t(wave * ipw * kWave + j * kWave + lane);
        }
      }
      lds_barrier();
    }
    // The next tile's loads have landed before this tile's stores leave, so
    // the next tile does not wait for these stores (on gfx9 one in-order
    // counter covers loads and stores).  The wait is on every path, as are
    // the ones after the other places that issue loads, so that the compiler
    // sees the tile's records complete at the top of the loop and places no
    // wait of its own there.
    __builtin_amdgcn_s_waitcnt(0x3F70);  // gfx9 encoding: vmcnt(0), lgkmcnt/expcnt not waited
    if (active) {
      bool oob = false;
      if (LINES && lines_on) {
        // buffered records completing a line go out first (they end right
        // before the digit's first record of this tile), then the tile:
        // records below their digit's limit are stored, the rest buffered
        for (uint32_t i = tid; i < kRadix * LREC; i += kScatterBlock) {
          const uint32_t d = i / LREC, k = i % LREC;
          if (d < nb && k < s_fl[d]) {
            const uint64_t at = s_gbase[d] + s_off[d] - s_fl[d] + k;
            if (at - bin.start < bin.size) store_rec<RW>(dst, at, s_line + uint64_t(i) * RW, nt);
            else oob = true;
          }
        }
        lds_barrier();  // those buffer slots are refilled below
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          const uint32_t p = j * kScatterBlock + tid;
          if (p < tn) {
            const uint32_t sl = s_perm[p];
            const uint64_t* r = s_rec + uint64_t(sl) * RW;
            uint64_t key[KW];
            key_of<KW>(r, P.kmask, key);
            const uint32_t d = bk.of(key);
            const uint64_t at = s_gbase[d] + p;
            if (at < s_lim[d]) {
              // never write outside the bin, whatever the counts say
              if (at - bin.start < bin.size) store_rec<RW>(dst, at, r, nt);
              else oob = true;
            } else {
              const uint64_t slot = at - s_ncst[d];
              if (slot < LREC) {
#pragma unroll
                for (int q = 0; q < RW; ++q) s_line[(uint64_t(d) * LREC + slot) * RW + q] = r[q];
              } else {
                oob = true;
              }
            }
          }
        }
      } else {
        // unrolled so that every LDS read of the write-out is in flight at once
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          const uint32_t p = j * kScatterBlock + tid;
          if (p < tn) {
            const uint32_t sl = s_perm[p];
            const uint64_t* r = s_rec + uint64_t(sl) * RW;
            uint64_t key[KW];
            key_of<KW>(r, P.kmask, key);
            const uint32_t d = bk.of(key);
            const uint64_t at = s_gbase[d] + p;
            // never write outside the bin, whatever the counts say
            if (at - bin.start < bin.size) store_rec<RW>(dst, at, r, nt);
            else oob = true;
          }
        }
      }
      if (oob) atomicOr(&c->error, kErrBounds);
    }
    lds_barrier();
    t = next;
    if (LINES && lines_on && active && (t >= r1 || !same)) {
      // the bin's part of this range ends: its buffered records go out as
      // they are (at most a partial line per digit)
      if (tid < nb) {
        bool bad = false;
        for (uint32_t k = 0; k < lcnt && k < LREC; ++k) {
          const uint64_t at = lcst + k;
          if (at - bin.start < bin.size) store_rec<RW>(dst, at, s_line + (uint64_t(tid) * LREC + k) * RW, nt);
          else bad = true;
        }
        if (bad) atomicOr(&c->error, kErrBounds);
      }
      lcnt = 0;
      lds_barrier();  // the buffers are reused by the next bin
    }
    if (t < r1 && !same) {
      enter_bin(t);
      if (active) issue_loads(t);
      __builtin_amdgcn_s_waitcnt(0x3F70);
    }
  }
}

// ------------------------------------------------------------ round: classify

constexpr uint32_t kNoChild = 0xFFFFu;

// Highest set bit below position i of a 256-bit mask held as four words, or -1.
__device__ __forceinline__ int mask_prev256(const uint64_t* m, uint32_t i) {
  int w = int(i >> 6);
  uint64_t x = m[w] & ((1ull << (i & 63u)) - 1ull);
  while (!x) {
    if (--w < 0) return -1;
    x = m[w];
  }
  return (w << 6) + 63 - __clzll(x);
}

// Lowest set bit above position i of a 256-bit mask, or n if there is none
// below n.
__device__ __forceinline__ uint32_t mask_next256(const uint64_t* m, uint32_t i, uint32_t n) {
  const uint32_t q = i + 1;
  if (q >= 256u) return n;
  uint32_t w = q >> 6;
  uint64_t x = m[w] & (~0ull << (q & 63u));
  while (!x) {
    if (++w >= 4u) return n;
    x = m[w];
  }
  const uint32_t r = (w << 6) + uint32_t(__builtin_ctzll(x));
  return r < n ? r : n;
}


// Decide what happens to each large bin after the round (Sec. 3.1-3.3): all
// keys equal -> finished; digit constant -> same bin, next differing digit;
// otherwise its children become next-round large bins or LDS jobs.  Small
// siblings are packed greedily into jobs of at most mid_max records (Sec. 3.3
// remarks that scanning empty sub-bins one by one costs time).
template <int KW>
__global__ void __launch_bounds__(256) k_classify(Params P, uint32_t cur, uint32_t round) {
  __shared__ uint32_t s_cnt[kRadix], s_off[kRadix], s_scan[8];
  __shared__ uint32_t s_px[kRadix + 1], s_jmp[kRadix], s_st[kRadix], s_wt[4], s_wm[4];
  __shared__ uint32_t s_jbase, s_tbase, s_eqn;
  __shared__ uint64_t s_bm[4], s_sm[4];
  Ctrl* c = P.L.ctrl;
  const uint32_t nbins = min(c->large_count[cur], P.L.cap_large);
  const uint32_t nxt = cur ^ 1;
  const uint32_t tid = threadIdx.x;
  // statistics, added to the control block once per workgroup (atomics on
  // its few words from every bin of a round with thousands of bins queue up)
  uint32_t n_scattered = 0;        // (thread 0)
  unsigned long long n_moved = 0;  // (thread 0)
  if (tid == 0) s_eqn = 0;
  for (uint32_t b = blockIdx.x; b < nbins; b += gridDim.x) {
    __syncthreads();
    const Bin bin = P.L.large[cur][b];
    // an equality split leaves the key bits as they were (buckets: below,
    // equal to, above the bin's equality key)
    const bool eqb = (bin.flags & kBinEq) != 0;
    const uint32_t w = eqb ? 2u : min(bin_width(P, bin), uint32_t(bin.bits));
    const uint32_t lob = eqb ? uint32_t(bin.bits) : bin.bits - w;
    const uint32_t nb = 1u << w;
    // with pair counts (second round only) the bin's row is its top digit's
    // row of pair_hist, and any key bit below the bin's digit may differ
    const bool fused = c->fused != 0;
    uint64_t dif[KW];
#pragma unroll
    for (int i = 0; i < KW; ++i) {
      const uint32_t b0 = 64u * uint32_t(i), bits = bin.bits;
      dif[i] = fused ? (bits >= b0 + 64 ? ~0ull : (bits > b0 ? (1ull << (bits - b0)) - 1ull : 0ull))
                     : P.L.diff[cur][uint64_t(b) * 8 + i];
    }
    const int tb = top_bit<KW>(dif);
    if (tb < 0) {  // every key equal: finished where it is
      if (bin.side == 1) push_copy_jobs(P, tid == 0, bin.array, bin.start, bin.size);
      continue;
    }
    const uint32_t* hrow = fused ? P.L.pair_hist + P.L.pair_d1[b] * kRadix
                                 : P.L.hist[cur] + uint64_t(b) * kRadix;
    const uint32_t h = tid < nb ? hrow[tid] : 0;
    // one digit for the whole bin, or (a root whose top was guessed from a
    // sample) keys that differ above its bits: nothing moved; split next
    // round from the highest differing bit
    if (tb >= int(bin.bits) || __syncthreads_or(tid < nb && h == bin.size)) {
      if (tid == 0) {
        Bin nbn = bin;
        nbn.bits = uint16_t(tb + 1);
        nbn.flags = uint8_t(bin.flags & (kBinRange | kBinWidthMask));
        const uint64_t none[KW] = {};
        push_large<KW>(P, nxt, nbn, none);
      }
      continue;
    }
    s_cnt[tid] = h;
    block_exclusive_scan256(h, s_off, s_scan);
    const uint8_t cside = bin.side ^ 1;
    if (tid == 0) {
      ++n_scattered;
      n_moved += bin.size;
    }
    if (lob == 0) {  // key exhausted: every child holds equal keys
      if (cside == 1) push_copy_jobs(P, tid == 0, bin.array, bin.start, bin.size);
      continue;
    }
    // the equal part of an equality split is finished: all its keys are equal
    const bool eq_done = eqb && tid == 1;
    if (eqb && cside == 1) push_copy_jobs(P, eq_done && h > 0, bin.array, bin.start + s_off[1], h);
    if (tid < nb && h > P.mid_max && !eq_done) {
      Bin ch;
      ch.start = bin.start + s_off[tid];
      ch.size = h;
      ch.array = bin.array;
      ch.bits = uint16_t(lob);
      ch.side = cside;
      ch.flags = uint8_t((eqb || (bin.flags & kBinRange)) ? kBinRange : 0);
      // a child that one key dominates is split on that key next round, if
      // the rounds left leave room for that round and the child's key bits
      uint64_t eqk[KW] = {};
      const uint32_t need = (lob + P.digit_bits - 1) / P.digit_bits;
      if (P.eq_split && round + 2 + need <= P.round_budget) {
        const ArrayDesc a = P.L.arrays[bin.array];
        const uint8_t* base = (cside ? a.tmp : a.recs) + uint64_t(ch.start) * P.R;
        if (dominant_key<KW>(base, h, P.R, P.kmask, eqk)) {
          ch.flags |= kBinEq;
          atomicAdd(&s_eqn, 1u);
        }
      }
      // a child of 1.6 to 230 jobs' worth of records is split next round on
      // the fewest bits that leave children of at most 0.9 mid_max each
      // (about one job each, all its bits in the job's first pass), when
      // that is fewer than a digit and the rounds left still cover the key
      // bits below; not where the second round takes the top level's pair
      // counts (they are per full digit)
      const uint32_t target = P.mid_max - P.mid_max / 10u;
      if (!(ch.flags & kBinEq) && !(P.pair && round == 0) &&
          uint64_t(h) * 5u >= uint64_t(P.mid_max) * 8u && h <= 256u * target) {
        uint32_t wn = 1;
        while (wn < 8u && (h >> wn) > target) ++wn;
        const uint32_t need_n = (lob - min(wn, lob) + P.digit_bits - 1) / P.digit_bits;
        if (wn < min(P.digit_bits, lob) && round + 2 + need_n <= P.round_budget)
          ch.flags |= uint8_t(wn << kBinWidthShift);
      }
      push_large<KW>(P, nxt, ch, eqk);
    }
    // no child small enough for a sort job (the usual case at the top level)
    if (!__syncthreads_or(tid < nb && h > 0 && h <= P.mid_max && !eq_done)) continue;
    // Greedy packing of the small children into jobs, in digit order: a job
    // closes before a child that would take it past mid_max records and at
    // every child too large for a job (the finished equal part of an
    // equality split counts as one).  The scan is sequential by nature (a
    // loop over the digits took ~35 us per bin); it is computed in parallel
    // instead.  Every small child finds by binary search over the prefix
    // sums of the small children where a job starting at it would end and
    // which child would start the next job; the job starts -- the children
    // reached by those jumps from the first small child after each large
    // one -- are marked by pointer doubling (eight steps cover 256
    // children).  The jobs are the same as the loop's.
    {
      const uint32_t M = P.mid_max;
      const uint32_t lane = tid & (kWave - 1), wave = tid >> 6;
      const uint32_t cd = tid < nb ? ((eqb && tid == 1 && s_cnt[1]) ? M + 1 : s_cnt[tid]) : 0u;
      const bool big = cd > M;
      const bool small = cd != 0 && !big;
      const uint64_t bmask = __ballot(big), smask = __ballot(small);
      if (lane == 0) {
        s_bm[wave] = bmask;
        s_sm[wave] = smask;
      }
      // s_px[i]: records of the small children before child i (s_px[256]: all)
      block_exclusive_scan256(small ? cd : 0u, s_px, s_scan);
      if (tid == kRadix - 1) s_px[kRadix] = s_px[tid] + (small ? cd : 0u);
      lds_barrier();
      uint32_t jn = 0, nxt_start = kNoChild;
      bool root = false;
      if (small) {
        const uint32_t i = tid;
        const uint32_t nbig = mask_next256(s_bm, i, nb);  // first large child after i, or nb
        const int pbig = mask_prev256(s_bm, i), psmall = mask_prev256(s_sm, i);
        root = psmall < 0 || psmall < pbig;
        // first m in [i+2, nb] with s_px[m] > s_px[i] + M: child m-1 would
        // take a job starting at i past M (child i alone never does)
        const uint64_t lim = uint64_t(s_px[i]) + M;
        uint32_t lo = i + 2, hi = nb + 1;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (uint64_t(s_px[mid]) > lim) hi = mid;
          else lo = mid + 1;
        }
        const uint32_t k = lo <= nb ? lo - 1 : nb;  // next job's first child, or nb
        const uint32_t end = k < nbig ? k : nbig;
        jn = s_px[end] - s_px[i];
        nxt_start = k < nbig ? k : kNoChild;
      }
      s_jmp[tid] = nxt_start;
      s_st[tid] = root ? 1u : 0u;
      bool more = __syncthreads_or(nxt_start != kNoChild);
      while (more) {  // at most eight rounds: chains are shorter than 256
        const uint32_t j = s_jmp[tid];
        const uint32_t st = s_st[tid];
        const uint32_t jj = j != kNoChild ? s_jmp[j] : kNoChild;
        lds_barrier();
        if (st && j != kNoChild) s_st[j] = 1u;
        s_jmp[tid] = jj;
        more = __syncthreads_or(jj != kNoChild);
      }
      // (a lone record in recs is in place)
      const bool emit = small && s_st[tid] && (jn > 1 || cside != 0);
      const bool tj = jn <= P.tiny_job;
      const uint64_t tball = __ballot(emit && tj), mball = __ballot(emit && !tj);
      if (lane == 0) {
        s_wt[wave] = uint32_t(__popcll(tball));
        s_wm[wave] = uint32_t(__popcll(mball));
      }
      lds_barrier();
      if (tid == 0) {
        const uint32_t nt = s_wt[0] + s_wt[1] + s_wt[2] + s_wt[3];
        const uint32_t nm = s_wm[0] + s_wm[1] + s_wm[2] + s_wm[3];
        s_tbase = nt ? atomicAdd(&c->tiny_count, nt) : 0u;
        s_jbase = nm ? atomicAdd(&c->mid_count, nm) : 0u;
      }
      lds_barrier();
      if (emit) {
        uint32_t before = 0;
        for (uint32_t w = 0; w < wave; ++w) before += tj ? s_wt[w] : s_wm[w];
        const uint64_t mine = tj ? tball : mball;
        const uint32_t i = (tj ? s_tbase : s_jbase) + before + uint32_t(__popcll(mine & lanemask_lt()));
        if (i < P.L.cap_mid) {
          const ArrayDesc a = P.L.arrays[bin.array];
          const uint64_t st = uint64_t(bin.start) + s_off[tid];
          MidJob j;
          j.src = (cside ? a.tmp : a.recs) + st * P.R;
          j.dst = a.recs + st * P.R;
          j.size = jn;
          j.pad[0] = j.pad[1] = j.pad[2] = 0;
          (tj ? P.L.tiny : P.L.mid)[i] = j;
        } else {
          atomicOr(&c->error, kErrCapacity);
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (n_scattered) {
      atomicAdd(&c->scattered_bins, n_scattered);
      atomicAdd(&c->moved_records, n_moved);
    }
    if (s_eqn) atomicAdd(&c->eq_bins, s_eqn);
  }
}

// ------------------------------------------------------------ LDS sorter

// Highest set bit of the boundary bitmap in [lo, p], or -1.
__device__ __forceinline__ int bm_prev(const uint32_t* bm, int p, int lo) {
  int w = p >> 5;
  uint32_t m = bm[w] & (uint32_t(2u << (p & 31)) - 1u);
  while (!m) {
    if ((w << 5) <= lo) return -1;
    --w;
    m = bm[w];
  }
  const int r = (w << 5) + 31 - __clz(m);
  return r >= lo ? r : -1;
}

// Lowest set bit of the boundary bitmap in (p, hi], or -1.
__device__ __forceinline__ int bm_next(const uint32_t* bm, int p, int hi) {
  if (p >= hi) return -1;
  const int q = p + 1;
  int w = q >> 5;
  uint32_t m = bm[w] & ~((1u << (q & 31)) - 1u);
  for (;;) {
    if (m) {
      const int r = (w << 5) + __ffs(m) - 1;
      return r <= hi ? r : -1;
    }
    ++w;
    if ((w << 5) > hi) return -1;
    m = bm[w];
  }
}

// LDS state of one LDS-sort workgroup.  The job's keys stay in LDS in input
// order; every pass permutes `perm`, the slots (input positions) in sorted
// order.
struct MidLds {
  uint64_t* kp;     // [KW][T] key words of the job's records in input order: word q of
                    // record i at kp[q * T + i] (planes, so that neighbouring slots sit
                    // in neighbouring banks)
  uint64_t* pay;    // [T][RW - KW] payload words of the job's records, input order
  uint32_t T;       // records per key plane (the job capacity)
  uint64_t kmask;   // mask of the key bytes in the top key word
  uint16_t* perm;   // [T] position -> slot
  uint32_t* cnt;    // [kMidCounterWords] digit counters / offsets of a pass
  uint32_t* bm;     // boundary bitmap: bit p set where a sub-range starts
  uint32_t* bmb;    // positions left to later passes by the first pass
  uint32_t* big;    // ranges waiting for a workgroup pass (start | size << 16)
  uint32_t* list0;  // ranges waiting for a wave pass, double-buffered by round
  uint32_t* list1;
  uint32_t* nbig;
  uint32_t* nlist;  // [2]
  uint32_t* claim;  // next entry of the current list to claim
  uint32_t* scan;   // [kMidWaves], 16-byte aligned
  unsigned long long* diff;  // [kMidWaves * (KW + 1)]
};

// Order inside a job: by key, then by slot.  Sorting by this pair is the
// stable sort of the job, and every pair is distinct, so the passes below
// need not be stable: equal keys are put back in input order by slot.

template <int KW>
__device__ __forceinline__ void slot_key(const MidLds& L, uint32_t slot, uint64_t (&k)[KW]) {
#pragma unroll
  for (int q = 0; q < KW; ++q) k[q] = L.kp[uint32_t(q) * L.T + slot];
  k[KW - 1] &= L.kmask;
}

// Digit [lob, lob + w) of the pair (key, slot): of the key, or of the slot
// once the keys of the range are all equal.
template <int KW>
__device__ __forceinline__ uint32_t pair_digit(const uint64_t (&k)[KW], uint32_t slot,
                                               bool by_slot, uint32_t lob, uint32_t w) {
  return by_slot ? (slot >> lob) & ((1u << w) - 1u) : digit_of<KW>(k, lob, w);
}

// Highest differing bit of a range from the OR of (key ^ key0) and of
// (slot ^ slot0) over it: returns hb = that bit + 1 (0 if the range has one
// element) and whether it is a slot bit.
template <int KW>
__device__ __forceinline__ uint32_t pair_top(const uint64_t (&dk)[KW], uint32_t ds, bool& by_slot) {
  const int tb = top_bit<KW>(dk);
  by_slot = tb < 0;
  if (!by_slot) return uint32_t(tb) + 1;
  return ds ? 32u - uint32_t(__clz(ds)) : 0u;
}

// Route a sub-range: it starts a run in the boundary bitmap; ranges above
// tiny_max wait for a workgroup pass (> wave capacity) or a wave pass.
__device__ __forceinline__ void mid_route(const Params& P, MidLds& L, uint32_t st, uint32_t cnt,
                                          uint32_t wave_cap, uint32_t lst) {
  atomicOr(&L.bm[st >> 5], 1u << (st & 31));
  if (cnt <= P.tiny_max) return;
  const uint32_t e = st | (cnt << 16);
  if (cnt > wave_cap) {
    const uint32_t k = atomicAdd(L.nbig, 1u);
    if (k < kMidBigCap) L.big[k] = e;
    else atomicOr(&P.L.ctrl->error, kErrCapacity);
  } else {
    const uint32_t k = atomicAdd(&L.nlist[lst], 1u);
    if (k < kMidListCap) (lst ? L.list1 : L.list0)[k] = e;
    else atomicOr(&P.L.ctrl->error, kErrCapacity);
  }
}

// Sets bits [st, st + len) of an LDS bitmap.
__device__ __forceinline__ void set_bits(uint32_t* b, uint32_t st, uint32_t len) {
  for (uint32_t p = st, e = st + len; p < e;) {
    const uint32_t lo = p & 31, n = min(32u - lo, e - p);
    atomicOr(&b[p >> 5], (n == 32 ? ~0u : ((1u << n) - 1u)) << lo);
    p += n;
  }
}

// Counters of a workgroup pass: two 16-bit counts (later offsets) per word,
// digit d in half d & 1 of word d >> 1.  Jobs hold fewer than 2^16 records,
// so a half never carries into the other.
__device__ __forceinline__ uint32_t pair_count(uint32_t* cnt, uint32_t d) {
  const uint32_t sh = (d & 1u) << 4;
  return (atomicAdd(&cnt[d >> 1], 1u << sh) >> sh) & 0xFFFFu;
}
__device__ __forceinline__ uint32_t pair_get(const uint32_t* cnt, uint32_t d) {
  return (cnt[d >> 1] >> ((d & 1u) << 4)) & 0xFFFFu;
}

// One non-empty digit's sub-range [st, st + cnt) of a workgroup pass.  In a
// job's first pass only sub-ranges above tiny_max are routed (the others are
// finished by the enumeration sort that follows, which needs no boundary
// bits), and they are marked in bmb and get a boundary bit at their end too,
// so that the runs later passes cut out of them are bounded on both sides.
__device__ __forceinline__ void mid_scan_route_one(const Params& P, MidLds& L, uint32_t st,
                                                   uint32_t cnt, uint32_t wave_cap, bool first) {
  if (!first) {
    mid_route(P, L, st, cnt, wave_cap, 0);
  } else if (cnt > P.tiny_max) {
    mid_route(P, L, st, cnt, wave_cap, 0);
    set_bits(L.bmb, st, cnt);
    const uint32_t e = st + cnt;
    atomicOr(&L.bm[e >> 5], 1u << (e & 31));
  }
}

constexpr int kMidScanPer = int(kMidCounterWords / kMidBlock);  // counter words per thread

// Offsets of a first pass are below 2^13; bit 15 of a counter half marks a
// bucket that is left to the per-record enumeration sort (see k_mid).
constexpr uint32_t kOffMask = 0x1FFFu, kOffFlag = 0x8000u;
static_assert(uint32_t(kMidBlock) * mid_lane_items(1) <= kOffMask, "a job's offsets fit 13 bits");

// Exclusive scan of the nd (even, <= 2 * kMidCounterWords) packed counters
// in place over the workgroup, routing every non-empty digit's sub-range of
// the range that starts at s (with `first`, only those left to later passes;
// see mid_scan_route_one).  Thread t scans words [t * per, t * per + per).
// With KEEP every thread also keeps the counts (cw) and the starts (ow) of
// the digits of its words, packed two 16-bit values per word like the
// counters (0 counts for words past nd).  All threads call; ends with a
// barrier.
template <bool KEEP>
__device__ __forceinline__ void mid_scan_route_k(const Params& P, MidLds& L, uint32_t tid, uint32_t s,
                                                 uint32_t nd, uint32_t wave_cap, bool first,
                                                 uint32_t (&cw)[kMidScanPer], uint32_t (&ow)[kMidScanPer]) {
  constexpr int kPer = kMidScanPer;
  const uint32_t lane = tid & 63, wave = uni(tid >> 6);
  const uint32_t nw = nd >> 1;
  const uint32_t per = (nw + kMidBlock - 1) / kMidBlock;
  const uint32_t base = tid * per;
  uint32_t v[kPer], sum = 0;
  if (per == uint32_t(kPer)) {
    const uint4 q = reinterpret_cast<const uint4*>(L.cnt)[tid];
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  } else {
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = (uint32_t(k) < per && base + k < nw) ? L.cnt[base + k] : 0u;
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) sum += (v[k] & 0xFFFFu) + (v[k] >> 16);
  const uint32_t incl = wave_inclusive_scan(sum);
  if (lane == 63) L.scan[wave] = incl;
  lds_barrier();
  uint32_t run = incl - sum;
  // the totals of the waves before this one: a prefix over lanes 0..15
  {
    const uint32_t tv = lane < uint32_t(kMidWaves) ? L.scan[lane] : 0u;
    const uint32_t ti = wave_inclusive_scan(tv);
    run += uint32_t(__builtin_amdgcn_readlane(int(ti - tv), int(wave)));
  }
  uint32_t out[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t c0 = v[k] & 0xFFFFu, c1 = v[k] >> 16;
    out[k] = run | ((run + c0) << 16);
    if (KEEP) {
      cw[k] = v[k];
      ow[k] = out[k];
    }
    if (uint32_t(k) < per && base + k < nw) {
      if (c0) mid_scan_route_one(P, L, s + run, c0, wave_cap, first);
      if (c1) mid_scan_route_one(P, L, s + run + c0, c1, wave_cap, first);
      run += c0 + c1;
    }
  }
  if (per == uint32_t(kPer)) {
    reinterpret_cast<uint4*>(L.cnt)[tid] = make_uint4(out[0], out[1], out[2], out[3]);
  } else {
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (uint32_t(k) < per && base + k < nw) L.cnt[base + k] = out[k];
  }
  lds_barrier();
}
__device__ __forceinline__ void mid_scan_route(const Params& P, MidLds& L, uint32_t tid, uint32_t s,
                                               uint32_t nd, uint32_t wave_cap, bool first) {
  uint32_t cw[kMidScanPer], ow[kMidScanPer];
  mid_scan_route_k<false>(P, L, tid, s, nd, wave_cap, first, cw, ow);
}

// Workgroup pass: records with slots src[] and digits dg[] (ITEMS per thread,
// of the range [s, s + m)) are counted, the counters scanned, sub-ranges
// routed and the slots written to their places in perm.  The counters of the
// 2^w digits must be zero and every read of perm[s, s + m) done before the
// call.  Afterwards they hold each digit's offset.  All threads call; ends
// with a barrier.
template <int ITEMS>
__device__ __forceinline__ void mid_wg_place(const Params& P, MidLds& L, uint32_t tid, uint32_t s, uint32_t w,
                                             const uint32_t (&src)[ITEMS], const uint32_t (&dg)[ITEMS],
                                             const bool (&valid)[ITEMS], uint32_t wave_cap, bool first) {
  uint32_t r[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) r[j] = valid[j] ? pair_count(L.cnt, dg[j]) : 0u;
  lds_barrier();
  mid_scan_route(P, L, tid, s, 1u << w, wave_cap, first);
#pragma unroll
  for (int j = 0; j < ITEMS; ++j)
    if (valid[j]) L.perm[s + pair_get(L.cnt, dg[j]) + r[j]] = uint16_t(src[j]);
  lds_barrier();
}

// OR of per-thread spreads over the workgroup.  All threads call.
template <int KW>
__device__ __forceinline__ uint32_t mid_wg_spread(MidLds& L, uint32_t tid, uint64_t (&dk)[KW], uint32_t ds) {
  constexpr int W = kMidWaves;
  const uint32_t lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int q = 0; q < KW; ++q) {
    const uint64_t v = wave_or(dk[q]);
    if (lane == 0) L.diff[wave * (KW + 1) + q] = v;
  }
  const uint64_t vs = wave_or(uint64_t(ds));
  if (lane == 0) L.diff[wave * (KW + 1) + KW] = vs;
  lds_barrier();
  uint64_t as = 0;
#pragma unroll
  for (int q = 0; q < KW; ++q) dk[q] = 0;
  for (int w2 = 0; w2 < W; ++w2) {
#pragma unroll
    for (int q = 0; q < KW; ++q) dk[q] |= L.diff[w2 * (KW + 1) + q];
    as |= L.diff[w2 * (KW + 1) + KW];
  }
  // no barrier here: every path from one call to the next passes barriers
  // (the pass that follows each call has them), so no wave rewrites L.diff
  // while another still reads it
  return uint32_t(as);
}

// Workgroup pass over a range larger than one wave can hold: split it on the
// top digit_bits of the highest bits in which its (key, slot) pairs differ.
template <int KW, int ITEMS>
__device__ __forceinline__ void mid_wg_pass(const Params& P, MidLds& L, uint32_t tid, uint32_t s, uint32_t m,
                                            uint32_t wave_cap) {
  uint32_t src[ITEMS];
  bool valid[ITEMS];
  uint64_t key0[KW], dk[KW];
  const uint32_t slot0 = L.perm[s];
  slot_key<KW>(L, slot0, key0);
  uint32_t ds = 0;
#pragma unroll
  for (int q = 0; q < KW; ++q) dk[q] = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t i = j * kMidBlock + tid;
    valid[j] = i < m;
    src[j] = 0;
    if (valid[j]) {
      src[j] = L.perm[s + i];
      uint64_t k[KW];
      slot_key<KW>(L, src[j], k);
#pragma unroll
      for (int q = 0; q < KW; ++q) dk[q] |= k[q] ^ key0[q];
      ds |= src[j] ^ slot0;
    }
  }
  ds = mid_wg_spread<KW>(L, tid, dk, ds);
  bool by_slot;
  const uint32_t hb = pair_top<KW>(dk, ds, by_slot);
  if (KW == 1 && by_slot) {
    // every key of the range is equal: its order is the order of its slots,
    // read off a bitmap of them (the prefix count of set bits below a slot
    // is its place), in one step instead of radix passes over slot bits
    // (one-word keys only: with wider keys the registers run out, and those
    // keys rarely repeat)
    uint32_t* bits = L.cnt;        // bitmap of the range's slots
    uint32_t* pre = L.cnt + 256;   // set bits before each bitmap word
    const uint32_t nwords = (P.mid_max + 31u) / 32u;  // <= 256
    for (uint32_t q = tid; q < nwords; q += kMidBlock) bits[q] = 0;
    lds_barrier();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (valid[j]) atomicOr(&bits[src[j] >> 5], 1u << (src[j] & 31u));
    lds_barrier();
    block_exclusive_scan256(tid < nwords ? uint32_t(__popc(bits[tid])) : 0u, pre, L.scan);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (valid[j]) {
        const uint32_t wd = src[j] >> 5;
        const uint32_t at =
            s + pre[wd] + uint32_t(__popc(bits[wd] & ((1u << (src[j] & 31u)) - 1u)));
        L.perm[at] = uint16_t(src[j]);
        // the range is final: the windows' enumeration sort skips it
        atomicAnd(&L.bmb[at >> 5], ~(1u << (at & 31u)));
      }
    }
    lds_barrier();
    return;
  }
  const uint32_t w = min(P.digit_bits, hb);
  const uint32_t lob = hb - w;
  uint32_t dg[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    dg[j] = 0;
    if (valid[j]) {
      uint64_t k[KW];
      slot_key<KW>(L, src[j], k);
      dg[j] = pair_digit<KW>(k, src[j], by_slot, lob, w);
    }
  }
  for (uint32_t q = tid; q < (1u << w) / 2; q += kMidBlock) L.cnt[q] = 0;
  lds_barrier();
  mid_wg_place<ITEMS>(P, L, tid, s, w, src, dg, valid, wave_cap, false);
}

// Pass of one wave over positions [s, s + m), m <= 64 * WI: split on the top
// digit_bits of the highest bits in which the (key, slot) pairs differ;
// sub-ranges go to list `nxt`.  Uses this wave's 256 counters.
template <int KW, int WI>
__device__ __forceinline__ void mid_wave_pass(const Params& P, MidLds& L, uint32_t tid, uint32_t s, uint32_t m,
                                              uint32_t nxt, uint32_t wave_cap) {
  const uint32_t lane = tid & 63, wave = tid >> 6;
  uint32_t src[WI];
  bool valid[WI];
  uint64_t key0[KW], dk[KW];
  const uint32_t slot0 = L.perm[s];
  slot_key<KW>(L, slot0, key0);
  uint32_t ds = 0;
#pragma unroll
  for (int q = 0; q < KW; ++q) dk[q] = 0;
#pragma unroll
  for (int j = 0; j < WI; ++j) {
    const uint32_t i = j * kWave + lane;
    valid[j] = i < m;
    src[j] = 0;
    if (valid[j]) {
      src[j] = L.perm[s + i];
      uint64_t k[KW];
      slot_key<KW>(L, src[j], k);
#pragma unroll
      for (int q = 0; q < KW; ++q) dk[q] |= k[q] ^ key0[q];
      ds |= src[j] ^ slot0;
    }
  }
#pragma unroll
  for (int q = 0; q < KW; ++q) dk[q] = wave_or(dk[q]);
  ds = uint32_t(wave_or(uint64_t(ds)));
  bool by_slot;
  const uint32_t hb = pair_top<KW>(dk, ds, by_slot);
  const uint32_t w = min(P.digit_bits, hb);
  const uint32_t lob = hb - w;
  uint32_t* wc = L.cnt + wave * kRadix;
#pragma unroll
  for (int q = 0; q < kRadix / kWave; ++q) wc[lane * 4 + q] = 0;
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
  if (KW == 1 && by_slot) {
    // every key of the range is equal: its order is the order of its slots,
    // read off a bitmap of them in this wave's 256 counter words (8192 bits,
    // more than any slot): a slot's place is the number of set bits below it
    // (one-word keys only, as in the workgroup pass)
#pragma unroll
    for (int j = 0; j < WI; ++j)
      if (valid[j]) atomicOr(&wc[src[j] >> 5], 1u << (src[j] & 31u));
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) sum += uint32_t(__popc(wc[lane * 4 + q]));
    const uint32_t start = wave_inclusive_scan(sum) - sum;  // set bits before word 4 * lane
    // (all reads of this range's perm entries are done, so places are
    // written as they are found)
#pragma unroll
    for (int j = 0; j < WI; ++j) {
      const uint32_t wd = valid[j] ? src[j] >> 5 : 0u;  // every lane takes part in the shuffle
      uint32_t place = uint32_t(__shfl(int(start), int(wd >> 2)));
#pragma unroll
      for (uint32_t q = 0; q < 3; ++q)
        place += q < (wd & 3u) ? uint32_t(__popc(wc[(wd & ~3u) + q])) : 0u;
      place += uint32_t(__popc(wc[wd] & ((1u << (src[j] & 31u)) - 1u)));
      if (valid[j]) {
        const uint32_t at = s + place;
        L.perm[at] = uint16_t(src[j]);
        // the range is final: the windows' enumeration sort skips it
        atomicAnd(&L.bmb[at >> 5], ~(1u << (at & 31u)));
      }
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
    return;
  }
  uint32_t dg[WI], r[WI];
#pragma unroll
  for (int j = 0; j < WI; ++j) {
    dg[j] = 0;
    r[j] = 0;
    if (valid[j]) {
      uint64_t k[KW];
      slot_key<KW>(L, src[j], k);
      dg[j] = pair_digit<KW>(k, src[j], by_slot, lob, w);
      r[j] = atomicAdd(&wc[dg[j]], 1u);
    }
  }
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
  // exclusive scan of the 256 counters inside the wave: 4 per lane
  uint32_t c[4], sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c[q] = wc[lane * 4 + q];
    sum += c[q];
  }
  const uint32_t incl = wave_inclusive_scan(sum);
  uint32_t run = incl - sum;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    wc[lane * 4 + q] = run;
    if (c[q]) mid_route(P, L, s + run, c[q], wave_cap, nxt);
    run += c[q];
  }
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
#pragma unroll
  for (int j = 0; j < WI; ++j)
    if (valid[j]) L.perm[s + wc[dg[j]] + r[j]] = uint16_t(src[j]);
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// Descriptors of upcoming jobs are read with vector loads and made uniform
// with readfirstlane when used: scalar loads share their wait counter with
// LDS operations, so a scalar load issued in the middle of a job would be
// waited for at the next LDS barrier.
__device__ __forceinline__ uint32_t vzero() {
  uint32_t z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}
struct JobV {  // a job descriptor in vector registers
  uint32_t w[5];
};
__device__ __forceinline__ JobV vload_job(const MidJob* p) {
  const RADULS_GLOBAL uint32_t* q = gmem(reinterpret_cast<const uint32_t*>(p)) + vzero();
  JobV v;
#pragma unroll
  for (int i = 0; i < 5; ++i) v.w[i] = q[i];
  return v;
}
__device__ __forceinline__ MidJob uni_job(const JobV& v) {
  MidJob j;
  j.src = reinterpret_cast<uint8_t*>((uint64_t(uni(v.w[1])) << 32) | uni(v.w[0]));
  j.dst = reinterpret_cast<uint8_t*>((uint64_t(uni(v.w[3])) << 32) | uni(v.w[2]));
  j.size = uni(v.w[4]);
  return j;
}

// Records [0, m) of a job (source `src`) into registers, all loads in flight
// together, and the first record's key words, unmasked (every thread's
// reference for the key spread; masking them here would wait for the load);
// m = 0 loads nothing.  Items past m keep what they held (never used).
template <int RW, int KW, int ITEMS>
__device__ __forceinline__ void mid_fetch(const uint8_t* src, uint32_t m, uint32_t tid,
                                          uint64_t (&kr)[ITEMS][RW], uint64_t (&key0)[KW]) {
  const RADULS_GLOBAL uint64_t* s0 = gmem(reinterpret_cast<const uint64_t*>(src));
#pragma unroll
  for (int q = 0; q < KW; ++q) key0[q] = m ? s0[q] : 0ull;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t i = j * kMidBlock + tid;
    if (i < m) load_rec<RW>(src, i, kr[j]);
  }
}

// Digit [lob, lob + w) of a masked key; a single shift for one-word keys.
template <int KW>
__device__ __forceinline__ uint32_t key_digit(const uint64_t (&k)[KW], uint32_t lob, uint32_t w) {
  if constexpr (KW == 1) {
    return uint32_t(k[0] >> lob) & ((1u << w) - 1u);
  } else {
    return digit_of<KW>(k, lob, w);
  }
}

// Record i of a job from registers into LDS: key words to their planes,
// payload words to the record's payload row.
template <int RW, int KW>
__device__ __forceinline__ void mid_put(const MidLds& L, uint32_t i, const uint64_t (&w)[RW]) {
  constexpr int PW = RW - KW;
#pragma unroll
  for (int q = 0; q < KW; ++q) L.kp[uint32_t(q) * L.T + i] = w[q];
  if constexpr (PW > 0) {
    if constexpr (PW % 2 == 0) {
      u64x2* d = reinterpret_cast<u64x2*>(L.pay + i * uint32_t(PW));
#pragma unroll
      for (int q = 0; q < PW / 2; ++q) {
        u64x2 v;
        v.x = w[KW + 2 * q];
        v.y = w[KW + 2 * q + 1];
        d[q] = v;
      }
    } else {
#pragma unroll
      for (int q = 0; q < PW; ++q) L.pay[i * uint32_t(PW) + q] = w[KW + q];
    }
  }
}

// Record `slot` of a job from LDS (unmasked key words, then payload).
template <int RW, int KW>
__device__ __forceinline__ void mid_get(const MidLds& L, uint32_t slot, uint64_t (&w)[RW]) {
  constexpr int PW = RW - KW;
#pragma unroll
  for (int q = 0; q < KW; ++q) w[q] = L.kp[uint32_t(q) * L.T + slot];
  if constexpr (PW > 0) {
    if constexpr (PW % 2 == 0) {
      const u64x2* s = reinterpret_cast<const u64x2*>(L.pay + slot * uint32_t(PW));
#pragma unroll
      for (int q = 0; q < PW / 2; ++q) {
        const u64x2 v = s[q];
        w[KW + 2 * q] = v.x;
        w[KW + 2 * q + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < PW; ++q) w[KW + q] = L.pay[slot * uint32_t(PW) + q];
    }
  }
}

// Sorts the positions [st, st + cn) of perm, 2 <= cn <= N, in registers:
// the members' slots and then their keys are read together, each member's
// place is the number of members whose (key, slot) pair is smaller, and the
// slots are written back in that order.  Positions past the bucket reread
// its last member and count for nobody.
template <int KW, int N>
__device__ __forceinline__ void mid_sort_bucket(const MidLds& L, uint32_t st, uint32_t cn) {
  uint32_t sv[N], rk[N];
  uint64_t kv[N][KW];
#pragma unroll
  for (int v = 0; v < N; ++v) sv[v] = L.perm[st + min(uint32_t(v), cn - 1u)];
#pragma unroll
  for (int v = 0; v < N; ++v) {
    slot_key<KW>(L, sv[v], kv[v]);
    rk[v] = 0;
  }
#pragma unroll
  for (int x = 0; x < N; ++x) {
#pragma unroll
    for (int y = x + 1; y < N; ++y) {
      const bool yx = key_lt<KW>(kv[y], kv[x]) || (sv[y] < sv[x] && key_eq<KW>(kv[y], kv[x]));
      const bool in = uint32_t(y) < cn;
      rk[x] += (in && yx) ? 1u : 0u;
      rk[y] += (in && !yx) ? 1u : 0u;
    }
  }
#pragma unroll
  for (int v = 0; v < N; ++v)
    if (uint32_t(v) < cn) L.perm[st + rk[v]] = uint16_t(sv[v]);
}

// Sorts the positions [st, st + cn) of perm, 2 <= cn <= 64, with one wave:
// lane v holds member v's slot and key, and counts the members whose (key,
// slot) pair is smaller as they are broadcast one by one; then it writes its
// slot to its place (one wave's LDS accesses stay in order, so every read of
// the bucket precedes these writes).
template <int KW>
__device__ __forceinline__ void mid_wave_sort_bucket(const MidLds& L, uint32_t st, uint32_t cn,
                                                     uint32_t lane) {
  const uint32_t sv = L.perm[st + min(lane, cn - 1u)];
  uint64_t kv[KW];
  slot_key<KW>(L, sv, kv);
  uint32_t rk = 0;
  for (uint32_t u = 0; u < cn; ++u) {
    uint64_t ku[KW];
#pragma unroll
    for (int q = 0; q < KW; ++q) {
      const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(kv[q])), int(u)));
      const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(kv[q] >> 32)), int(u)));
      ku[q] = uint64_t(lo) | (uint64_t(hi) << 32);
    }
    const uint32_t su = uint32_t(__builtin_amdgcn_readlane(int(sv), int(u)));
    rk += (key_lt<KW>(ku, kv) || (su < sv && key_eq<KW>(ku, kv))) ? 1u : 0u;
  }
  if (lane < cn) L.perm[st + rk] = uint16_t(sv);
}

// ------------------------------------------------------------ resident server

// A workgroup's claimed run of tickets [first, first + count); idx of them
// taken so far.
struct ServeCursor {
  uint64_t first, count, idx;
  uint64_t start;  // the 100 MHz clock when the workgroup started
};

// Claim a run of queued requests of a resident server (all threads call; the
// result is uniform).  Wave 0 does the waiting: it claims the oldest queued
// requests (a compare-and-swap on the device queue's head; an eighth of the
// queue, 1..kServeChunk of them, so that a long queue is taken in runs and a
// short one a request at a time); when none is queued it takes the dispatch
// lock and moves newly published requests from the host ring into the device
// queue -- each lane reads one slot with an acquire at system scope, the
// published run from the oldest on is copied, and the queue's tail advances
// past it with a release.  The claimant also acquires at system scope, so
// that the requests' inputs (written before they were submitted) are visible
// to it.  It gives up when the host sets the stop word or after P.serve_idle
// ticks of the 100 MHz clock without a request; every wait of the server is
// bounded that way.  With a lease (P.serve_lease ticks, non-zero) it also
// gives up before claiming once the workgroup has run that long, queued
// requests or not: the host relaunches the kernel for them, and work queued
// behind the kernel on a shared hardware queue runs in between.  Returns
// false to exit.
__device__ __forceinline__ bool serve_claim(const Params& P, ServeCursor& cur) {
  __shared__ uint64_t s_first, s_count;
  __shared__ uint32_t s_got;
  if (threadIdx.x < kWave) {
    const uint32_t lane = threadIdx.x;
    ServeState* S = P.serve;
    const uint32_t width = min(uint32_t(kWave), P.serve_slots);  // distinct ring slots per read
    const uint64_t t0 = wall_clock64();
    uint32_t got = 0, spins = 0, lost = 0;
    for (;;) {
      uint32_t won = 0, queued = 0, expired = 0;
      if (lane == 0 && P.serve_lease && wall_clock64() - cur.start > P.serve_lease) {
        __hip_atomic_store(&P.ring->reason, 3u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        expired = 1;
      }
      if (__builtin_amdgcn_readfirstlane(expired)) break;
      if (lane == 0) {
        const uint64_t h = __hip_atomic_load(&S->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t = __hip_atomic_load(&S->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        queued = h < t ? 1u : 0u;
        if (queued) {
          const uint64_t take = min(max((t - h) / 8u, uint64_t(1)), uint64_t(kServeChunk));
          uint64_t expect = h;
          won = __hip_atomic_compare_exchange_strong(&S->head, &expect, h + take, __ATOMIC_ACQ_REL,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    ? 1u
                    : 0u;
          if (won) {
            // (an acquire at system scope here too: the wave that read the
            // ring may run on another XCD, whose caches are not this one's)
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
            s_first = h;
            s_count = take;
          }
        }
      }
      if (__builtin_amdgcn_readfirstlane(won)) {
        got = 1;
        break;
      }
      if (__builtin_amdgcn_readfirstlane(queued)) {
        // another workgroup took them: retry after a pause that grows with
        // the claims lost in a row (staggered by workgroup), so that many
        // workgroups do not keep hammering the head
        lost = min(lost + 1u, 6u);
        for (uint32_t k = (blockIdx.x & 3u) + (1u << lost); k > 0; --k) __builtin_amdgcn_s_sleep(1);
        continue;
      }
      lost = 0;
      // nothing queued: move published requests from the ring, if the lock is free
      uint32_t locked = 0;
      if (lane == 0 &&
          __hip_atomic_load(&S->lock, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
        uint32_t expect = 0u;
        locked = __hip_atomic_compare_exchange_strong(&S->lock, &expect, 1u, __ATOMIC_ACQUIRE,
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     ? 1u
                     : 0u;
      }
      if (__builtin_amdgcn_readfirstlane(locked)) {
        __atomic_thread_fence(__ATOMIC_ACQUIRE);  // (every lane, after lane 0's acquire)
        const uint64_t base = __hip_atomic_load(&S->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t tk = base + lane;
        bool pub = false;
        uint64_t recs = 0, n = 0;
        if (lane < width) {
          ServeSlot* sl = &P.ring->slot[tk % P.serve_slots];
          pub = __hip_atomic_load(&sl->seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) == tk + 1;
          if (pub) {
            recs = __hip_atomic_load(&sl->recs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            n = __hip_atomic_load(&sl->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          }
        }
        // the published run from the oldest slot on
        const uint64_t missing = __ballot(!pub);
        const uint32_t cnt = missing ? uint32_t(__builtin_ctzll(missing)) : uint32_t(kWave);
        if (lane < cnt) {
          ServeJob q;
          q.recs = recs;
          q.n = n;
          P.serve_queue[tk % P.serve_slots] = q;
        }
        __threadfence();  // the queue entries before the tail
        if (lane == 0) {
          if (cnt) __hip_atomic_store(&S->tail, base + cnt, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&S->lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (cnt) {
          spins = 0;
          continue;  // claim some of them
        }
      }
      uint32_t quit = 0;
      if (lane == 0) {
        if (__hip_atomic_load(&P.ring->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
          __hip_atomic_store(&P.ring->reason, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          quit = 1;
        } else if (wall_clock64() - t0 > P.serve_idle) {
          __hip_atomic_store(&P.ring->reason, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          quit = 1;
        }
      }
      if (__builtin_amdgcn_readfirstlane(quit)) break;
      // short naps while requests are coming, longer ones when idle
      if (++spins < 256) __builtin_amdgcn_s_sleep(2);
      else __builtin_amdgcn_s_sleep(60);
    }
    if (lane == 0) s_got = got;
  }
  __syncthreads();
  if (!s_got) return false;
  cur.first = s_first;
  cur.count = s_count;
  cur.idx = 0;
  return true;
}

// The next request of a resident server: the next of the workgroup's
// claimed run, or the first of a new run (all threads call).
__device__ __forceinline__ bool serve_next(const Params& P, ServeCursor& cur, MidJob& job,
                                           uint64_t& ticket) {
  __shared__ uint64_t s_recs, s_n;
  if (cur.idx >= cur.count && !serve_claim(P, cur)) return false;
  ticket = cur.first + cur.idx;
  ++cur.idx;
  if (threadIdx.x == 0) {
    const ServeJob* q = P.serve_queue + ticket % P.serve_slots;
    s_recs = __hip_atomic_load(&q->recs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_n = __hip_atomic_load(&q->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  job.src = job.dst = reinterpret_cast<uint8_t*>(s_recs);
  job.size = uint32_t(s_n);
  job.pad[0] = job.pad[1] = job.pad[2] = 0;
  return true;
}

// A server request's stores are done (all threads call): thread 0 writes the
// request's status (the workgroup's error bits, cleared for the next one).
// At the end of the workgroup's run every thread waits until its stores have
// reached the device cache, and after a barrier wave 0 publishes the run's
// completion words with release stores at system scope, whose write-back
// of the cache then covers every thread's records: one write-back per run
// instead of one per wave.
__device__ __forceinline__ void serve_complete(const Params& P, Ctrl* c, uint64_t ticket,
                                               const ServeCursor& cur) {
  if (threadIdx.x == 0) {
    const uint32_t err = atomicExch(&c->error, 0u);
    __hip_atomic_store(&P.ring->slot[ticket % P.serve_slots].status, err, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (cur.idx < cur.count) return;
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
  __syncthreads();
  if (threadIdx.x < cur.count) {
    const uint64_t t = cur.first + threadIdx.x;
    __hip_atomic_store(&P.ring->slot[t % P.serve_slots].done, t + 1, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Sorts jobs of at most mid_max records entirely in LDS (the small-bin case of
// Sec. 3.2, with LDS in the role of the cache).  A job's records are read from
// HBM once and kept in LDS in input order; every pass permutes a 16-bit slot
// array instead of moving records.  The first pass splits the job on up to
// kMidFirstBits of the highest bits in which its keys differ, with the digits
// taken from keys still in registers.  Its buckets of at most tiny_max records
// are finished at once by enumeration sort (Sec. 2.2, 3.3): each record's
// place is the number of (key, slot) pairs of its bucket below its own, every
// thread stepping through the buckets of all its records together so that
// their LDS reads overlap.  Sub-ranges still larger than tiny_max get further
// passes, by the whole workgroup when they exceed one wave's capacity, else by
// single waves in parallel, round by round, and their tiny ranges are again
// finished by enumeration sort.  The job is written out in order, each thread
// gathering its records from LDS through the permutation, in coalesced stores.
//
// Jobs are pipelined so that no wave waits for HBM in the middle of a job:
// workgroups claim jobs from a shared counter (after a first one of their
// own), so that faster CUs take more of them.  While job i is sorted, the
// records of job i+1 travel into registers (they are loaded before job i's
// stores are issued, so waiting for them never waits for those stores), the
// descriptor of job i+2 is on its way and the claim for job i+3 is made.
//
// SERVE = 1 is the resident server: no job list and no pipelining; each
// workgroup claims one request at a time from the submission ring (waiting
// for it, bounded), sorts it in place and publishes its completion.
template <int RW, int KW, int SERVE = 0>
__global__ void __launch_bounds__(kMidBlock) k_mid(Params P) {
  constexpr int W = kMidWaves;
  constexpr int WI = mid_wave_items(RW);
  constexpr int ITEMS = mid_items(RW, KW);
  // keys of the job's records stay in registers through the first pass
  // (digits and the enumeration sort's own key without LDS reads) when they
  // are short; longer ones are read back from their LDS planes
  constexpr bool kKeep = KW <= 2;
  constexpr int KK = kKeep ? KW : 1;
  // first-pass buckets of 2..kOwnMax records are sorted in registers by one
  // thread each (pairs only for long keys: the registers run out), larger
  // ones up to 64 records by one wave each
  constexpr uint32_t kOwnMax = kKeep ? 4u : 2u;
  constexpr uint32_t kEsCap = 1024;    // entries of the workgroup's list of such buckets
  constexpr uint32_t kEsWaveCap = 128; // entries of its list of buckets sorted by a wave
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint32_t s_big[kMidBigCap];
  __shared__ uint32_t s_list[2][kMidListCap];
  __shared__ uint32_t s_nbig, s_nlist[2], s_claim, s_next, s_next2;
  __shared__ __align__(16) uint32_t s_scan[W];
  __shared__ unsigned long long s_diff[W * (KW + 1)];
  __shared__ uint32_t s_hb[2];  // highest differing key bit + 1 of a job, by job parity
  __shared__ uint32_t s_flag[2];  // a job's first pass left buckets for the fallback enumeration sort
  __shared__ uint32_t s_esn[2];  // a job's listed buckets: thread list | wave list << 16
  __shared__ uint32_t s_es[kEsCap], s_wbk[kEsWaveCap];

  const uint32_t T = P.mid_max;  // largest job (<= the LDS layout's capacity)
  // the LDS layout is laid out for the largest job of this record width, so
  // that its offsets are compile-time constants
  constexpr uint32_t TC = mid_cap(RW, KW);
  MidLds L;
  L.kp = reinterpret_cast<uint64_t*>(smem);
  L.pay = L.kp + TC * uint32_t(KW);
  L.T = TC;
  L.kmask = P.kmask;
  L.perm = reinterpret_cast<uint16_t*>(L.kp + TC * uint32_t(RW));
  L.cnt = reinterpret_cast<uint32_t*>(L.perm + align_up(TC, 2));
  L.bm = L.cnt + kMidCounterWords;
  L.bmb = L.bm + (TC >> 5) + 2;
  L.big = s_big;
  L.list0 = s_list[0];
  L.list1 = s_list[1];
  L.nbig = &s_nbig;
  L.nlist = s_nlist;
  L.claim = &s_claim;
  L.scan = s_scan;
  L.diff = s_diff;

  Ctrl* c = SERVE ? P.serve_ctrl + blockIdx.x : P.L.ctrl;
  const uint32_t njobs = SERVE ? 0u : min(c->mid_count, P.L.cap_mid);
  const uint32_t tiny = P.tiny_max;
  const uint32_t wave_cap = kWave * WI;
  const uint32_t G = gridDim.x;
  MidJob job{};  // job i
  uint64_t ticket = 0;  // (server) the request being sorted
  ServeCursor scur{0, 0, 0, SERVE ? wall_clock64() : 0ull};
  if constexpr (SERVE) {
    if (!serve_next(P, scur, job, ticket)) return;
  } else {
    if (blockIdx.x >= njobs) return;
    job = P.L.mid[blockIdx.x];
  }
  uint64_t kr[ITEMS][RW] = {}, key0[KW];
  mid_fetch<RW, KW, ITEMS>(job.src, job.size <= T ? job.size : 0u, threadIdx.x, kr, key0);
  if (threadIdx.x == 0) {
    s_next = SERVE ? 0u : G + atomicAdd(&c->mid_claim, 1u);
    s_next2 = SERVE ? 0u : G + atomicAdd(&c->mid_claim, 1u);
    s_hb[0] = 0;
    s_hb[1] = 0;
    s_flag[0] = 0;
    s_flag[1] = 0;
    s_esn[0] = 0;
    s_esn[1] = 0;
  }
  __syncthreads();
  bool have1 = s_next < njobs;  // job i+1 exists
  uint32_t idx2 = s_next2;      // index of job i+2
  MidJob nxt{};                 // descriptor of job i+1
  if (have1) nxt = P.L.mid[s_next];
  // nothing of the set-up stays in flight into the loop, so that no wait is
  // placed at its head
  __builtin_amdgcn_s_waitcnt(0);

  for (uint32_t par = 0;; par ^= 1u) {
    // the thread index is made opaque per job so that the per-item
    // addresses derived from it are recomputed instead of held in registers
    // across the whole loop
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t lane = tid & 63, wave = tid >> 6;
    if (job.size > T && tid == 0) atomicOr(&c->error, kErrMidSize);
    const uint32_t m = job.size <= T ? job.size : 0u;

    // the records (already in registers) into LDS; their keys kept; the
    // keys' spread against the first key
    uint64_t dk[KW], kk[ITEMS][KK];
#pragma unroll
    for (int q = 0; q < KW; ++q) dk[q] = 0;
    key0[KW - 1] &= P.kmask;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t i = j * kMidBlock + tid;
      uint64_t k[KW];
      key_of<KW>(kr[j], P.kmask, k);
#pragma unroll
      for (int q = 0; q < KK; ++q) kk[j][q] = k[q];
      if (i < m) {
#pragma unroll
        for (int q = 0; q < KW; ++q) dk[q] |= k[q] ^ key0[q];
        mid_put<RW, KW>(L, i, kr[j]);
      }
    }
    // into the freed registers the records of job i+1; then the descriptor of
    // job i+2 and the claim of job i+3, which are read in the middle of this
    // job, before its stores are issued
    if (have1) mid_fetch<RW, KW, ITEMS>(nxt.src, nxt.size <= T ? nxt.size : 0u, tid, kr, key0);
    const bool have2 = have1 && idx2 < njobs;
    JobV nextv{};
    uint32_t claimv = 0;
    if (have2) {
      nextv = vload_job(P.L.mid + idx2);
      // (the address is made opaque so that the atomic stays a single lane's
      // and its result is not waited for here)
      if (tid == 0) claimv = atomicAdd(&c->mid_claim + vzero(), 1u);
    }
    for (uint32_t q = tid; q < (m >> 5) + 2; q += kMidBlock) {
      L.bm[q] = 0;
      L.bmb[q] = 0;
    }
    static_assert(kMidCounterWords == 4 * kMidBlock, "one 16-byte clear per thread");
    reinterpret_cast<uint4*>(L.cnt)[tid] = make_uint4(0, 0, 0, 0);
    if (tid == 0) {
      s_nbig = 0;
      s_nlist[0] = 0;
      s_nlist[1] = 0;
    }
    // the job's highest differing key bit: per wave, then the workgroup's
    // maximum by one LDS atomic per wave (slots start in input order, so only
    // the keys can differ)
    {
      uint64_t o[KW];
#pragma unroll
      for (int q = 0; q < KW; ++q) o[q] = wave_or(dk[q]);
      const int tb = top_bit<KW>(o);
      if (lane == 0 && tb >= 0) atomicMax(&s_hb[par], uint32_t(tb + 1));
    }
    lds_barrier();
    const uint32_t hb = uni(s_hb[par]);
    // (the other parity's words were last read before this job's barriers)
    // (a zero made at the point of use: a zero kept in registers across the
    // loop gets spilled, and its reload would wait for the prefetch loads)
    if (tid == 0) {
      const uint32_t z = vzero();
      s_hb[par ^ 1u] = z;
      s_flag[par ^ 1u] = z;
      s_esn[par ^ 1u] = z;
    }
    bool windows = false;  // tiny ranges left for the window enumeration sort
    bool later = false;    // ranges left for later passes
    if (m > min(tiny, P.es_job) && hb > 0) {
      // first pass over the whole job, on digits from the kept keys: about
      // two buckets per record (2^w >= 2m), so that most buckets hold one
      // record or none
      const uint32_t lg = 32u - uint32_t(__clz(m));
      const uint32_t w = min(min(hb, uint32_t(kMidFirstBits)), lg + 1u);
      const uint32_t lob = hb - w;
      const uint32_t nd = 1u << w;
      uint32_t dg[ITEMS], r[ITEMS];
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = j * kMidBlock + tid;
        uint64_t k[KW];
        if constexpr (kKeep) {
#pragma unroll
          for (int q = 0; q < KW; ++q) k[q] = kk[j][q];
        } else {
          slot_key<KW>(L, i < m ? i : 0u, k);
        }
        dg[j] = i < m ? key_digit<KW>(k, lob, w) : 0u;
        r[j] = i < m ? pair_count(L.cnt, dg[j]) : 0u;
      }
      lds_barrier();
      uint32_t cw[kMidScanPer], ow[kMidScanPer];
      mid_scan_route_k<true>(P, L, tid, 0, nd, wave_cap, true, cw, ow);
      // Buckets of 2..tiny_max records are finished by enumeration sort once
      // every record is placed.  The thread that scanned a bucket's counters
      // lists it: buckets of 2..kOwnMax records in the thread list, larger
      // ones up to 64 in the wave list (a wave reserves room in both for all
      // of its lanes' entries with one atomic on a packed pair of counts).
      // After the places are written a thread sorts one bucket of the thread
      // list in registers and a wave one of the wave list, so that the work
      // is spread evenly over lanes whatever the buckets' sizes.  A bucket
      // that finds its list full is marked in bit 15 of its (13-bit) offset
      // and left, like buckets of more than 64 records, to the per-record
      // fallback.
      const uint32_t lim1 = min(kOwnMax, tiny), lim2 = min(uint32_t(kWave), tiny);
      uint32_t own1 = 0, own2 = 0;
      bool fb = false;
#pragma unroll
      for (int k = 0; k < kMidScanPer; ++k) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t cn = (cw[k] >> (16 * h)) & 0xFFFFu;
          own1 |= (cn >= 2 && cn <= lim1) ? (1u << (2 * k + h)) : 0u;
          own2 |= (cn > lim1 && cn >= 2 && cn <= lim2) ? (1u << (2 * k + h)) : 0u;
          fb = fb || (cn > lim2 && cn <= tiny);
        }
      }
      const uint32_t no = uint32_t(__popc(own1)) | (uint32_t(__popc(own2)) << 16);
      const uint32_t incl = wave_inclusive_scan(no);
      uint32_t wb = 0;
      if (lane == 63 && incl) wb = atomicAdd(&s_esn[par], incl);
      uint32_t idx = uint32_t(__builtin_amdgcn_readlane(int(wb), 63)) + incl - no;
      // every record to its place (its bucket's offset from the scanned
      // counters, masked: owners may be marking buckets meanwhile)
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = j * kMidBlock + tid;
        const uint32_t d = dg[j];
        const uint32_t lo = (L.cnt[d >> 1] >> ((d & 1u) << 4)) & kOffMask;
        if (i < m) L.perm[lo + r[j]] = uint16_t(i);
      }
      // this thread's list entries (a select over its counter words per entry)
      uint32_t both = own1 | own2;
      while (both) {
        const uint32_t bit = uint32_t(__ffs(both)) - 1u;
        both &= both - 1u;
        uint32_t wc = cw[0], wo = ow[0];
#pragma unroll
        for (int k = 1; k < kMidScanPer; ++k) {
          wc = (bit >> 1) == uint32_t(k) ? cw[k] : wc;
          wo = (bit >> 1) == uint32_t(k) ? ow[k] : wo;
        }
        const uint32_t sh = (bit & 1u) << 4;
        const uint32_t ent = ((wo >> sh) & 0xFFFFu) | (((wc >> sh) & 0xFFFFu) << 16);
        const bool first = (own1 >> bit) & 1u;
        const uint32_t at = first ? (idx & 0xFFFFu) : (idx >> 16);
        if (first && at < kEsCap) {
          s_es[at] = ent;
        } else if (!first && at < kEsWaveCap) {
          s_wbk[at] = ent;
        } else {
          // (this thread alone writes its counter words in this phase; the
          // others only read their offsets, masked)
          const uint32_t wi = tid * ((nd / 2 + kMidBlock - 1) / kMidBlock) + (bit >> 1);
          L.cnt[wi] |= kOffFlag << sh;
          fb = true;
        }
        idx += first ? 1u : 0x10000u;
      }
      if (fb) s_flag[par] = 1u;
      lds_barrier();
      const bool fallback = s_flag[par] != 0;
      // (the lists of ranges for later passes were filled by the scan)
      later = (s_nbig | s_nlist[0]) != 0;
      // the listed buckets; nobody else touches their positions, so no
      // barrier is needed
      const uint32_t esn = s_esn[par];
      for (uint32_t e = tid; e < min(esn & 0xFFFFu, kEsCap); e += kMidBlock) {
        const uint32_t ent = s_es[e];
        mid_sort_bucket<KW, kOwnMax>(L, ent & 0xFFFFu, ent >> 16);
      }
      for (uint32_t e = wave; e < min(esn >> 16, kEsWaveCap); e += W) {
        const uint32_t ent = uni(s_wbk[e]);
        mid_wave_sort_bucket<KW>(L, ent & 0xFFFFu, ent >> 16, lane);
      }
      if (fallback) {
        // buckets of 65..tiny_max records and marked ones: each member
        // counts the (key, slot) pairs of its bucket below its own
        uint32_t fin[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          const uint32_t i = j * kMidBlock + tid;
          const uint32_t d = dg[j];
          const uint32_t wd = L.cnt[d >> 1];
          const uint32_t wn = L.cnt[min((d >> 1) + 1, (nd >> 1) - 1)];
          const uint32_t h0 = (d & 1u) ? wd >> 16 : wd & 0xFFFFu;
          const uint32_t lo = h0 & kOffMask;
          const uint32_t hi = (d & 1u) ? (d + 1 < nd ? wn & kOffMask : m) : (wd >> 16) & kOffMask;
          const uint32_t cnt = hi - lo;
          fin[j] = ~0u;
          if (!(i < m && ((cnt > uint32_t(kWave) && cnt <= tiny) || (h0 & kOffFlag)))) continue;
          uint64_t kp[KW];
          slot_key<KW>(L, i, kp);
          uint32_t rnk = 0;
          // with multi-word keys four members per step, their slots and then
          // their keys read together (positions past the bucket reread its
          // last member and are not counted)
          constexpr uint32_t kStep = KW >= 2 && KW <= 4 ? 4u : 1u;
          for (uint32_t q = lo; q < hi; q += kStep) {
            uint32_t sq[kStep];
#pragma unroll
            for (uint32_t u = 0; u < kStep; ++u) sq[u] = L.perm[kStep > 1 ? min(q + u, hi - 1) : q];
#pragma unroll
            for (uint32_t u = 0; u < kStep; ++u) {
              uint64_t kq[KW];
              slot_key<KW>(L, sq[u], kq);
              rnk += (q + u < hi && (key_lt<KW>(kq, kp) || (sq[u] < i && key_eq<KW>(kq, kp)))) ? 1u : 0u;
            }
          }
          fin[j] = lo + rnk;
        }
        lds_barrier();  // every read of perm is done
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
          if (fin[j] != ~0u) L.perm[fin[j]] = uint16_t(j * kMidBlock + tid);
        lds_barrier();
      }
      // (the later passes touch only ranges above tiny_max, which these
      // buckets are not part of, and the write-out waits at a barrier)
    } else {
      // one key (already in slot order), or a job small enough for the
      // enumeration sort below
      for (uint32_t i = tid; i < m; i += kMidBlock) L.perm[i] = uint16_t(i);
      if (tid == 0) L.bm[0] = 1u;
      if (hb > 0) {
        windows = true;
        for (uint32_t q = tid; q < (m + 31) >> 5; q += kMidBlock)
          L.bmb[q] = q < (m >> 5) ? ~0u : ((1u << (m & 31)) - 1u);
      }
      lds_barrier();
    }
    // ranges too large for one wave
    bool passes = false;  // (uniform: taken from LDS counters after barriers)
    for (; later;) {
      const uint32_t nbig = min(s_nbig, kMidBigCap);
      if (nbig == 0) break;
      passes = true;
      const uint32_t e = s_big[nbig - 1];
      lds_barrier();
      if (tid == 0) s_nbig = nbig - 1;
      lds_barrier();
      mid_wg_pass<KW, ITEMS>(P, L, tid, e & 0xFFFFu, e >> 16, wave_cap);
    }
    // medium ranges: one wave each, round by round
    for (uint32_t cur = 0; later; cur ^= 1) {
      const uint32_t nl = min(s_nlist[cur], kMidListCap);
      if (nl == 0) break;
      passes = true;
      if (tid == 0) {
        s_claim = 0;
        s_nlist[cur ^ 1] = 0;
      }
      lds_barrier();
      for (;;) {
        uint32_t k = 0;
        if (lane == 0) k = atomicAdd(&s_claim, 1u);
        k = __shfl(k, 0);
        if (k >= nl) break;
        const uint32_t e = s_list[cur][k];
        mid_wave_pass<KW, WI>(P, L, tid, e & 0xFFFFu, e >> 16, cur ^ 1, wave_cap);
      }
      lds_barrier();
      if (tid == 0) s_nlist[cur] = 0;
    }
    if (passes) lds_barrier();  // without later passes perm is complete already
    windows = windows || passes;

    // ---- tiny ranges the later passes produced (inside positions marked in
    // bmb): enumeration sort; everything else is in place.  A range belongs
    // to the wave that owns the 64-position window its first position falls
    // in, so each wave reads, ranks and rewrites only positions no other wave
    // touches.  Without later passes the first pass finished every range.
    const uint32_t nwin = windows ? (m + kWave - 1) / kWave : 0u;
    for (uint32_t k = wave; k < nwin; k += W) {
      const uint32_t w0 = k * kWave;
      if ((L.bmb[w0 >> 5] | L.bmb[(w0 >> 5) + 1]) == 0) continue;
      uint32_t dst[kMidEsItems], slot[kMidEsItems];
      bool act[kMidEsItems];
#pragma unroll
      for (int h = 0; h < kMidEsItems; ++h) {
        const uint32_t p = w0 + h * kWave + lane;
        act[h] = false;
        dst[h] = p;
        slot[h] = 0;
        if (p >= m || uint32_t(h) * kWave > tiny + kWave) continue;
        if (!((L.bmb[p >> 5] >> (p & 31)) & 1u)) continue;
        // a run start here: a range of another window, or a single record
        const bool st = (L.bm[p >> 5] >> (p & 31)) & 1u;
        if (st && (h > 0 || p + 1 == m || ((L.bm[(p + 1) >> 5] >> ((p + 1) & 31)) & 1u))) continue;
        const int lo = int(p) > int(tiny) ? int(p - tiny) : 0;
        const int s = bm_prev(L.bm, int(p), lo);
        if (s < int(w0) || s >= int(w0 + kWave)) continue;  // not a range of this window
        const int hi = min(s + int(tiny), int(m) - 1);
        int e = bm_next(L.bm, int(p), hi);
        if (e < 0 && s + int(tiny) >= int(m)) e = int(m);
        if (e < 0 || e - s < 2) continue;
        slot[h] = L.perm[p];
        uint64_t kp[KW];
        slot_key<KW>(L, slot[h], kp);
        uint32_t r = 0;
        // four members per step with multi-word keys: their slots and then
        // their keys read together (positions past the range reread its last
        // member and are not counted)
        constexpr int kStep = KW >= 2 && KW <= 4 ? 4 : 1;
        for (int q = s; q < e; q += kStep) {
          uint32_t sq[kStep];
#pragma unroll
          for (int u = 0; u < kStep; ++u) sq[u] = L.perm[kStep > 1 ? min(q + u, e - 1) : q];
#pragma unroll
          for (int u = 0; u < kStep; ++u) {
            uint64_t kq[KW];
            slot_key<KW>(L, sq[u], kq);
            r += (q + u < e && (key_lt<KW>(kq, kp) || (sq[u] < slot[h] && key_eq<KW>(kq, kp)))) ? 1u : 0u;
          }
        }
        dst[h] = uint32_t(s) + r;
        act[h] = true;
      }
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_wave_barrier();
      asm volatile("" ::: "memory");
#pragma unroll
      for (int h = 0; h < kMidEsItems; ++h)
        if (act[h]) L.perm[dst[h]] = uint16_t(slot[h]);
    }
    // every load issued at the start of this job has landed (all of them,
    // on every path, so that nothing loaded is still counted as in flight
    // when the next job starts and this job's stores are out); then the
    // descriptor of job i+2 and the index of job i+3, published by the same
    // barrier that completes perm
    __builtin_amdgcn_s_waitcnt(0x3F70);  // gfx9 encoding: vmcnt(0), lgkmcnt/expcnt not waited
    MidJob nxt2{};
    if (have2) nxt2 = uni_job(nextv);
    if (tid == 0) s_next = have2 ? G + claimv : njobs;
    lds_barrier();
    const uint32_t idx3 = s_next;
    // the job in order: each thread gathers records from LDS through the
    // permutation and stores them coalesced (the slots of all its positions
    // read first, with no branch, so that those reads overlap)
    {
      uint32_t sl[ITEMS];
      bool bad = false;
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t p = j * kMidBlock + tid;
        sl[j] = L.perm[p < m ? p : 0u];
      }
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t p = j * kMidBlock + tid;
        // (never out of range while the passes above keep perm a permutation)
        bad = bad || (p < m && sl[j] >= m);
        sl[j] = sl[j] < m ? sl[j] : 0u;
      }
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t p = j * kMidBlock + tid;
        uint64_t r[RW];
        mid_get<RW, KW>(L, sl[j], r);
        if (p < m) store_rec<RW>(reinterpret_cast<uint8_t*>(job.dst), p, r, false);
      }
      if (bad) atomicOr(&c->error, kErrBounds);
    }
    lds_barrier();  // the records are rewritten by the next job
    if constexpr (SERVE) {
      serve_complete(P, c, ticket, scur);
      if (!serve_next(P, scur, job, ticket)) break;
      mid_fetch<RW, KW, ITEMS>(job.src, job.size <= T ? job.size : 0u, threadIdx.x, kr, key0);
      __builtin_amdgcn_s_waitcnt(0);
      continue;
    }
    if (!have1) break;
    job = nxt;
    nxt = nxt2;
    have1 = have2;
    idx2 = idx3;
  }
}

// ------------------------------------------------------------ copies

// Jobs of at most one wave of records (tiny bins, Sec. 3.3, and tiny arrays
// of a batch) are sorted in registers with Batcher's bitonic network over
// the jobs' (key, slot) pairs -- branch-free, the kind of network Sec. 3.3
// uses for tiny bins -- padded with pairs above any real one; then lane r of
// a job fetches the record of the r-th pair from the lane that loaded it and
// stores it at position r.  The pairs are distinct, so the order is the
// stable one.
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  const uint32_t lo = uint32_t(__shfl(int(uint32_t(v)), src));
  const uint32_t hi = uint32_t(__shfl(int(uint32_t(v >> 32)), src));
  return uint64_t(lo) | (uint64_t(hi) << 32);
}

// One pass of a wave over 64 / S consecutive tiny jobs (first, first + 1,
// ...; ids from n on are empty), S lanes per job.  Lanes of a job form one
// segment; the network's compare-exchanges stay inside it (partner lane ^ j
// with j < S) and every segment ends ascending.
template <int RW, int KW, int S>
__device__ __forceinline__ void tiny_pass(const Params& P, uint32_t first, uint32_t n,
                                          uint32_t lane) {
  const uint32_t seg = lane / uint32_t(S), idx = lane % uint32_t(S);
  const uint32_t jid = first + seg;
  MidJob job{};
  if (jid < n) job = P.L.tiny[jid];
  const uint32_t m = jid < n ? min(job.size, uint32_t(S)) : 0u;
  uint64_t rec[RW];
#pragma unroll
  for (int q = 0; q < RW; ++q) rec[q] = 0;
  if (idx < m) load_rec<RW>(job.src, idx, rec);
  uint64_t key[KW];
#pragma unroll
  for (int q = 0; q < KW; ++q) key[q] = idx < m ? rec[q] : ~0ull;
  if (idx < m) key[KW - 1] &= P.kmask;
  uint32_t slot = idx;
  // bitonic network: stages k = 2..S, steps j = k/2..1; a lane keeps the
  // smaller pair when it is the lower lane of an ascending block (or the
  // upper lane of a descending one)
#pragma unroll
  for (uint32_t k = 2; k <= uint32_t(S); k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      uint64_t ok[KW];
#pragma unroll
      for (int q = 0; q < KW; ++q) ok[q] = shfl64(key[q], int(lane ^ j));
      const uint32_t os = uint32_t(__shfl(int(slot), int(lane ^ j)));
      const bool other_less = key_lt<KW>(ok, key) || (key_eq<KW>(ok, key) && os < slot);
      const bool keep_min = ((idx & j) == 0) == ((idx & k) == 0);
      const bool take = keep_min ? other_less : !other_less;
#pragma unroll
      for (int q = 0; q < KW; ++q) key[q] = take ? ok[q] : key[q];
      slot = take ? os : slot;
    }
  }
  uint64_t out[RW];
#pragma unroll
  for (int q = 0; q < RW; ++q) out[q] = shfl64(rec[q], int(seg * uint32_t(S) + slot));
  if (idx < m) store_rec<RW>(job.dst, idx, out, false);
}

// One wave sorts one job of 65..64E records with Batcher's bitonic network
// over its (key, slot) pairs, E pairs per lane: lane l holds positions
// l * E .. l * E + E - 1, so compare-exchanges at distances below E stay
// inside a lane and longer ones exchange with lane l ^ (j / E).  Positions
// past the job hold pairs above any real one.  The sorted slots go to the
// wave's permutation in LDS; then lane l writes positions e * 64 + l
// (coalesced), each record read from the job's source by its slot (the key
// loads brought those lines into the cache); all of them are read before
// the first is written, since the source may be the destination.
template <int RW, int KW, int E>
__device__ __forceinline__ void tiny_pass_wide(const Params& P, uint32_t jid, uint32_t lane,
                                               uint16_t* perm) {
  constexpr uint32_t N = uint32_t(kWave) * E;
  const MidJob job = P.L.tiny[jid];
  const uint32_t m = min(job.size, N);
  const RADULS_GLOBAL uint64_t* src = gmem(reinterpret_cast<const uint64_t*>(job.src));
  uint64_t key[E][KW];
  uint32_t slot[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t p = lane * E + uint32_t(e);
    slot[e] = p;
    const uint32_t pl = p < m ? p : 0u;  // (every lane loads; padding is replaced below)
#pragma unroll
    for (int q = 0; q < KW; ++q) key[e][q] = src[uint64_t(pl) * RW + q];
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool pad = lane * E + uint32_t(e) >= m;
    key[e][KW - 1] &= P.kmask;
#pragma unroll
    for (int q = 0; q < KW; ++q) key[e][q] = pad ? ~0ull : key[e][q];
  }
  // (stage and step loops stay loops: unrolled, the network of every key
  // width made the code too large to compile in reasonable time)
#pragma unroll 1
  for (uint32_t k = 2; k <= N; k <<= 1) {
#pragma unroll 1
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j >= uint32_t(E)) {
        const int partner = int(lane ^ (j / E));
        const bool lower = (lane & (j / E)) == 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          uint64_t ok[KW];
#pragma unroll
          for (int q = 0; q < KW; ++q) ok[q] = shfl64(key[e][q], partner);
          const uint32_t os = uint32_t(__shfl(int(slot[e]), partner));
          const bool other_less = key_lt<KW>(ok, key[e]) || (key_eq<KW>(ok, key[e]) && os < slot[e]);
          const bool up = ((lane * E + uint32_t(e)) & k) == 0;
          const bool take = (lower == up) ? other_less : !other_less;
#pragma unroll
          for (int q = 0; q < KW; ++q) key[e][q] = take ? ok[q] : key[e][q];
          slot[e] = take ? os : slot[e];
        }
      } else {
        // inside a lane: distance 1, or 2 when E = 4
#pragma unroll
        for (int e = 0; e < E; ++e) {
#pragma unroll
          for (int jj = 1; jj < E; jj <<= 1) {
            if (uint32_t(jj) != j || (e & jj) != 0) continue;
            const int f = e + jj;
            const bool up = ((lane * E + uint32_t(e)) & k) == 0;
            const bool f_less =
                key_lt<KW>(key[f], key[e]) || (key_eq<KW>(key[f], key[e]) && slot[f] < slot[e]);
            const bool swap = up ? f_less : !f_less;  // (pairs are distinct)
#pragma unroll
            for (int q = 0; q < KW; ++q) {
              const uint64_t x = key[e][q], y = key[f][q];
              key[e][q] = swap ? y : x;
              key[f][q] = swap ? x : y;
            }
            const uint32_t sx = slot[e], sy = slot[f];
            slot[e] = swap ? sy : sx;
            slot[f] = swap ? sx : sy;
          }
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) perm[lane * E + uint32_t(e)] = uint16_t(slot[e]);
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
  // every record of the job is read before any is written: source and
  // destination are the same buffer when the job sits in its output already
  uint64_t rec[E][RW];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t q = uint32_t(e) * kWave + lane;
    load_rec<RW>(job.src, perm[q < m ? q : 0u], rec[e]);
  }
  __builtin_amdgcn_s_waitcnt(0x3F70);  // gfx9 encoding: vmcnt(0)
  asm volatile("" ::: "memory");
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t q = uint32_t(e) * kWave + lane;
    if (q < m) store_rec<RW>(job.dst, q, rec[e], false);
  }
  // (the next job rewrites perm only after every lane has read it)
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// Jobs come in groups of four per wave: four jobs of at most 16 records
// share one pass (16 lanes each), jobs of at most 32 go two per pass, larger
// ones one per pass (several bins per wave when they are small), those of
// more than 64 records with two or four records per lane.
template <int RW, int KW>
__global__ void __launch_bounds__(kMidBlock) k_tiny(Params P) {
  __shared__ uint16_t s_perm[kMidWaves][kTinyJob];
  const Ctrl* c = P.L.ctrl;
  const uint32_t n = min(c->tiny_count, P.L.cap_mid);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t waves = gridDim.x * uint32_t(kMidWaves);
  uint16_t* perm = s_perm[threadIdx.x >> 6];
  constexpr uint32_t G = 4;
  for (uint32_t g = blockIdx.x * uint32_t(kMidWaves) + (threadIdx.x >> 6); g < (n + G - 1) / G;
       g += waves) {
    const uint32_t first = g * G;
    uint32_t mx = 0;
    if (lane < G && first + lane < n) mx = P.L.tiny[first + lane].size;
    mx = max(mx, uint32_t(__shfl_xor(int(mx), 1)));
    mx = max(mx, uint32_t(__shfl_xor(int(mx), 2)));
    mx = uint32_t(__shfl(int(mx), 0));
    if (mx <= 16) {
      tiny_pass<RW, KW, 16>(P, first, n, lane);
    } else if (mx <= 32) {
      tiny_pass<RW, KW, 32>(P, first, n, lane);
      tiny_pass<RW, KW, 32>(P, first + 2, n, lane);
    } else {
#pragma unroll 1
      for (uint32_t u = 0; u < G && first + u < n; ++u) {
        const uint32_t sz = __builtin_amdgcn_readfirstlane(P.L.tiny[first + u].size);
        if (sz <= uint32_t(kWave)) {
          tiny_pass<RW, KW, kWave>(P, first + u, n, lane);
        } else if (sz <= 2u * kWave) {
          tiny_pass_wide<RW, KW, 2>(P, first + u, lane, perm);
        } else if constexpr (KW <= 2 && RW <= 4) {
          tiny_pass_wide<RW, KW, 4>(P, first + u, lane, perm);
        }
      }
    }
  }
}

// ------------------------------------------------------------ step outputs

// Copies the single bin's histogram (and its exclusive prefix) out of the
// workspace for the step entry points.
static __global__ void __launch_bounds__(256) k_step_out(Params P) {
  __shared__ uint32_t s_off[kRadix], s_scan[8];
  const uint32_t w = min(P.step_width, P.step_bits);
  const uint32_t nb = 1u << w;
  const uint32_t tid = threadIdx.x;
  const uint32_t h = tid < nb ? P.L.hist[0][tid] : 0;
  block_exclusive_scan256(h, s_off, s_scan);
  if (tid < nb) {
    if (P.d_counts_out) P.d_counts_out[tid] = h;
    if (P.d_offsets_out) P.d_offsets_out[tid] = s_off[tid];
  }
}

// ------------------------------------------------------------ launch sequence

template <auto Kern>
inline void set_lds_limit(uint32_t bytes) {
  static uint32_t done = 0;
  if (done < bytes) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(Kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    done = bytes;
  }
}

// Optional measurement events (see raduls_set_profile_events): pairs of
// events recorded around kernel classes on the launch stream.
struct ProfileEvents {
  hipEvent_t ev[2 * kProfileSlots];
  uint32_t count;
};
extern ProfileEvents g_profile;

inline void prof_mark(uint32_t slot, int end, hipStream_t s) {
  const uint32_t i = 2 * slot + uint32_t(end);
  if (i < g_profile.count && g_profile.ev[i]) (void)hipEventRecord(g_profile.ev[i], s);
}

template <int RW, int KW, int TOP>
inline void launch_scatter(const Params& P, uint32_t cur, hipStream_t s) {
  if (P.lookback) {
    k_scatter<RW, KW, TOP, 1><<<P.grid_scatter, kScatterBlock, P.scatter_lds_bytes, s>>>(P, cur);
  } else {
    k_carry<<<kRadix, 1024, 0, s>>>(P, P.grid_hist);
    k_scatter_carry<RW, KW, TOP><<<P.grid_hist, kScatterBlock, P.scatter_lds_bytes, s>>>(P, cur);
  }
}

template <int RW, int KW>
hipError_t run_sequence(const Params& P, hipStream_t s) {
  set_lds_limit<k_scatter_carry<RW, KW, 1>>(P.scatter_lds_bytes);
  set_lds_limit<k_scatter_carry<RW, KW, 0>>(P.scatter_lds_bytes);
  set_lds_limit<k_scatter<RW, KW, 1, 1>>(P.scatter_lds_bytes);
  set_lds_limit<k_scatter<RW, KW, 0, 1>>(P.scatter_lds_bytes);
  set_lds_limit<k_mid<RW, KW>>(P.mid_lds_bytes);
  if (P.pair) set_lds_limit<k_hist<RW, KW, 2>>(kPairWords * 4);
  if (P.mode == kModeBatch) {
    k_zero_ctrl<<<1, 64, 0, s>>>(P);
    const uint32_t g = P.count ? (P.count + 255) / 256 : 1;
    k_seed_batch<<<g < 1024 ? g : 1024, 256, 0, s>>>(P);
  } else {
    k_seed_single<<<1, 64, 0, s>>>(P);
  }
  if (P.mode == kModeHist || P.mode == kModePartition) {
    k_prep<<<1, 1024, 0, s>>>(P, 0, 0);
    k_hist<RW, KW, 1><<<P.grid_hist, kScatterBlock, 0, s>>>(P, 0);
    if (P.mode == kModePartition) launch_scatter<RW, KW, 1>(P, 0, s);
    k_step_out<<<1, 256, 0, s>>>(P);
    return hipGetLastError();
  }
  for (uint32_t r = 0; r < P.rounds; ++r) {
    const uint32_t cur = r & 1;
    const uint32_t slot = r == 0 ? kProfTopHist : kProfRoundHist;
    k_prep<<<1, 1024, 0, s>>>(P, cur, r);
    if (r <= 1) prof_mark(slot, 0, s);
    if (r == 0 && P.pair) {
      k_hist<RW, KW, 2><<<P.grid_hist, kScatterBlock, kPairWords * 4, s>>>(P, cur);
      k_pair_reduce<<<(kPairWords / 256) * kPairGroups, 256, 0, s>>>(P, P.grid_hist);
    } else if (r == 0) {
      k_hist<RW, KW, 1><<<P.grid_hist, kScatterBlock, 0, s>>>(P, cur);
    } else {
      k_hist<RW, KW, 0><<<P.grid_hist, kScatterBlock, 0, s>>>(P, cur);
    }
    if (r <= 1) prof_mark(slot, 1, s);
    if (r <= 1) prof_mark(slot + 1, 0, s);
    if (r == 0) launch_scatter<RW, KW, 1>(P, cur, s);
    else launch_scatter<RW, KW, 0>(P, cur, s);
    if (r <= 1) prof_mark(slot + 1, 1, s);
    k_classify<KW><<<P.grid_classify, 256, 0, s>>>(P, cur, r);
  }
  if (P.inspect) return hipGetLastError();
  // a single array of at most mid_max records (no rounds) is one job, which
  // the seed put on the tiny list or the LDS list by its size; nothing can
  // end in tmp.  Only that job's sorter is launched.
  const bool one_job = P.mode == kModeSort && P.rounds == 0;
  prof_mark(kProfMid, 0, s);
  if (!one_job || P.n <= P.tiny_job) k_tiny<RW, KW><<<P.grid_tiny, kMidBlock, 0, s>>>(P);
  if (!one_job || P.n > P.tiny_job)
    k_mid<RW, KW><<<P.grid_mid, kMidBlock, P.mid_lds_bytes, s>>>(P);
  prof_mark(kProfMid, 1, s);
  return hipGetLastError();
}

template <int RW>
hipError_t run_rw(const Params& P, uint32_t kw, hipStream_t s) {
  switch (kw) {
#define RADULS_KW_CASE(N) \
  case N:                 \
    if constexpr (N <= RW) return run_sequence<RW, N>(P, s); \
    break;
    RADULS_KW_CASE(1)
    RADULS_KW_CASE(2)
    RADULS_KW_CASE(3)
    RADULS_KW_CASE(4)
    RADULS_KW_CASE(5)
    RADULS_KW_CASE(6)
    RADULS_KW_CASE(7)
    RADULS_KW_CASE(8)
#undef RADULS_KW_CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

// The resident server's launch: `wgs` workgroups of the LDS sorter in server
// mode, which stay until the ring's stop word is set or they idle out.
template <int RW, int KW>
hipError_t serve_launch(const Params& P, uint32_t wgs, hipStream_t s) {
  set_lds_limit<k_mid<RW, KW, 1>>(P.mid_lds_bytes);
  k_mid<RW, KW, 1><<<wgs, kMidBlock, P.mid_lds_bytes, s>>>(P);
  return hipGetLastError();
}

template <int RW>
hipError_t serve_rw(const Params& P, uint32_t kw, uint32_t wgs, hipStream_t s) {
  switch (kw) {
#define RADULS_KW_CASE(N) \
  case N:                 \
    if constexpr (N <= RW) return serve_launch<RW, N>(P, wgs, s); \
    break;
    RADULS_KW_CASE(1)
    RADULS_KW_CASE(2)
    RADULS_KW_CASE(3)
    RADULS_KW_CASE(4)
    RADULS_KW_CASE(5)
    RADULS_KW_CASE(6)
    RADULS_KW_CASE(7)
    RADULS_KW_CASE(8)
#undef RADULS_KW_CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace raduls
