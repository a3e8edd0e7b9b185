// Device kernels of libraduls (gfx950, wave64).  Included by one translation
// unit per record width; each instantiates the kernels for its R = 8*RW and
// every key width KW = ceil(K/8) <= RW.
//
// The sort is an MSD radix sort of fixed-size records (RADULS2, Sec. 3):
//   round r (large bins):  k_prep     tile counts of the round's bins
//                          k_hist     per-bin digit histogram (+ key spread)
//                          k_scatter  stable scatter with decoupled look-back
//                          k_classify child bins -> next round / LDS jobs
//   then                   k_mid      bins that fit in LDS, sorted there; tiny
//                                     sub-bins by enumeration sort
//                          k_copy     finished bins left in tmp -> recs
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

// Bits [lo, lo + w) of a multi-word key, 1 <= w <= 8.
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

__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t u = __shfl_up(v, o);
    if (lane >= uint32_t(o)) v += u;
  }
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
__device__ __forceinline__ void push_large(const Params& P, uint32_t nxt, const Bin& b) {
  uint32_t i;
  if (!push_bin(P.L.large[nxt], &P.L.ctrl->large_count[nxt], P.L.cap_large, b, &P.L.ctrl->error, &i))
    return;
  uint4* h = reinterpret_cast<uint4*>(P.L.hist[nxt] + uint64_t(i) * kRadix);
  for (int q = 0; q < kRadix / 4; ++q) h[q] = make_uint4(0, 0, 0, 0);
  uint64_t* df = P.L.diff[nxt] + uint64_t(i) * 8;
  for (int q = 0; q < 8; ++q) df[q] = 0;
}

// Copy jobs for a finished run of records that sits in tmp.
__device__ __forceinline__ void push_copy(const Params& P, uint32_t array, uint32_t start,
                                          uint32_t size) {
  const uint32_t chunks = (size + kCopyChunk - 1) / kCopyChunk;
  const uint32_t i0 = atomicAdd(&P.L.ctrl->copy_count, chunks);
  for (uint32_t c = 0; c < chunks; ++c) {
    if (i0 + c >= P.L.cap_copy) {
      atomicOr(&P.L.ctrl->error, kErrCapacity);
      return;
    }
    Bin j;
    j.start = start + c * kCopyChunk;
    j.size = min(kCopyChunk, size - c * kCopyChunk);
    j.array = array;
    j.bits = 0;
    j.side = 1;
    j.flags = 0;
    P.L.copy[i0 + c] = j;
  }
}

// ------------------------------------------------------------ seeding

// Clears the control block and installs the root bin of a single-array call.
static __global__ void __launch_bounds__(64) k_seed_single(Params P) {
  Ctrl* c = P.L.ctrl;
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
      b.bits = uint16_t(8 * P.K);
      if (P.n > P.mid_max) {
        P.L.large[0][0] = b;
        c->large_count[0] = 1;
      } else if (P.n >= 2) {
        P.L.mid[0] = b;
        c->mid_count = 1;
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
    if (d.n > P.mid_max) push_large(P, 0, b);
    else if (d.n >= 2) push_bin(P.L.mid, &c->mid_count, P.L.cap_mid, b, &c->error);
  }
}

// ------------------------------------------------------------ round: prep

// Tile prefix over the round's large bins (one workgroup).
static __global__ void __launch_bounds__(1024) k_prep(Params P, uint32_t cur) {
  __shared__ uint32_t s_part[16];
  __shared__ unsigned long long s_sz[16];
  Ctrl* c = P.L.ctrl;
  const uint32_t nb = min(c->large_count[cur], P.L.cap_large);
  const Bin* bins = P.L.large[cur];
  const uint32_t t = threadIdx.x, wave = t >> 6, lane = t & 63;
  uint32_t running = 0;
  unsigned long long records = 0;
  for (uint32_t base = 0; base < nb; base += 1024) {
    const uint32_t i = base + t;
    uint32_t v = 0;
    uint32_t sz = 0;
    if (i < nb) {
      sz = bins[i].size;
      v = (sz + P.tile - 1) / P.tile;
    }
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
  if (t == 0) {
    P.L.tile_prefix[nb] = running;
    c->round_tiles = running;
    c->ticket = 0;
    c->large_count[cur ^ 1] = 0;
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
template <int RW, int KW, int TOP>
__global__ void __launch_bounds__(kScatterBlock) k_hist(Params P, uint32_t cur) {
  constexpr int ITEMS = scatter_items(RW);
  constexpr int W = kScatterWaves;
  constexpr uint32_t TILE = kScatterBlock * ITEMS;
  __shared__ uint32_t s_cnt[W * kRadix];
  __shared__ unsigned long long s_diff[W][KW];

  const Ctrl* c = P.L.ctrl;
  const uint32_t total = c->round_tiles;
  const uint32_t nbins = min(c->large_count[cur], P.L.cap_large);
  if (total == 0) return;
  const uint32_t t0 = uint32_t(uint64_t(total) * blockIdx.x / gridDim.x);
  const uint32_t t1 = uint32_t(uint64_t(total) * (blockIdx.x + 1) / gridDim.x);
  if (t0 >= t1) return;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

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

  Bin bin = P.L.large[cur][b];
  ArrayDesc arr = P.L.arrays[bin.array];
  const uint8_t* src = bin.side ? arr.tmp : arr.recs;
  uint64_t key0[KW];
  key_of<KW>(gmem(reinterpret_cast<const uint64_t*>(src)) + uint64_t(bin.start) * RW, P.kmask, key0);

  for (uint32_t t = t0; t < t1; ++t) {
    while (b + 1 < nbins && t >= tp[b + 1]) {
      flush(b, false);
      ++b;
      bin = P.L.large[cur][b];
      arr = P.L.arrays[bin.array];
      src = bin.side ? arr.tmp : arr.recs;
      key_of<KW>(gmem(reinterpret_cast<const uint64_t*>(src)) + uint64_t(bin.start) * RW, P.kmask, key0);
    }
    if (tid == 0) P.L.tile_bin[t] = b;
    const uint32_t k = t - tp[b];
    const uint32_t tbeg = bin.start + k * TILE;
    const uint32_t tn = min(TILE, bin.size - k * TILE);
    const uint32_t ipw = (tn + kWave * W - 1) / (kWave * W);
    const uint32_t w = min(P.digit_bits, uint32_t(bin.bits));
    const uint32_t lob = bin.bits - w;
    const RADULS_GLOBAL uint64_t* sw = gmem(reinterpret_cast<const uint64_t*>(src));
    uint32_t dg[ITEMS];
    bool valid[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t i = wave * ipw * kWave + j * kWave + lane;
      valid[j] = (uint32_t(j) < ipw) && (i < tn);
      dg[j] = 0;
      if (valid[j]) {
        uint64_t key[KW];
        key_of<KW>(sw + uint64_t(tbeg + i) * RW, P.kmask, key);
        dg[j] = digit_of<KW>(key, lob, w);
#pragma unroll
        for (int q = 0; q < KW; ++q) dacc[q] |= key[q] ^ key0[q];
      }
    }
    uint32_t* wc = s_cnt + wave * kRadix;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint64_t peers = match_digit(dg[j], valid[j], w);
      if (valid[j] && __popcll(peers & lanemask_lt()) == 0) wc[dg[j]] += __popcll(peers);
    }
  }
  flush(b, true);
  if (tid == 0) {
    // bit 0: the range starts a bin; bit 1: the whole range lies in one bin
    P.L.wg_flag[blockIdx.x] = (t0 == tp[b_first] ? 1u : 0u) | (b_first == b ? 2u : 0u);
  }
}

// Carry of every histogram range: the per-digit count of records of the
// range's first bin that lie in earlier ranges (the blocked form of the
// exclusive scan over tiles).  One workgroup, one thread per digit.
static __global__ void __launch_bounds__(256) k_carry(Params P, uint32_t nranges) {
  const Ctrl* c = P.L.ctrl;
  const uint32_t total = c->round_tiles;
  if (total == 0) return;
  const uint32_t d = threadIdx.x;
  uint32_t carry = 0, tail = 0, single = 0;
  for (uint32_t g = 0; g < nranges; ++g) {
    const uint32_t t0 = uint32_t(uint64_t(total) * g / nranges);
    const uint32_t t1 = uint32_t(uint64_t(total) * (g + 1) / nranges);
    if (t0 >= t1) continue;
    const uint32_t f = P.L.wg_flag[g];
    carry = (f & 1u) ? 0u : tail + (single ? carry : 0u);
    P.L.wg_carry[uint64_t(g) * kRadix + d] = carry;
    tail = P.L.wg_tail[uint64_t(g) * kRadix + d];
    single = f & 2u;
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
    const uint32_t w = min(P.digit_bits, uint32_t(bin.bits));
    const uint32_t lob = bin.bits - w;
    const uint32_t nb = 1u << w;

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

    const uint32_t tbeg = bin.start + k * TILE;
    const uint32_t tn = min(TILE, bin.size - k * TILE);
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
        dg[j] = digit_of<KW>(key, lob, w);
      }
    }
    uint16_t* wc = s_cnt + wave * kRadix;
    for (int q = lane; q < kRadix; q += kWave) wc[q] = 0;
    wave_rank<ITEMS>(dg, valid, w, wc, rank);
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
  uint64_t* s_rec = reinterpret_cast<uint64_t*>(smem);
  uint8_t* s_dig = reinterpret_cast<uint8_t*>(s_rec + TILE * RW);
  uint16_t* s_cnt = reinterpret_cast<uint16_t*>(s_dig + TILE);
  uint32_t* s_tot = reinterpret_cast<uint32_t*>(s_cnt + W * kRadix);
  uint32_t* s_off = s_tot + kRadix;
  uint32_t* s_binoff = s_off + kRadix;
  uint64_t* s_gbase = reinterpret_cast<uint64_t*>(s_binoff + kRadix);
  __shared__ uint32_t s_scan[8];

  Ctrl* c = P.L.ctrl;
  const uint32_t total = c->round_tiles;
  const uint32_t r0 = uint32_t(uint64_t(total) * blockIdx.x / gridDim.x);
  const uint32_t r1 = uint32_t(uint64_t(total) * (blockIdx.x + 1) / gridDim.x);
  if (r0 >= r1) return;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const bool nt = P.nontemporal != 2;
  uint32_t running = tid < kRadix ? P.L.wg_carry[uint64_t(blockIdx.x) * kRadix + tid] : 0;

  // state of the bin the current tile belongs to (uniform)
  uint32_t b = 0, w = 0, lob = 0, nb = 0;
  Bin bin{};
  const uint8_t* src = nullptr;
  uint8_t* dst = nullptr;
  bool active = false;
  auto enter_bin = [&](uint32_t t) {
    b = P.L.tile_bin[t];
    bin = P.L.large[cur][b];
    const ArrayDesc arr = P.L.arrays[bin.array];
    src = bin.side ? arr.tmp : arr.recs;
    dst = bin.side ? arr.recs : arr.tmp;
    w = min(P.digit_bits, uint32_t(bin.bits));
    lob = bin.bits - w;
    nb = 1u << w;
    const uint32_t h = tid < nb ? P.L.hist[cur][uint64_t(b) * kRadix + tid] : 0;
    active = true;
    if (P.mode != kModePartition) {
      uint64_t any = 0;
#pragma unroll
      for (int i = 0; i < KW; ++i) any |= P.L.diff[cur][uint64_t(b) * 8 + i];
      // all keys equal, or a digit shared by the whole bin: nothing moves
      active = any != 0 && !__syncthreads_or(tid < nb && h == bin.size);
    }
    if (active) block_exclusive_scan256(h, s_binoff, s_scan);
  };

  uint64_t rec[ITEMS][RW];
  auto tile_span = [&](uint32_t t, uint32_t& tbeg, uint32_t& tn, uint32_t& ipw) {
    const uint32_t k = t - P.L.tile_prefix[b];
    tbeg = bin.start + k * TILE;
    tn = min(TILE, bin.size - k * TILE);
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
  while (t < r1) {
    if (t == P.L.tile_prefix[b]) running = 0;  // a new bin starts inside the range
    uint32_t tbeg, tn, ipw;
    tile_span(t, tbeg, tn, ipw);
    uint32_t dg[ITEMS];
    bool valid[ITEMS];
    if (active) {
      uint32_t rank[ITEMS];
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = wave * ipw * kWave + j * kWave + lane;
        valid[j] = (uint32_t(j) < ipw) && (i < tn);
        dg[j] = 0;
        if (valid[j]) {
          uint64_t key[KW];
          key_of<KW>(rec[j], P.kmask, key);
          dg[j] = digit_of<KW>(key, lob, w);
        }
      }
      uint16_t* wc = s_cnt + wave * kRadix;
      for (int q = lane; q < kRadix; q += kWave) wc[q] = 0;
      wave_rank<ITEMS>(dg, valid, w, wc, rank);
      lds_barrier();
      block_digit_scan<W>(s_cnt, s_tot, s_off, s_scan);
      if (tid < nb) {
        s_gbase[tid] = uint64_t(bin.start) + s_binoff[tid] + running - s_off[tid];
        running += s_tot[tid];
      }
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        if (valid[j]) {
          const uint32_t pos = s_off[dg[j]] + wc[dg[j]] + rank[j];
#pragma unroll
          for (int q = 0; q < RW; ++q) s_rec[pos * RW + q] = rec[j][q];
          s_dig[pos] = uint8_t(dg[j]);
        }
      }
      lds_barrier();
    }
    const uint32_t next = t + 1;
    const bool same = next < r1 && P.L.tile_bin[next] == b;
    if (active && same) issue_loads(next);  // registers are free once staged
    if (active) {
      bool oob = false;
      for (uint32_t p = tid; p < tn; p += kScatterBlock) {
        const uint32_t d = s_dig[p];
        const uint64_t at = s_gbase[d] + p;
        // never write outside the bin, whatever the counts say
        if (at - bin.start < bin.size) store_rec<RW>(dst, at, s_rec + uint64_t(p) * RW, nt);
        else oob = true;
      }
      if (oob) atomicOr(&c->error, kErrBounds);
    }
    lds_barrier();
    t = next;
    if (t < r1 && !same) {
      enter_bin(t);
      if (active) issue_loads(t);
    }
  }
}

// ------------------------------------------------------------ round: classify

// Decide what happens to each large bin after the round (Sec. 3.1-3.3): all
// keys equal -> finished; digit constant -> same bin, next differing digit;
// otherwise its children become next-round large bins or LDS jobs.  Small
// siblings are packed greedily into jobs of at most mid_max records (Sec. 3.3
// remarks that scanning empty sub-bins one by one costs time).
template <int KW>
__global__ void __launch_bounds__(256) k_classify(Params P, uint32_t cur) {
  __shared__ uint32_t s_cnt[kRadix], s_off[kRadix], s_scan[8];
  Ctrl* c = P.L.ctrl;
  const uint32_t nbins = min(c->large_count[cur], P.L.cap_large);
  const uint32_t nxt = cur ^ 1;
  const uint32_t tid = threadIdx.x;
  for (uint32_t b = blockIdx.x; b < nbins; b += gridDim.x) {
    __syncthreads();
    const Bin bin = P.L.large[cur][b];
    const uint32_t w = min(P.digit_bits, uint32_t(bin.bits));
    const uint32_t lob = bin.bits - w;
    const uint32_t nb = 1u << w;
    uint64_t dif[KW];
#pragma unroll
    for (int i = 0; i < KW; ++i) dif[i] = P.L.diff[cur][uint64_t(b) * 8 + i];
    const int tb = top_bit<KW>(dif);
    if (tb < 0) {  // every key equal: finished where it is
      if (tid == 0 && bin.side == 1) push_copy(P, bin.array, bin.start, bin.size);
      continue;
    }
    const uint32_t h = tid < nb ? P.L.hist[cur][uint64_t(b) * kRadix + tid] : 0;
    if (__syncthreads_or(tid < nb && h == bin.size)) {
      if (tid == 0) {
        Bin nbn = bin;
        nbn.bits = uint16_t(tb + 1);
        push_large(P, nxt, nbn);
      }
      continue;
    }
    s_cnt[tid] = h;
    block_exclusive_scan256(h, s_off, s_scan);
    const uint8_t cside = bin.side ^ 1;
    if (tid == 0) {
      atomicAdd(&c->scattered_bins, 1u);
      atomicAdd(&c->moved_records, (unsigned long long)bin.size);
    }
    if (lob == 0) {  // key exhausted: every child holds equal keys
      if (tid == 0 && cside == 1) push_copy(P, bin.array, bin.start, bin.size);
      continue;
    }
    if (tid < nb && h > P.mid_max) {
      Bin ch;
      ch.start = bin.start + s_off[tid];
      ch.size = h;
      ch.array = bin.array;
      ch.bits = uint16_t(lob);
      ch.side = cside;
      ch.flags = 0;
      push_large(P, nxt, ch);
    }
    if (tid == 0) {
      uint32_t js = 0, jn = 0, jc = 0;
      auto flush = [&]() {
        if (jn > 0 && !(jn == 1 && cside == 0)) {
          Bin j;
          j.start = bin.start + js;
          j.size = jn;
          j.array = bin.array;
          j.bits = uint16_t(jc == 1 ? lob : bin.bits);
          j.side = cside;
          j.flags = uint8_t(jc > 1);
          push_bin(P.L.mid, &c->mid_count, P.L.cap_mid, j, &c->error);
        }
        jn = 0;
        jc = 0;
      };
      for (uint32_t d = 0; d < nb; ++d) {
        const uint32_t cd = s_cnt[d];
        if (cd == 0) continue;
        if (cd > P.mid_max) {
          flush();
          continue;
        }
        if (jn + cd > P.mid_max) flush();
        if (jn == 0) js = s_off[d];
        jn += cd;
        ++jc;
      }
      flush();
    }
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
// order; every pass permutes `perm`, the slots in sorted order.
struct MidLds {
  uint64_t* key;    // [T * KW] keys of the job (masked), input order
  uint16_t* perm;   // [T] position -> record slot
  uint16_t* cnt;    // [kMidWaves * kRadix] per-wave ranking counters
  uint32_t* bm;     // boundary bitmap: bit p set where a sub-range starts
  uint32_t* big;    // ranges waiting for a workgroup pass (start | size << 16)
  uint32_t* list0;  // ranges waiting for a wave pass, double-buffered by round
  uint32_t* list1;
  uint32_t* nbig;
  uint32_t* nlist;  // [2]
  uint32_t* claim;  // next entry of the current list to claim
  uint32_t* tot;    // [kRadix]
  uint32_t* off;    // [kRadix]
  uint32_t* scan;   // [8]
  unsigned long long* diff;  // [kMidWaves * KW]
};

template <int RW, int KW>
__device__ __forceinline__ void slot_key(const Params& P, const MidLds& L, uint32_t slot,
                                         uint64_t (&k)[KW]) {
#pragma unroll
  for (int q = 0; q < KW; ++q) k[q] = L.key[uint64_t(slot) * KW + q];
}

// Route a sub-range by size: > wave capacity -> workgroup pass, > tiny ->
// wave pass, else enumeration sort later.  Its start is always marked.
__device__ __forceinline__ void mid_route(const Params& P, MidLds& L, uint32_t st, uint32_t cnt,
                                          uint32_t bits_left, uint32_t wave_cap, uint32_t lst) {
  atomicOr(&L.bm[st >> 5], 1u << (st & 31));
  if (cnt <= P.tiny_max || bits_left == 0) return;
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

// Stable workgroup pass over positions [s, s + m): ranks the records at those
// positions by the digit [lob, lob + w) and rewrites perm[s .. s+m) in digit
// order.  When `identity`, perm is not read (position i holds slot i).
// Returns through L.tot / L.off the digit counts and offsets.  All threads call.
template <int RW, int KW, int ITEMS>
__device__ __forceinline__ void mid_wg_digit(const Params& P, MidLds& L, uint32_t s, uint32_t m,
                                             uint32_t lob, uint32_t w, bool identity) {
  constexpr int W = kMidWaves;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t ipw = (m + kWave * W - 1) / (kWave * W);
  uint32_t src[ITEMS], dg[ITEMS], rank[ITEMS];
  bool valid[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t i = wave * ipw * kWave + j * kWave + lane;
    valid[j] = (uint32_t(j) < ipw) && (i < m);
    src[j] = 0;
    dg[j] = 0;
    if (valid[j]) {
      src[j] = identity ? s + i : L.perm[s + i];
      uint64_t key[KW];
      slot_key<RW, KW>(P, L, src[j], key);
      dg[j] = digit_of<KW>(key, lob, w);
    }
  }
  uint16_t* wc = L.cnt + wave * kRadix;
  for (int q = lane; q < kRadix; q += kWave) wc[q] = 0;
  wave_rank<ITEMS>(dg, valid, w, wc, rank);
  lds_barrier();  // every perm entry of the range has been read
  block_digit_scan<W>(L.cnt, L.tot, L.off, L.scan);
#pragma unroll
  for (int j = 0; j < ITEMS; ++j)
    if (valid[j]) L.perm[s + L.off[dg[j]] + wc[dg[j]] + rank[j]] = uint16_t(src[j]);
}

// Key spread of positions [s, s + m) over the workgroup: the highest bit in
// which their keys differ, or -1.  All threads call.
template <int RW, int KW>
__device__ __forceinline__ int mid_wg_top_bit(const Params& P, MidLds& L, uint32_t s, uint32_t m,
                                              bool identity) {
  constexpr int W = kMidWaves;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint64_t key0[KW], dacc[KW];
  slot_key<RW, KW>(P, L, identity ? s : L.perm[s], key0);
#pragma unroll
  for (int q = 0; q < KW; ++q) dacc[q] = 0;
  for (uint32_t i = threadIdx.x; i < m; i += kMidBlock) {
    uint64_t key[KW];
    slot_key<RW, KW>(P, L, identity ? s + i : L.perm[s + i], key);
#pragma unroll
    for (int q = 0; q < KW; ++q) dacc[q] |= key[q] ^ key0[q];
  }
#pragma unroll
  for (int q = 0; q < KW; ++q) {
    const uint64_t v = wave_or(dacc[q]);
    if (lane == 0) L.diff[wave * KW + q] = v;
  }
  lds_barrier();
  uint64_t dall[KW];
#pragma unroll
  for (int q = 0; q < KW; ++q) {
    dall[q] = 0;
    for (int w2 = 0; w2 < W; ++w2) dall[q] |= L.diff[w2 * KW + q];
  }
  lds_barrier();  // L.diff is reused by the next call
  return top_bit<KW>(dall);
}

// Workgroup pass over a range larger than one wave can hold: split it on the
// highest digit in which its keys differ and route the sub-ranges.
template <int RW, int KW>
__device__ __forceinline__ void mid_wg_pass(const Params& P, MidLds& L, uint32_t s, uint32_t m,
                                            uint32_t wave_cap) {
  const int tb = mid_wg_top_bit<RW, KW>(P, L, s, m, false);
  if (tb < 0) return;  // all keys equal: in order
  const uint32_t hb = uint32_t(tb) + 1;
  const uint32_t w = min(P.digit_bits, hb);
  const uint32_t lob = hb - w;
  mid_wg_digit<RW, KW, mid_items(RW, KW)>(P, L, s, m, lob, w, false);
  const uint32_t tid = threadIdx.x;
  if (tid < (1u << w) && L.tot[tid]) mid_route(P, L, s + L.off[tid], L.tot[tid], lob, wave_cap, 0);
  lds_barrier();
}

// Stable pass of one wave over positions [s, s + m), m <= 64 * WI, on the
// highest digit in which their keys differ; sub-ranges go to list `nxt`.
template <int RW, int KW, int WI>
__device__ __forceinline__ void mid_wave_pass(const Params& P, MidLds& L, uint32_t s, uint32_t m,
                                              uint32_t nxt, uint32_t wave_cap) {
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t src[WI];
  bool valid[WI];
  uint64_t key0[KW], dacc[KW];
  slot_key<RW, KW>(P, L, L.perm[s], key0);
#pragma unroll
  for (int q = 0; q < KW; ++q) dacc[q] = 0;
#pragma unroll
  for (int j = 0; j < WI; ++j) {
    const uint32_t i = j * kWave + lane;
    valid[j] = i < m;
    src[j] = 0;
    if (valid[j]) {
      src[j] = L.perm[s + i];
      uint64_t key[KW];
      slot_key<RW, KW>(P, L, src[j], key);
#pragma unroll
      for (int q = 0; q < KW; ++q) dacc[q] |= key[q] ^ key0[q];
    }
  }
#pragma unroll
  for (int q = 0; q < KW; ++q) dacc[q] = wave_or(dacc[q]);
  const int tb = top_bit<KW>(dacc);
  if (tb < 0) return;  // all keys equal
  const uint32_t hb = uint32_t(tb) + 1;
  const uint32_t w = min(P.digit_bits, hb);
  const uint32_t lob = hb - w;
  uint32_t dg[WI], rank[WI];
#pragma unroll
  for (int j = 0; j < WI; ++j) {
    dg[j] = 0;
    if (valid[j]) {
      uint64_t key[KW];
      slot_key<RW, KW>(P, L, src[j], key);
      dg[j] = digit_of<KW>(key, lob, w);
    }
  }
  uint16_t* wc = L.cnt + wave * kRadix;
#pragma unroll
  for (int q = 0; q < kRadix / kWave; ++q) wc[lane * 4 + q] = 0;
  __builtin_amdgcn_wave_barrier();
  wave_rank<WI>(dg, valid, w, wc, rank);
  __builtin_amdgcn_wave_barrier();
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
    wc[lane * 4 + q] = uint16_t(run);
    if (c[q]) mid_route(P, L, s + run, c[q], lob, wave_cap, nxt);
    run += c[q];
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < WI; ++j)
    if (valid[j]) L.perm[s + wc[dg[j]] + rank[j]] = uint16_t(src[j]);
}

// First split of a job: the highest key bit in which its records differ
// gives the top of the next two digits; two stable digit passes (lower digit
// first, so the pair acts as one 2*digit_bits-bit digit) order the job by
// those bits.  Runs of equal bits are marked in the boundary bitmap; runs
// longer than tiny_max with key bits left below are routed to further passes.
template <int RW, int KW>
__device__ __forceinline__ void mid_first_split(const Params& P, MidLds& L, uint32_t m,
                                                uint32_t wave_cap) {
  constexpr int ITEMS = mid_items(RW, KW);
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tb = mid_wg_top_bit<RW, KW>(P, L, 0, m, true);
  if (tb < 0) {  // the whole job holds one key: it stays in input order
    for (uint32_t i = tid; i < m; i += kMidBlock) L.perm[i] = uint16_t(i);
    if (tid == 0) L.bm[0] = 1u;
    lds_barrier();
    return;
  }
  const uint32_t hb = uint32_t(tb) + 1;
  const uint32_t dw = P.digit_bits;
  const uint32_t lo2 = hb > 2 * dw ? hb - 2 * dw : 0;
  const uint32_t wa = min(dw, hb - lo2);
  mid_wg_digit<RW, KW, ITEMS>(P, L, 0, m, lo2, wa, true);
  if (hb > lo2 + wa) {
    lds_barrier();
    mid_wg_digit<RW, KW, ITEMS>(P, L, 0, m, lo2 + wa, hb - lo2 - wa, false);
  }
  lds_barrier();
  // run starts: the key bits [lo2, hb) differ from the previous record's
  const uint32_t fw = hb - lo2;
  for (uint32_t base = wave * kWave; base < m; base += kMidBlock) {
    const uint32_t p = base + lane;
    bool start = false;
    if (p < m) {
      start = p == 0;
      if (p > 0) {
        uint64_t kp[KW], kq[KW];
        slot_key<RW, KW>(P, L, L.perm[p], kp);
        slot_key<RW, KW>(P, L, L.perm[p - 1], kq);
        start = digit_of<KW>(kp, lo2, fw) != digit_of<KW>(kq, lo2, fw);
      }
    }
    const uint64_t bal = __ballot(start);
    if (lane == 0) {
      L.bm[base >> 5] = uint32_t(bal);
      L.bm[(base >> 5) + 1] = uint32_t(bal >> 32);
    }
  }
  lds_barrier();
  if (lo2 > 0) {
    for (uint32_t p = tid; p < m; p += kMidBlock) {
      if (L.bm[p >> 5] & (1u << (p & 31))) {
        const int e = bm_next(L.bm, int(p), int(m) - 1);
        const uint32_t len = (e < 0 ? m : uint32_t(e)) - p;
        if (len > P.tiny_max) mid_route(P, L, p, len, lo2, wave_cap, 0);
      }
    }
  }
  lds_barrier();
}

// Sorts jobs of at most mid_max records entirely in LDS (the small-bin case of
// Sec. 3.2, with LDS in the role of the cache).  The job's keys are read from
// HBM once into LDS, where they stay; every pass permutes a 16-bit index array
// instead of moving records.  A first split orders the job by the 2*digit_bits
// key bits below the highest bit in which its keys differ; ranges still larger
// than tiny_max get further passes, by the whole workgroup when they exceed
// one wave's capacity, else by single waves in parallel, round by round.
// Ranges of at most tiny_max records are finished by enumeration sort
// (Sec. 2.2, 3.3): each record's place is the number of smaller keys plus the
// number of equal keys before it.  Finally every thread gathers its records
// through the permutation from the job's source (just read, so it is served
// from cache), the workgroup waits until all of them are in registers, and
// the job is written back in one coalesced pass.
template <int RW, int KW>
__global__ void __launch_bounds__(kMidBlock, 4) k_mid(Params P) {
  constexpr int W = kMidWaves;
  constexpr int WI = mid_wave_items(RW);
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint32_t s_big[kMidBigCap];
  __shared__ uint32_t s_list[2][kMidListCap];
  __shared__ uint32_t s_nbig, s_nlist[2], s_claim;
  __shared__ uint32_t s_tot[kRadix], s_off[kRadix], s_scan[8];
  __shared__ unsigned long long s_diff[W * KW];

  const uint32_t T = P.mid_max;
  MidLds L;
  L.key = reinterpret_cast<uint64_t*>(smem);
  L.perm = reinterpret_cast<uint16_t*>(L.key + uint64_t(T) * KW);
  L.cnt = L.perm + align_up(T, 2);
  L.bm = reinterpret_cast<uint32_t*>(L.cnt + W * kRadix);
  L.big = s_big;
  L.list0 = s_list[0];
  L.list1 = s_list[1];
  L.nbig = &s_nbig;
  L.nlist = s_nlist;
  L.claim = &s_claim;
  L.tot = s_tot;
  L.off = s_off;
  L.scan = s_scan;
  L.diff = s_diff;

  Ctrl* c = P.L.ctrl;
  const uint32_t njobs = min(c->mid_count, P.L.cap_mid);
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t tiny = P.tiny_max;
  const uint32_t wave_cap = kWave * WI;

  for (uint32_t jb = blockIdx.x; jb < njobs; jb += gridDim.x) {
    const Bin job = P.L.mid[jb];
    const uint32_t m = job.size;
    if (m > T) {
      if (tid == 0) atomicOr(&c->error, kErrMidSize);
      continue;
    }
    const ArrayDesc arr = P.L.arrays[job.array];
    const uint64_t* sw = reinterpret_cast<const uint64_t*>(job.side ? arr.tmp : arr.recs) +
                         uint64_t(job.start) * RW;
    uint64_t* dw = reinterpret_cast<uint64_t*>(arr.recs) + uint64_t(job.start) * RW;

    // the job's keys, once, from HBM into LDS in input order
    for (uint32_t i = tid; i < m; i += kMidBlock) {
      uint64_t k[KW];
      key_of<KW>(gmem(sw) + uint64_t(i) * RW, P.kmask, k);
#pragma unroll
      for (int q = 0; q < KW; ++q) L.key[uint64_t(i) * KW + q] = k[q];
    }
    for (uint32_t q = tid; q < (m >> 5) + 2; q += kMidBlock) L.bm[q] = 0;
    if (tid == 0) {
      s_nbig = 0;
      s_nlist[0] = 0;
      s_nlist[1] = 0;
    }
    lds_barrier();
    if (m > tiny) {
      mid_first_split<RW, KW>(P, L, m, wave_cap);
    } else {
      for (uint32_t i = tid; i < m; i += kMidBlock) L.perm[i] = uint16_t(i);
      if (tid == 0) L.bm[0] = 1u;
      lds_barrier();
    }
    // ranges too large for one wave
    for (;;) {
      const uint32_t nbig = min(s_nbig, kMidBigCap);
      if (nbig == 0) break;
      const uint32_t e = s_big[nbig - 1];
      lds_barrier();
      if (tid == 0) s_nbig = nbig - 1;
      lds_barrier();
      mid_wg_pass<RW, KW>(P, L, e & 0xFFFFu, e >> 16, wave_cap);
    }
    // medium ranges: one wave each, round by round
    for (uint32_t cur = 0;; cur ^= 1) {
      const uint32_t nl = min(s_nlist[cur], kMidListCap);
      if (nl == 0) break;
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
        mid_wave_pass<RW, KW, WI>(P, L, e & 0xFFFFu, e >> 16, cur ^ 1, wave_cap);
      }
      lds_barrier();
      if (tid == 0) s_nlist[cur] = 0;
    }
    lds_barrier();

    // ---- tiny ranges: enumeration sort; everything else stays in place.
    // A range of at most tiny_max records belongs to the wave that owns the
    // 64-position window its first position falls in, so each wave reads,
    // ranks and rewrites only positions no other wave touches.
    const uint32_t wave = tid >> 6;
    const uint32_t nwin = (m + kWave - 1) / kWave;
    for (uint32_t k = wave; k < nwin; k += W) {
      const uint32_t w0 = k * kWave;
      uint32_t dst[kMidEsItems], slot[kMidEsItems];
      bool act[kMidEsItems];
#pragma unroll
      for (int h = 0; h < kMidEsItems; ++h) {
        const uint32_t p = w0 + h * kWave + lane;
        act[h] = false;
        dst[h] = p;
        slot[h] = 0;
        if (p >= m || uint32_t(h) * kWave > tiny + kWave) continue;
        const int lo = int(p) > int(tiny) ? int(p - tiny) : 0;
        const int s = bm_prev(L.bm, int(p), lo);
        if (s < int(w0) || s >= int(w0 + kWave)) continue;  // not a range of this window
        const int hi = min(s + int(tiny), int(m) - 1);
        int e = bm_next(L.bm, int(p), hi);
        if (e < 0 && s + int(tiny) >= int(m)) e = int(m);
        if (e < 0 || e - s < 2) continue;
        slot[h] = L.perm[p];
        uint64_t kp[KW];
        slot_key<RW, KW>(P, L, slot[h], kp);
        uint32_t r = 0;
        for (int q = s; q < e; ++q) {
          uint64_t kq[KW];
          slot_key<RW, KW>(P, L, L.perm[q], kq);
          r += (key_lt<KW>(kq, kp) || (q < int(p) && key_eq<KW>(kq, kp))) ? 1u : 0u;
        }
        dst[h] = uint32_t(s) + r;
        act[h] = true;
      }
      __builtin_amdgcn_wave_barrier();
      asm volatile("" ::: "memory");
#pragma unroll
      for (int h = 0; h < kMidEsItems; ++h)
        if (act[h]) L.perm[dst[h]] = uint16_t(slot[h]);
    }
    lds_barrier();
    // gather every record of the job (all loads complete before any store:
    // source and destination may be the same buffer), then write in order
    constexpr int WO = mid_items(RW, KW);
    uint64_t out[WO][RW];
#pragma unroll
    for (int u = 0; u < WO; ++u) {
      const uint32_t p = tid + u * kMidBlock;
      if (p < m) {
        uint32_t sl = L.perm[p];
        if (sl >= m) {  // never taken while the passes above keep perm a permutation
          atomicOr(&c->error, kErrBounds);
          sl = 0;
        }
        load_rec<RW>(reinterpret_cast<const uint8_t*>(sw), sl, out[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < WO; ++u) {
      const uint32_t p = tid + u * kMidBlock;
      if (p < m) store_rec<RW>(reinterpret_cast<uint8_t*>(dw), p, out[u], false);
    }
    lds_barrier();
  }
}

// ------------------------------------------------------------ copies

template <int RW>
__global__ void __launch_bounds__(256) k_copy(Params P) {
  Ctrl* c = P.L.ctrl;
  const uint32_t njobs = min(c->copy_count, P.L.cap_copy);
  for (uint32_t jb = blockIdx.x; jb < njobs; jb += gridDim.x) {
    const Bin job = P.L.copy[jb];
    const ArrayDesc arr = P.L.arrays[job.array];
    const RADULS_GLOBAL uint64_t* s =
        gmem(reinterpret_cast<const uint64_t*>(arr.tmp)) + uint64_t(job.start) * RW;
    RADULS_GLOBAL uint64_t* d = gmem(reinterpret_cast<uint64_t*>(arr.recs)) + uint64_t(job.start) * RW;
    const uint64_t words = uint64_t(job.size) * RW;
    if ((reinterpret_cast<uintptr_t>(s) & 15) == 0 && (reinterpret_cast<uintptr_t>(d) & 15) == 0) {
      const RADULS_GLOBAL u64x2* s2 = reinterpret_cast<const RADULS_GLOBAL u64x2*>(s);
      RADULS_GLOBAL u64x2* d2 = reinterpret_cast<RADULS_GLOBAL u64x2*>(d);
      for (uint64_t q = threadIdx.x; q < words / 2; q += 256) d2[q] = s2[q];
      if ((words & 1) && threadIdx.x == 0) d[words - 1] = s[words - 1];
    } else {
      for (uint64_t q = threadIdx.x; q < words; q += 256) d[q] = s[q];
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
    k_carry<<<1, 256, 0, s>>>(P, P.grid_hist);
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
  if (P.mode == kModeBatch) {
    k_zero_ctrl<<<1, 64, 0, s>>>(P);
    const uint32_t g = P.count ? (P.count + 255) / 256 : 1;
    k_seed_batch<<<g < 1024 ? g : 1024, 256, 0, s>>>(P);
  } else {
    k_seed_single<<<1, 64, 0, s>>>(P);
  }
  if (P.mode == kModeHist || P.mode == kModePartition) {
    k_prep<<<1, 1024, 0, s>>>(P, 0);
    k_hist<RW, KW, 1><<<P.grid_hist, kScatterBlock, 0, s>>>(P, 0);
    if (P.mode == kModePartition) launch_scatter<RW, KW, 1>(P, 0, s);
    k_step_out<<<1, 256, 0, s>>>(P);
    return hipGetLastError();
  }
  for (uint32_t r = 0; r < P.rounds; ++r) {
    const uint32_t cur = r & 1;
    const uint32_t slot = r == 0 ? kProfTopHist : kProfRoundHist;
    k_prep<<<1, 1024, 0, s>>>(P, cur);
    if (r <= 1) prof_mark(slot, 0, s);
    if (r == 0) k_hist<RW, KW, 1><<<P.grid_hist, kScatterBlock, 0, s>>>(P, cur);
    else k_hist<RW, KW, 0><<<P.grid_hist, kScatterBlock, 0, s>>>(P, cur);
    if (r <= 1) prof_mark(slot, 1, s);
    if (r <= 1) prof_mark(slot + 1, 0, s);
    if (r == 0) launch_scatter<RW, KW, 1>(P, cur, s);
    else launch_scatter<RW, KW, 0>(P, cur, s);
    if (r <= 1) prof_mark(slot + 1, 1, s);
    k_classify<KW><<<P.grid_classify, 256, 0, s>>>(P, cur);
  }
  prof_mark(kProfMid, 0, s);
  k_mid<RW, KW><<<P.grid_mid, kMidBlock, P.mid_lds_bytes, s>>>(P);
  prof_mark(kProfMid, 1, s);
  k_copy<RW><<<P.grid_copy, 256, 0, s>>>(P);
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

}  // namespace raduls
