// Shared host/device definitions of libraduls: workspace layout, bin and job
// descriptors, launch parameters.  Device code and host runtime both include
// this file; nothing here touches torch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace raduls {

// ---------------------------------------------------------------- constants

constexpr int kRadixBitsMax = 8;
constexpr int kRadix = 1 << kRadixBitsMax;  // buckets per digit (upper bound)
constexpr int kWave = 64;                   // CDNA wavefront width

// Scatter / histogram workgroups: 16 waves, one per CU.  Records per thread
// per tile are chosen per record width so that a tile stages up to about
// 100-130 KiB in LDS: big tiles give every digit long runs per tile.  For
// 32-byte records three per thread leave room for the line buffers below.
constexpr int kScatterBlock = 1024;
constexpr int kScatterWaves = kScatterBlock / kWave;
__host__ __device__ constexpr int scatter_items(int rw) {
  return rw == 1 ? 7 : rw == 2 ? 6 : rw == 3 ? 5 : rw == 4 ? 3 : rw == 5 ? 3 : 2;
}
// Records of 8, 16 and 32 bytes leave the carry-mode scatter through
// per-digit line buffers in LDS, so that every store but the first and last
// line of a digit's output in a workgroup's range covers whole 128-byte
// lines (longer records take too much LDS; 24, 40, 48 and 56 bytes do not
// divide a line).
__host__ __device__ constexpr bool scatter_lines(int rw) { return rw <= 2 || rw == 4; }
// Dynamic LDS of one scatter workgroup: the tile's records (input order) and
// a 16-bit permutation (or, for the look-back variant, the records in digit
// order and their digits), per-wave counters, three 256-entry tables, the
// per-digit global bases and, with line buffers, 128 bytes per digit plus
// three more per-digit tables.
__host__ __device__ constexpr uint32_t scatter_lds_bytes(int rw) {
  return uint32_t(kScatterBlock * scatter_items(rw)) * (8u * rw + 2u) +
         uint32_t(kScatterWaves * 256 * 2) + 3u * 256u * 4u + 256u * 8u +
         (scatter_lines(rw) ? 256u * 128u + 2u * 256u * 8u + 256u * 4u : 0u);
}

// LDS sorter workgroups: 16 waves, one workgroup per CU, which owns the
// CU's LDS.  Keys and a 16-bit permutation live in LDS; every thread holds
// the records of its slots in registers.
constexpr int kMidBlock = 1024;
constexpr int kMidWaves = kMidBlock / kWave;
constexpr uint32_t kLdsBytes = 160 * 1024;
constexpr uint32_t kMidStaticLds = 11 * 1024;  // static LDS of the LDS sorter (upper bound)
// Widest digit of a job's first pass; its counters are 16-bit, two per
// word (the words also hold the 256 counters of each wave in single-wave
// passes).
constexpr int kMidFirstBits = 13;
constexpr uint32_t kMidCounterWords = 1u << (kMidFirstBits - 1);
static_assert(kMidCounterWords >= uint32_t(kMidWaves) * 256u, "wave counters share the pass counters");
static_assert(kMidCounterWords % kMidBlock == 0, "counter scan splits evenly over the workgroup");
// Dynamic LDS for jobs of up to T records of rw words: the records (in input
// order), the permutation, the counters and two bitmaps.
__host__ __device__ constexpr uint32_t mid_dynamic_lds(uint32_t T, int rw) {
  return T * uint32_t(rw) * 8u + ((T + 1u) / 2u) * 4u + kMidCounterWords * 4u + 8u * ((T >> 5) + 2u);
}
// Records per lane of a whole job: while a job is sorted, every thread holds
// the next job's records of its slots in registers (at most 32 VGPRs).
__host__ __device__ constexpr uint32_t mid_lane_items(int rw) {
  return rw <= 2 ? 5u : 16u / uint32_t(rw);
}
// Largest job (records, a multiple of 64): its records fit the lanes'
// registers and its LDS state the CU's LDS.
__host__ __device__ constexpr uint32_t mid_cap(int rw, int kw) {
  (void)kw;
  uint32_t t = uint32_t(kMidBlock) * mid_lane_items(rw);
  while (t > 64u && mid_dynamic_lds(t, rw) + kMidStaticLds > kLdsBytes) t -= 64u;
  return t;
}
// Records per thread of a workgroup-wide LDS pass over a whole job.
__host__ __device__ constexpr int mid_items(int rw, int kw) {
  return int((mid_cap(rw, kw) + kMidBlock - 1) / kMidBlock);
}
// Records per lane of a single-wave LDS pass (a wave handles ranges of up to
// 64 * mid_wave_items records).
__host__ __device__ constexpr int mid_wave_items(int rw) { return rw <= 2 ? 8 : rw <= 4 ? 4 : 2; }
constexpr uint32_t kMidListCap = 384;   // ranges waiting for a wave pass (per round)
constexpr uint32_t kMidBigCap = 64;     // ranges waiting for a workgroup pass
// Positions per lane of the enumeration phase: a range of at most 256 records
// starting in a 64-position window ends within 5 windows.
constexpr int kMidEsItems = 5;
// Jobs of at most this many records (by default; tuning es_job_max) skip the
// first pass and are finished by one enumeration sort over the whole job;
// larger ones (even those below tiny_max) take the first pass, whose buckets
// make the enumeration cheaper.
constexpr uint32_t kMidDirectEs = 16;
// Jobs of at most kTinyJob records go to a separate list and are sorted by
// single waves in registers (k_tiny), not by a whole workgroup: up to 64
// records with one record per lane, up to 128 or 256 with two or four (four
// only for keys of at most two words and records of at most four, whose
// pairs and records still fit the registers).
constexpr uint32_t kTinyJob = 4 * kWave;
__host__ __device__ constexpr uint32_t tiny_job_max(int rw, int kw) {
  return kw <= 2 && rw <= 4 ? 4u * kWave : 2u * kWave;
}

// Most workgroups of the histogram / carry-scan scatter grid.
constexpr uint32_t kMaxRanges = 4096;

// Second-digit counts of the top-level histogram pass: 2^16 (top digit,
// second digit) pairs as 16-bit halves of 2^15 words per workgroup, and at
// most this many workgroups when they are taken.
constexpr uint32_t kPairWords = 1u << 15;
constexpr uint32_t kPairRanges = 512;

// Device error bits (raduls_stats.error).
constexpr uint32_t kErrCapacity = 1u << 0;
constexpr uint32_t kErrSpin = 1u << 1;
constexpr uint32_t kErrMidSize = 1u << 2;
constexpr uint32_t kErrBatchTotal = 1u << 3;
constexpr uint32_t kErrBounds = 1u << 4;

// Measurement slots of raduls_set_profile_events (event pairs).
constexpr uint32_t kProfTopHist = 0;    // top-level histogram
constexpr uint32_t kProfTopScatter = 1; // top-level scatter
constexpr uint32_t kProfRoundHist = 2;  // second round histogram
constexpr uint32_t kProfRoundScatter = 3;
constexpr uint32_t kProfMid = 4;        // LDS sorter
constexpr uint32_t kProfileSlots = 5;

// Look-back status word: [63:62] flag, [61:0] count.
constexpr uint64_t kFlagAggregate = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
// Earlier tiles read per look-back round trip.
constexpr int kLookback = 8;

// ---------------------------------------------------------------- descriptors

struct ArrayDesc {  // same layout as raduls_array
  uint8_t* recs;
  uint8_t* tmp;
  uint64_t n;
};

// Bin flags.  kBinEq: the next round splits the bin three ways on its
// equality key (keys below it, equal to it, above it) instead of on a digit.
// kBinRange: the bin is one side of such a split, a key range inside a run of
// records that share all key bits above `bits`, not the whole run.
constexpr uint8_t kBinEq = 1;
constexpr uint8_t kBinRange = 2;
// Bits 2-5: the width of the digit the next round splits the bin on, when
// narrower than digit_bits (0: digit_bits).  A bin a little larger than an
// LDS job is split on just enough bits that its children fit one job each,
// instead of on a full digit into children that must be packed many to a job.
constexpr uint32_t kBinWidthShift = 2;
constexpr uint8_t kBinWidthMask = 0x3C;
// Extra rounds that a sort of many records allows for equality splits (a
// split consumes a round but no key bit), and the samples that decide one.
constexpr uint32_t kEqRounds = 2;
constexpr uint32_t kEqSamples = 16, kEqDominant = 12;
// Records sampled (evenly spaced) to guess the root's highest differing key bit.
constexpr uint32_t kSpecSamples = 1024;

// A bin (a contiguous run of records that share all key bits above `bits`)
// or an LDS sort job / copy job over such runs.  16 bytes.
struct Bin {
  uint32_t start;  // first record, relative to the array
  uint32_t size;   // records
  uint32_t array;  // index into the array table
  uint16_t bits;   // key bits [0, bits) still to be sorted
  uint8_t side;    // 0: records currently in recs, 1: in tmp
  uint8_t flags;
};

// An LDS-sort job: a run of at most mid_max records, sorted from src into
// dst (the same address when the run already sits in the output buffer).
struct MidJob {
  uint8_t* src;
  uint8_t* dst;
  uint32_t size;
  uint32_t pad[3];
};
static_assert(sizeof(MidJob) == 32, "job descriptors are read as two 16-byte vectors");

// Device control block at the start of the auxiliary workspace; cleared at
// the start of every call.
struct Ctrl {
  uint32_t large_count[2];  // large-bin list sizes (ping-pong by round)
  uint32_t mid_count;      // LDS-sort jobs, including the copy jobs
  uint32_t copy_count;     // copy jobs (finished runs in tmp) among them
  uint32_t ticket;       // scatter tile tickets of the current round
  uint32_t round_tiles;  // tiles of the current round
  uint32_t error;
  uint32_t rounds;
  uint32_t large_bins;
  uint32_t scattered_bins;
  uint32_t mid_claim;  // LDS-sort jobs handed out beyond the first one per workgroup
  uint32_t fused;      // 1: this round's histograms came from the top-level pair counts
  uint32_t pair_rounds;  // rounds that did so
  uint32_t tiny_count;   // jobs in the tiny-job list
  uint32_t eq_bins;      // bins marked for an equality split
  unsigned long long moved_records;
  unsigned long long large_records;
  unsigned long long batch_total;
};

// ---- resident server: requests of at most mid_max records, each sorted in
// place by one workgroup of a kernel that stays resident until stopped.
// The submission ring lives in host-pinned memory: the host fills a slot and
// then publishes it by writing its sequence word; the device writes the
// slot's completion word once the request is sorted and visible.
constexpr uint32_t kServeMaxSlots = 1u << 20;
constexpr uint32_t kServeMaxIdleMs = 600000;     // 10 minutes
constexpr uint32_t kServeDefaultIdleMs = 10000;  // idle_ms = 0
constexpr uint32_t kServeMaxLeaseMs = 600000;    // 10 minutes
constexpr uint32_t kServeChunk = 8;              // most requests a workgroup claims at once

struct ServeSlot {
  uint64_t seq;     // host: ticket + 1 once recs and n are written
  uint64_t recs;    // device address of the request's [n, R] records
  uint64_t n;       // records (<= mid_max)
  uint64_t done;    // device: ticket + 1 once the sorted records are visible
  uint32_t status;  // device: error bits of the request (0: sorted)
  uint32_t pad[7];
};
static_assert(sizeof(ServeSlot) == 64, "one slot per 64-byte line");

struct ServeRing {
  uint64_t stop;      // host: non-zero asks every workgroup to exit
  uint64_t pad0[7];
  uint32_t reason;    // device: why the last workgroup to leave left (1 stop, 2 idle, 3 lease)
  uint32_t pad1[15];
  ServeSlot slot[1];  // [slots] (allocated past the struct's end)
};

// Device-memory state of a server.  Requests move from the host ring into a
// device queue (entry t % slots for ticket t) in batches of up to one wave's
// worth, read in parallel by the wave that holds the dispatch lock; `tail`
// counts the requests queued, `head` the ones claimed by workgroups.
struct ServeState {
  uint32_t lock;
  uint32_t pad;
  uint64_t head;
  uint64_t tail;
  uint64_t pad1[5];
};
struct ServeJob {
  uint64_t recs;
  uint64_t n;
};

// Device pointers into the auxiliary workspace.
struct Layout {
  Ctrl* ctrl;
  ArrayDesc* arrays;
  Bin* large[2];
  uint32_t* hist[2];      // [cap_large][kRadix]
  uint64_t* diff[2];      // [cap_large][8]
  uint64_t* eqkey[2];     // [cap_large][8] equality key of a kBinEq bin (masked key words)
  uint32_t* tile_prefix;  // [cap_large + 1]
  uint32_t* tile_bin;     // [cap_tiles]: bin index of each tile of the round
  uint64_t* status;       // [cap_tiles][kRadix] look-back status words
  uint32_t* wg_tail;      // [cap_ranges][kRadix] counts of each range's last bin segment
  uint32_t* wg_carry;     // [cap_ranges][kRadix] prefix carried into each range
  uint32_t* wg_flag;      // [cap_ranges] range starts a bin (1) / lies in one bin (2)
  MidJob* mid;
  MidJob* tiny;           // [cap_mid] jobs of at most kTinyJob records
  uint32_t* pair_part;    // [kPairRanges][kPairWords] per-range packed pair counts
  uint32_t* pair_hist;    // [2^16] pair counts of the whole array
  uint32_t* pair_d1;      // [kRadix] top digit of each second-round bin (when used)
  uint32_t cap_large, cap_tiles, cap_mid, cap_ranges;
};

enum Mode : uint32_t { kModeSort = 0, kModeBatch = 1, kModeHist = 2, kModePartition = 3 };

// Everything a launch sequence needs; passed to kernels by value.
struct Params {
  Layout L;
  uint32_t R, K;
  uint64_t kmask;         // mask of the key bytes in the top key word
  uint32_t digit_bits;    // 1..8
  uint32_t tiny_job;      // largest job of the wave-level sorter (<= tiny_job_max; 0: none)
  uint32_t es_job;        // LDS jobs of at most this many records: one enumeration sort
  uint32_t tiny_max;
  uint32_t mid_max;       // <= LDS capacity
  uint32_t tile;          // records per scatter tile
  uint32_t nontemporal;
  uint32_t lookback;      // 1: decoupled look-back scatter, 0: carry scan
  uint32_t pair;          // 1: the top-level histogram also counts digit pairs
  uint32_t spec;          // 1: the root's first split starts at the highest key bit in
                          // which sampled records differ (checked by round 0)
  uint32_t pair_min_bins; // fewest second-round bins that take the pair counts
  uint32_t rounds;         // rounds launched
  uint32_t round_budget;  // rounds a full sort launches (equality splits must fit in them)
  uint32_t eq_split;      // 1: classify may mark dominated bins for an equality split
  uint32_t inspect;       // 1: stop after the rounds (no LDS, tiny or copy kernels)
  uint32_t mode;
  uint32_t count;          // arrays
  uint64_t total_cap;      // batch: records the workspace was sized for
  // single array / step calls
  uint8_t* recs;
  uint8_t* tmp;
  uint64_t n;
  const ArrayDesc* d_arrays_in;  // batch descriptors (device)
  uint32_t step_bits, step_width;
  uint32_t* d_counts_out;
  uint32_t* d_offsets_out;
  // launch shapes
  uint32_t grid_hist, grid_scatter, grid_classify, grid_mid, grid_tiny;
  uint32_t mid_lds_bytes, scatter_lds_bytes;
  // resident server
  ServeRing* ring;          // device address of the host-pinned ring
  ServeState* serve;        // device memory
  Ctrl* serve_ctrl;         // [workgroups] error bits of each workgroup's request
  ServeJob* serve_queue;    // [serve_slots] requests moved from the ring
  uint32_t serve_slots;
  uint64_t serve_idle;      // ticks of the 100 MHz constant clock a workgroup waits idle
  uint64_t serve_lease;     // ticks a workgroup serves before it leaves (0: no limit)
};

__host__ __device__ inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace raduls
