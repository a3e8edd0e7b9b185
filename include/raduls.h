/*
 * raduls.h -- C ABI of libraduls.so, an MI355X (gfx950) MSD radix sort of
 * fixed-size records after RADULS2 (Kokot, Deorowicz, Dlugosz, "Even faster
 * sorting of (not only) integers", arXiv 1703.00687).
 *
 * Problem (paper: abstract, Sec. 3.1, Sec. 4.2).  An array holds n records of
 * R bytes each, stored contiguously (record i at byte offset i*R).  The key of
 * a record is its first K bytes read as an unsigned little-endian integer
 * (byte K-1 most significant; for K = 16 the word at offset 8 is the high
 * word).  Bytes at offsets K..R-1 are data: they travel with the record and
 * never affect the order.  Sorting permutes the records so that keys are
 * non-decreasing.  This library's result is also stable (records with equal
 * keys keep their input order), so it is unique.
 *
 * Method (Sec. 3): MSD radix sort on digits of `digit_bits` key bits (one
 * byte by default, as in the paper): per-bin digit histograms, exclusive
 * prefix scans into bucket offsets, a scatter of records into buckets, and
 * recursion into bins that are still large; small bins are finished inside one
 * workgroup's LDS, tiny buckets there by an enumeration sort, and bins of at
 * most 64 records by one wave with a bitonic sorting network (Sec. 2.2,
 * Sec. 3.3).
 *
 * Conventions for every call:
 *   - All calls are host calls.  Device work is enqueued on `stream` (0 = the
 *     null stream) and runs asynchronously; a call returns as soon as the work
 *     is enqueued.  The sort calls never allocate, free or synchronize, so
 *     they may be captured into a HIP graph.
 *   - Pointers named recs/tmp/src/dst/ws/d_* are DEVICE pointers owned by the
 *     caller, 16-byte aligned, valid until the enqueued work completes.
 *   - R (rec_bytes) must be a multiple of 8 in [8, 64]; K (key_bytes) in
 *     [1, R]; n < 2^32 per array.
 *   - Argument errors are returned synchronously, before anything is
 *     enqueued.  Errors found on the device (a workspace too small for the
 *     data, a bounded wait that expired) are recorded in the workspace and
 *     reported by raduls_check().
 */
#ifndef RADULS_H
#define RADULS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum raduls_status {
  RADULS_OK = 0,
  RADULS_E_INVALID = -1,     /* bad K, null pointer, overlapping buffers, bad digit */
  RADULS_E_ALIGN = -2,       /* a device pointer is not 16-byte aligned */
  RADULS_E_TMP_SMALL = -3,   /* tmp / ws smaller than the size query returned */
  RADULS_E_UNSUPPORTED = -4, /* R not a multiple of 8 in [8, 64], or n >= 2^32 */
  RADULS_E_HIP = -5,         /* a HIP runtime call or kernel launch failed */
  RADULS_E_DEVICE = -6,      /* raduls_check(): the device recorded an error */
  RADULS_E_SCRATCH = -7,     /* raduls_sort_static: n needs more than the static workspace */
  RADULS_E_BUSY = -8,        /* server: the ring slot of the next request is still in use */
  RADULS_E_STOPPED = -9,     /* server: its kernel has left (stopped or idle too long) */
  RADULS_E_TIMEOUT = -10     /* server: raduls_server_wait gave up */
} raduls_status;

/* Tuning knobs (process-global; set them before enqueuing sorts, never while
 * sorts are being enqueued from another thread).  Zero means "default".  The
 * result never depends on them, only the speed does. */
typedef struct raduls_tuning {
  uint32_t digit_bits;   /* radix digit width in bits, 1..8 (default 8: one byte, Sec. 3.1) */
  uint32_t tiny_max;     /* bins of <= tiny_max records are finished by enumeration
                            sort (Sec. 3.3); 1..256 (default 64) */
  uint32_t mid_max;      /* bins of <= mid_max records are sorted inside one workgroup's
                            LDS (the "small bin fits in cache" case, Sec. 3.2); clamped
                            to the LDS capacity for R; default = that capacity */
  uint32_t grid_blocks;  /* workgroups of the look-back scatter (lookback = 1; default
                            2 per CU); the other kernels size their grids themselves */
  uint32_t nontemporal;  /* 1: scatter stores use the nontemporal (streaming) cache
                            policy, 2: ordinary stores (default 1) */
  uint32_t lookback;     /* 0 (default): each scatter workgroup walks the contiguous tile
                            range of the histogram pass and starts from a carry computed
                            from the per-range counts; 1: tiles taken in ticket order get
                            their prefix by decoupled look-back over earlier tiles */
  uint32_t pair_hist;    /* raduls_sort with 8-bit digits on large inputs: 0 (default) or 1:
                            the top-level histogram pass also counts the second digit per
                            top digit, and when the second round's bins are many, of even
                            size and nowhere constant in that digit, the second round takes
                            its histograms from those counts instead of reading its bins
                            again (its scatter then gives each bin one workgroup); 2: never.
                            Costs 128 KiB of tmp per histogram workgroup (at most 64 MiB) */
  uint32_t wave_job_max; /* sort jobs (tiny bins, tiny arrays) of at most this many records are
                            sorted by one wave with a bitonic network (Sec. 3.3), larger ones by
                            a workgroup in LDS; 1 turns the wave sorter off; default and upper
                            bound 256 (128 for keys of more than 16 bytes or records of more
                            than 32) */
  uint32_t es_job_max;   /* LDS sort jobs of at most this many records skip the counting pass and
                            are finished by one enumeration sort (Sec. 2.2); 1..tiny_max
                            (default 16) */
  uint32_t tile_items;   /* records per thread of a histogram / scatter tile (a tile is 1024
                            times that); 1..8, clamped to the most the record width's LDS
                            staging holds, which is also the default (7, 6, 5, 4, 3, 2, 2, 2
                            for R = 8 .. 64) */
  uint32_t reserved[6];
} raduls_tuning;

/* Device-side counters left in the workspace by the last sort that used it. */
typedef struct raduls_stats {
  uint32_t error;          /* bit 0: list capacity exceeded; bit 1: bounded look-back
                              wait expired; bit 2: a bin larger than mid_max reached the
                              LDS sorter; bit 3: batch total exceeded its capacity;
                              bit 4: a destination fell outside its bin, or the LDS
                              sorter's permutation named a record outside its job
                              (write suppressed) */
  uint32_t rounds;         /* radix rounds that found at least one large bin */
  uint32_t large_bins;     /* large bins processed over all rounds */
  uint32_t scattered_bins; /* large bins that were moved (not constant / all equal) */
  uint32_t mid_jobs;       /* bins finished by a final sort job: in one workgroup's LDS,
                              or (at most 64 records) by one wave in registers */
  uint32_t copy_jobs;      /* tmp -> recs copies of finished runs (pieces of at most
                              mid_max records, taken by the LDS sorter) */
  uint64_t moved_records;  /* records moved by global scatter passes */
  uint64_t large_records;  /* records in large bins, summed over rounds */
  uint32_t pair_rounds;    /* 1 if the second round took its histograms from the
                              top-level digit pair counts (tuning pair_hist) */
  uint32_t eq_bins;        /* large bins that one key dominated, split three ways on it
                              (keys below, equal to, above it) instead of on a digit */
} raduls_stats;

/* Bytes of `tmp` that raduls_sort needs for n records: n*R for the scatter
 * ping-pong plus an auxiliary workspace (bin lists, look-back status, job
 * queues) placed after them.  Depends on the current tuning. */
int raduls_tmp_bytes(uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, uint64_t *out_bytes);

/* Sort n records in `recs` by their key (the whole method of Sec. 3).
 * recs: n*R bytes, in/out.  tmp: at least raduls_tmp_bytes() bytes of
 * scratch whose contents on return are undefined; it must not overlap recs.
 * n <= 1 is a no-op.  On completion of the enqueued work `recs` holds the
 * stably sorted records. */
int raduls_sort(void *recs, void *tmp, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                hipStream_t stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture that must not allocate, tight serving loops, harnesses that forbid
 * hipMalloc: raduls_sort with its auxiliary workspace (bin lists, histograms,
 * job queues) in a static device array of 64 MiB that the library holds on
 * every GPU it runs on until the process ends, instead of the tail of tmp.
 * tmp needs only n*R bytes.  Allocates and frees nothing.  The top-level
 * digit-pair counts (tuning pair_hist) are never used here.  Returns
 * RADULS_E_SCRATCH when the workspace for n records does not fit the array
 * (with 16-byte records and default tuning about 5.8e7 records fit).  Every
 * call on one GPU uses that GPU's one array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads)
 * race and must be serialized by the caller.  raduls_check(tmp, ...) does
 * not apply to these calls (the counters are not in tmp). */
int raduls_sort_static(void *recs, void *tmp, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                       hipStream_t stream);

/* A bin of the recursion: records [start, start + size) of the array that
 * share every key bit from `bits` up (bits 0 .. bits-1 are still to be
 * sorted); they sit in recs (side 0) or in the ping-pong half of tmp (side 1)
 * at the same offsets.  flags bit 0: the next round splits the bin on one key
 * that dominates it (keys below, equal to, above it); bit 1: the bin is one
 * side of such a split, a key range inside a run of records sharing the bits
 * from `bits` up rather than the whole run; bits 2-5: when non-zero, the
 * width of the digit the next round splits the bin on (narrower than the
 * tuning's digit width: the bin is split into children of about one LDS job
 * each). */
typedef struct raduls_bin {
  uint32_t start;
  uint32_t size;
  uint32_t bits;
  uint32_t side;
  uint32_t flags;
} raduls_bin;

/* Recursion inspection (Sec. 1: after each radix phase the array is split
 * into bins that are processed independently; Sec. 3.1-3.2: bins larger
 * than the LDS capacity get another global pass).  Runs the first `rounds`
 * (>= 1) global rounds of raduls_sort on recs (tmp as for raduls_sort) and
 * none of the later stages, then SYNCHRONIZES the stream and writes to the
 * HOST array `bins` (room for `cap` entries) the bins larger than mid_max
 * that those rounds left for the next round, in list order; *count receives
 * their number (which may exceed cap).  Afterwards the records are stably
 * partitioned into bins, each on the side its entry names; neither buffer
 * holds the sorted result.  For tests and diagnosis; n <= mid_max runs no
 * round and returns *count = 0.  Returns RADULS_E_DEVICE if the device
 * recorded an error. */
int raduls_inspect_rounds(void *recs, void *tmp, uint64_t n, uint32_t rec_bytes,
                          uint32_t key_bytes, uint32_t rounds, raduls_bin *bins, uint32_t cap,
                          uint32_t *count, hipStream_t stream);

/* One array of a batch: device pointers recs (n*R bytes) and tmp (at least
 * n*R bytes; no auxiliary tail needed), and its record count. */
typedef struct raduls_array {
  void *recs;
  void *tmp;
  uint64_t n;
} raduls_array;

/* Workspace bytes for raduls_sort_batch with `count` arrays holding at most
 * `total_n` records together. */
int raduls_batch_ws_bytes(uint32_t count, uint64_t total_n, uint32_t rec_bytes,
                          uint32_t key_bytes, uint64_t *out_bytes);

/* Sort `count` independent arrays in one set of launches.  d_arrays is a
 * DEVICE array of `count` raduls_array descriptors (it may be rewritten
 * between replays of a captured graph).  The sum of their n must not exceed
 * total_n, the capacity ws was sized for (checked on the device; see
 * raduls_check).  Every array is sorted as raduls_sort would sort it.  The
 * launch shapes depend only on (count, total_n, R, K) and the tuning, never on
 * the array contents, so one captured graph serves any batch within them. */
int raduls_sort_batch(const raduls_array *d_arrays, uint32_t count, uint64_t total_n,
                      uint32_t rec_bytes, uint32_t key_bytes, void *ws, uint64_t ws_bytes,
                      hipStream_t stream);

/* Workspace bytes for raduls_histogram / raduls_partition on n records. */
int raduls_step_ws_bytes(uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, uint64_t *out_bytes);

/* Digit histogram of one bin, the whole array (Sec. 1: counting step of a
 * radix phase).  The digit is key bits [bits - w, bits), w = min(width, bits),
 * 1 <= width <= 8, 1 <= bits <= 8K.  d_counts: DEVICE uint32[2^w], written. */
int raduls_histogram(const void *recs, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                     uint32_t bits, uint32_t width, uint32_t *d_counts, void *ws,
                     uint64_t ws_bytes, hipStream_t stream);

/* One stable counting-sort pass of the whole array on one digit (Sec. 1;
 * the scatter of Sec. 3.2): src -> dst, records grouped by digit in
 * increasing digit order, input order kept inside each group.  d_offsets
 * (DEVICE uint32[2^w], may be NULL) receives the exclusive prefix sum of the
 * digit counts, i.e. where each bucket starts in dst.  src and dst must not
 * overlap. */
int raduls_partition(const void *src, void *dst, uint64_t n, uint32_t rec_bytes,
                     uint32_t key_bytes, uint32_t bits, uint32_t width, uint32_t *d_offsets,
                     void *ws, uint64_t ws_bytes, hipStream_t stream);

/* Synchronously read the device counters of the last call that used this
 * workspace: for raduls_sort pass (tmp, n, R, 0); for raduls_sort_batch,
 * raduls_histogram and raduls_partition pass (ws, 0, R, 1).  Waits for
 * `stream` first.  Returns RADULS_OK, or RADULS_E_DEVICE if stats->error is
 * non-zero. */
int raduls_check(const void *tmp_or_ws, uint64_t n, uint32_t rec_bytes, int ws_only,
                 raduls_stats *stats, hipStream_t stream);

int raduls_set_tuning(const raduls_tuning *tuning);
int raduls_get_tuning(raduls_tuning *tuning);

/* Measurement aid.  With count > 0, later sort calls record events[2i] and
 * events[2i+1] (caller-created HIP events) on their stream just before and
 * after the launches of kernel class i: 0 top-level histogram, 1 top-level
 * scatter, 2 second-round histogram, 3 second-round scatter, 4 LDS sorter.
 * count = 0 turns it off.  Process-global; never set while sorts are being
 * enqueued or captured. */
int raduls_set_profile_events(hipEvent_t *events, uint32_t count);

/* Largest mid_max (records) the LDS sorter supports for records of R bytes
 * with K key bytes (0 for an unsupported shape). */
uint32_t raduls_mid_capacity(uint32_t rec_bytes, uint32_t key_bytes);

/* ---- Resident server: small arrays sorted without a launch per request.
 *
 * Paper: Sec. 3.2 sorts a small bin with one thread in the processor's cache
 * and Sec. 3.3 tiny bins in registers; a request of at most
 * raduls_server_max_records records is that case as a whole: one workgroup
 * sorts it in LDS.  raduls_server_create launches `workgroups` workgroups
 * of the LDS sorter (0: an eighth of the CUs) that stay resident on a stream
 * of the server's own and take requests from a submission ring of `slots`
 * entries in host-pinned memory: the host writes a request and publishes it;
 * the first free workgroup claims it, sorts it in place (stable, the same
 * result as raduls_sort) and publishes its completion.  The workgroups
 * occupy their CUs while the server lives; the other CUs stay free for other
 * work.
 *
 * Ownership and contracts:
 *   - create allocates the ring (pinned host memory), a small device state
 *     and the stream; destroy frees them.  No other server call allocates.
 *   - submit: `recs` is a device pointer to n <= max_records records of the
 *     server's R and K, written and visible on the device before the call
 *     (e.g. its producer's stream synchronized); the caller keeps it alive
 *     and does not touch it until the request completes.  It returns at once
 *     with a ticket (0, 1, 2, ... in submission order).  RADULS_E_BUSY: the
 *     ring slot the request needs still holds an uncompleted request from
 *     `slots` submissions ago (retry after a completion);
 *     RADULS_E_UNSUPPORTED: n > max_records; RADULS_E_STOPPED: the kernel
 *     could not be relaunched (destroyed, or the launch failed).  Calls
 *     are serialized.
 *   - poll returns 1 once the request's sorted records are visible to the
 *     host and to work enqueued afterwards (*status: 0, or the device's
 *     error bits), 0 while pending, RADULS_E_STOPPED if the kernel was
 *     stopped (or could not be relaunched) before completing it.  Poll a ticket before `slots` later submissions
 *     reuse its slot, or its status reads 0.  wait polls until done or
 *     `timeout_ms` (then RADULS_E_TIMEOUT).
 *   - Every wait of the kernel is bounded: a workgroup leaves when destroy
 *     sets the ring's stop word, or after `idle_ms` (0: 10 s; at most 10
 *     minutes) without a request, or, with `lease_ms` > 0 (at most 10
 *     minutes), before its next claim once it has run that long, requests
 *     queued or not.  A kernel that left idle or by its lease is relaunched
 *     (same stream, ring and state) by the next submit, or by a poll /
 *     completed / wait that finds requests pending: requests queued when it
 *     left progress only while the host makes such calls.  Only destroy's
 *     stop is final (info: running, reason 1 stopped / 2 idle / 3 lease).
 *   - The kernel holds its stream's hardware queue while it runs.  When a
 *     process has more streams than the device's hardware queues (HIP maps
 *     streams onto a few queues per device; a PyTorch program that creates
 *     one stream of its pool has dozens), streams share queues, and work on
 *     a stream that shares the server's queue waits until the kernel leaves.
 *     Such programs set a short lease (and idle time), which bounds that
 *     wait.  A device-wide synchronize also waits for the kernel.
 *   - destroy stops the kernel (requests being sorted finish; queued ones
 *     are not started), waits for it to leave and frees everything. */
typedef struct raduls_server raduls_server;
int raduls_server_max_records(uint32_t rec_bytes, uint32_t key_bytes, uint64_t *out_records);
int raduls_server_create(uint32_t rec_bytes, uint32_t key_bytes, uint32_t slots,
                         uint32_t workgroups, uint32_t idle_ms, uint32_t lease_ms,
                         raduls_server **out);
int raduls_server_submit(raduls_server *srv, void *recs, uint64_t n, uint64_t *ticket);
/* submit_many: requests recs[i] of n[i] records, i < count, in order, with
 * tickets *first_ticket, *first_ticket + 1, ...; stops early (without error)
 * at the first request whose ring slot is still in use and reports in
 * *accepted how many were submitted.  Arguments are checked for all of them
 * before any is submitted. */
int raduls_server_submit_many(raduls_server *srv, void *const *recs, const uint64_t *n,
                              uint32_t count, uint64_t *first_ticket, uint32_t *accepted);
int raduls_server_poll(raduls_server *srv, uint64_t ticket, uint32_t *status);
int raduls_server_wait(raduls_server *srv, uint64_t ticket, uint32_t timeout_ms, uint32_t *status);
/* wait_range: waits for tickets [first, first + count) (all submitted);
 * *status_or is the OR of their status words.  RADULS_OK, RADULS_E_TIMEOUT,
 * RADULS_E_STOPPED or RADULS_E_INVALID. */
int raduls_server_wait_range(raduls_server *srv, uint64_t first, uint64_t count,
                             uint32_t timeout_ms, uint32_t *status_or);
/* completed: *through = the number of leading tickets that have all
 * completed (every ticket below it is done), advanced from where the last
 * call left it; *status_or = the OR of the status words of the tickets this
 * call newly found done (so that a caller polling many requests needs one
 * call, and `poll` only to find which of them failed).  RADULS_E_STOPPED if
 * tickets are pending and the kernel was stopped or could not be
 * relaunched. */
int raduls_server_completed(raduls_server *srv, uint64_t *through, uint32_t *status_or);
int raduls_server_info(raduls_server *srv, uint64_t *max_records, uint32_t *workgroups,
                       uint32_t *running, uint32_t *reason);
int raduls_server_destroy(raduls_server *srv);

const char *raduls_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* RADULS_H */
