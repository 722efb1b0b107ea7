/* hive.h -- C ABI of an MI355X (gfx950) implementation of the Hive hash table
 * (Polak, Troendle, Jang, "Hive Hash Table: A Warp-Cooperative, Dynamically
 * Resizable Hash Table for GPUs", arXiv 2510.15095).
 *
 * The table maps 32-bit keys to 32-bit values.  Each entry is one 64-bit word,
 * value in the high half and key in the low half (Section III-A), stored in
 * buckets of S slots (Section III-B).  Keys 0 and 0xFFFFFFFF are reserved:
 * operations on them are no-ops that report "absent" and are counted in
 * hive_stats_t.invalid_keys.
 *
 * Conventions for every call below:
 *   - Pointers named d_* are device memory owned by the caller.  They must
 *     stay valid until the stream reaches the call.  The table owns all of its
 *     own memory (buckets, stash, pending list, worklists, scratch).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Batch calls only enqueue work and return; hive_create, hive_stats,
 *     hive_dump and hive_destroy synchronize the stream.
 *   - One handle must not be used from two host threads, or from two streams
 *     that are not ordered with each other, at the same time.  Different
 *     handles are independent.
 *   - Argument errors are returned at once (negative status) and nothing is
 *     enqueued.  Conditions found on the device (a full pending list, reserved
 *     keys) are latched and returned by the next hive_stats call.
 *   - A batch call is applied as if its operations ran one at a time in index
 *     order, provided the caller keeps the contract stated at each call.
 */
#ifndef HIVE_H
#define HIVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hive_table *hive_t;

typedef enum {
  HIVE_OK = 0,
  HIVE_ERR_ARG = -1,      /* invalid argument; nothing was enqueued */
  HIVE_ERR_OOM = -2,      /* device allocation failed */
  HIVE_ERR_HIP = -3,      /* a HIP runtime call failed */
  HIVE_ERR_BUDGET = -4,   /* the bucket arena or a fixed capacity is exhausted */
  HIVE_ERR_LOST = -5,     /* the pending list overflowed: entries were lost */
  HIVE_WARN_INVALID_KEYS = 1, /* reserved keys were seen (they were no-ops) */
  HIVE_WARN_PENDING = 2       /* entries wait in the pending list (data intact) */
} hive_status;

/* Bucket addressing.  FIXED reduces the mixed hash modulo the bucket count,
 * as the BitHash listing does (Section III-C); LINEAR uses the linear-hashing
 * index mask and split pointer (Section IV-C) and allows hive_resize. */
enum { HIVE_FIXED = 0, HIVE_LINEAR = 1 };

/* Flags for batch calls. */
enum {
  HIVE_UNIQUE = 1u /* caller promises no key repeats among the batch's inserts
                      and none among its deletes: skips the dedupe pass */
};

/* Op codes for hive_mixed_batch; HIVE_OP_MIXED marks a batch descriptor
 * whose per-operation codes are in d_ops. */
enum { HIVE_OP_INSERT = 0, HIVE_OP_DELETE = 1, HIVE_OP_LOOKUP = 2, HIVE_OP_MIXED = 3 };

typedef struct {
  uint32_t slots_per_bucket;  /* S: 16 (one 128-byte line) or 64 */
  uint32_t max_evictions;     /* bound on cuckoo displacements per insert
                                 (Section III-B "Global Metadata"); default 8 */
  uint64_t stash_capacity;    /* overflow stash entries (Section IV-A step 4);
                                 0 = max(1024, 1% of the slots of max_buckets).
                                 Held as an open-addressed table of at least
                                 twice as many words, so a search probes a
                                 short run instead of scanning */
  uint64_t pending_capacity;  /* entries beyond a full stash; 0 = stash_capacity */
  uint32_t addressing;        /* HIVE_FIXED or HIVE_LINEAR */
  uint32_t resize_k;          /* K: bucket pairs per split/merge step (Section
                                 IV-C); default 1024 */
  uint32_t lf_expand_pct;     /* expand when live > pct% of slots; default 90 */
  uint32_t lf_contract_pct;   /* contract when live < pct% of slots; default 25 */
  uint32_t pre_expand;        /* 1: before each insert batch of n inserts, grow
                                 until live + n fits under lf_expand_pct */
  uint32_t post_policy;       /* 1: after each batch apply the expand/contract
                                 rule (LINEAR tables) */
  uint64_t max_buckets;       /* bucket arena reserved at create (LINEAR:
                                 growth headroom; 0 = initial buckets) */
  uint64_t max_batch;         /* scratch preallocated for batches of this many
                                 operations (0 = grow on demand).  LINEAR
                                 tables with post_policy also hold a full
                                 stash drain beside a batch's eviction
                                 worklist: a batch with inserts is evicted
                                 once, after the post-batch rule */
  uint32_t probe_both;        /* S = 16: 1 = lookups and deletes load both
                                 candidate buckets in one round (one memory
                                 round trip fewer, more bytes); inserts always
                                 do.  0 = second bucket only after a miss.
                                 Plain launches only: the persistent
                                 executor always uses 0.  Results are the
                                 same either way */
  uint32_t hash_pair;         /* candidate-bucket hashes: HIVE_PAIR_BITHASH
                                 (BitHash1/2, Section III-C; the default),
                                 HIVE_PAIR_CRC (CRC-32, low half of CRC-64;
                                 tables in constant memory) or
                                 HIVE_PAIR_MURMUR (MurmurHash3, CityHash32),
                                 the hashes of the study below, or
                                 HIVE_PAIR_TRIPLE: three candidate buckets
                                 (BitHash1, BitHash2, CityHash32; lookups
                                 probe them in that order, inserts take the
                                 emptiest, ties to the lower hash, and an
                                 evicted entry moves to its next candidate in
                                 that order, cyclically).  The others
                                 need S = 16, FIXED addressing, probe_both = 0,
                                 plain launches (the executor and
                                 hive_placement refuse such tables) */
  uint32_t entry_bits;        /* 64 (or 0, the default): 32-bit keys with
                                 32-bit values packed in 64-bit words.  32: a
                                 key-only set of 32-bit entries (Section
                                 III-A), a 32-slot bucket being one 128-byte
                                 line; needs slots_per_bucket = 32, FIXED
                                 addressing, HIVE_PAIR_BITHASH, probe_both 0
                                 and plain launches.  Insert adds the key (a
                                 key already present is left as it is; d_vals
                                 is not read), lookup writes found flags (no
                                 values), delete as for 64-bit entries;
                                 hive_dump writes each key as a word with
                                 value 0 */
  uint32_t probe_tuning;      /* probe-kernel variant per operation kind,
                                 four bits each: bits 0-3 insert batches,
                                 4-7 delete, 8-11 lookup, 12-15 mixed.  A
                                 variant sets the occupancy target (waves
                                 per SIMD) and the bucket loads in flight
                                 per wave and probe chunk: 0 (default) 4 and
                                 16; 1: 6 and 16; 2: 8 and 8; 3: 6 and 8;
                                 4: 8 and 4.  Inserts take 0, 3 or 4 (their
                                 fused round holds twice the loads).
                                 Non-zero needs S = 16, HIVE_PAIR_BITHASH,
                                 probe_both 0 and 64-bit entries; results
                                 are the same for every variant.  Picked by
                                 measurement (the package's autotuner);
                                 HIVE_ERR_ARG for anything else */
  uint32_t probe_grid;        /* most blocks of 256 operations one probe
                                 launch starts; each block strides over the
                                 batch's tiles (0 = 32768, at most 2^20) */
} hive_config;

enum { HIVE_PAIR_BITHASH = 0, HIVE_PAIR_CRC = 1, HIVE_PAIR_MURMUR = 2, HIVE_PAIR_TRIPLE = 3 };

typedef struct {
  uint64_t live;            /* number of keys stored */
  uint64_t n_buckets;       /* current bucket count */
  uint64_t index_mask;      /* LINEAR: 2^m - 1 of the current round */
  uint64_t split_ptr;       /* LINEAR: buckets of this round already split */
  uint64_t stash_count;     /* stash entries in use (incl. deleted ones) */
  uint64_t pending_count;   /* pending entries in use (incl. deleted ones) */
  uint64_t evictions;       /* cuckoo displacements (Section IV-A step 3) */
  uint64_t stash_inserts;   /* entries that entered the stash */
  uint64_t pending_inserts; /* entries that entered the pending list */
  uint64_t full_chains;     /* inserts whose eviction chain ran all rounds */
  uint64_t invalid_keys;    /* operations on reserved keys */
  uint64_t evict_items;     /* inserts that needed step 3 (worklist items) */
  uint64_t bytes_reserved;  /* device bytes owned by the table */
  uint64_t slots_per_bucket;
  uint64_t max_buckets;
  uint64_t error_bits;      /* latched device conditions */
} hive_stats_t;

/* Fill *cfg with the defaults named above (S = 16, FIXED addressing). */
hive_status hive_config_default(hive_config *cfg);

/* Create a table with `initial_buckets` empty buckets (Section III-B).
 * LINEAR tables reserve max(cfg->max_buckets, initial_buckets) buckets of
 * arena up front, so growth never allocates.  Synchronizes `stream`. */
hive_status hive_create(const hive_config *cfg, uint64_t initial_buckets, void *stream, hive_t *out);

/* Synchronize the table's last stream and free everything it owns. */
hive_status hive_destroy(hive_t h);

/* Insert-or-replace n pairs (Section III-D Insert and Replace; the four-step
 * insert of Section IV-A).  d_keys, d_vals: n uint32 each.  Repeated keys:
 * the last occurrence wins, unless `flags` has HIVE_UNIQUE (then repeats are
 * the caller's error and their outcome is unspecified). */
hive_status hive_insert_batch(hive_t h, const uint32_t *d_keys, const uint32_t *d_vals, uint64_t n,
                              uint32_t flags, void *stream);

/* Search n keys (Section III-D Search; Section IV-B).  d_vals_out[i] gets
 * the value or 0xFFFFFFFF, d_found_out[i] 1 or 0.  Either output may be
 * NULL. */
hive_status hive_lookup_batch(hive_t h, const uint32_t *d_keys, uint64_t n, uint32_t *d_vals_out,
                              uint8_t *d_found_out, void *stream);

/* Delete n keys (Section III-D Delete; Algorithm 4).  d_deleted_out[i] (may
 * be NULL) is 1 when the key was present at that point of the batch; with
 * repeats, the first occurrence reports the deletion. */
hive_status hive_delete_batch(hive_t h, const uint32_t *d_keys, uint64_t n, uint32_t flags,
                              uint8_t *d_deleted_out, void *stream);

/* A batch of mixed operations (the paper's concurrent mix, Section V-C-2).
 * d_ops[i] is HIVE_OP_INSERT/DELETE/LOOKUP.  Contract: within one call the
 * keys of inserts, of deletes and of lookups form disjoint sets (a key may
 * repeat within one type).  Outputs, per operation: lookups write the value
 * (or 0xFFFFFFFF) and found; deletes write 0xFFFFFFFF and the deleted flag;
 * inserts write 0xFFFFFFFF and 0.  d_vals may be NULL when there are no
 * inserts; outputs may be NULL. */
hive_status hive_mixed_batch(hive_t h, const uint8_t *d_ops, const uint32_t *d_keys, const uint32_t *d_vals,
                             uint64_t n, uint32_t flags, uint32_t *d_vals_out, uint8_t *d_flags_out,
                             void *stream);

/* hive_mixed_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operation, outputs and contract, with no hipMalloc,
 * hipFree or other allocating call.  The batch's dedupe set (needed unless
 * `flags` has HIVE_UNIQUE) lives in a 128 MiB array of device memory that the
 * library holds on each GPU it runs on until the process ends, so with
 * dedupe a call takes at most 2^22 operations; the eviction worklist is the
 * table's own, preallocated at create, so n may not exceed
 * max(hive_config.max_batch, the table's stash + pending capacity).  Beyond
 * either limit the call returns HIVE_ERR_BUDGET (with a line on stderr) and
 * enqueues nothing.  Every call on one GPU shares that GPU's array: calls
 * whose work overlaps on the device (other streams, other host threads, other
 * tables) race on it and must be ordered by the caller.  Phase timing
 * (hive_phase_timing) is not recorded for these calls. */
hive_status hive_mixed_batch_noalloc(hive_t h, const uint8_t *d_ops, const uint32_t *d_keys,
                                     const uint32_t *d_vals, uint64_t n, uint32_t flags, uint32_t *d_vals_out,
                                     uint8_t *d_flags_out, void *stream);

/* Linear-hashing resize (Section IV-C), LINEAR tables only.
 * delta > 0: split up to delta buckets, K at a time (Section IV-C-1), then
 * re-insert the stash and pending entries; delta < 0: merge up to -delta
 * pairs from the top down, stopping at the first pair whose entries do not
 * fit (Section IV-C-2); delta == 0: apply the load-factor rule.  The
 * decisions are taken on the device; the call does not synchronize. */
hive_status hive_resize(hive_t h, int64_t delta, void *stream);

/* Copy counters and geometry to *out (synchronizes `stream`) and return the
 * latched device condition, if any: HIVE_ERR_LOST, HIVE_ERR_BUDGET,
 * HIVE_WARN_PENDING or HIVE_WARN_INVALID_KEYS, else HIVE_OK. */
hive_status hive_stats(hive_t h, hive_stats_t *out, void *stream);

/* Write every live entry to d_words (packed words) and its place to d_where
 * (bucket index, -1 for the stash, -2 for the pending list; may be NULL),
 * in no particular order, at most `capacity` of them; *n_out gets the number
 * of live entries.  Synchronizes `stream`. */
hive_status hive_dump(hive_t h, uint64_t *d_words, int64_t *d_where, uint64_t capacity, uint64_t *n_out,
                      void *stream);

/* Placement census: out[0] = live bucket entries in their first candidate
 * bucket, out[1] = in their second (different) candidate, out[2] = stash and
 * pending slots in use (including deleted ones).  With two-choice placement
 * a successful lookup touches one bucket for out[0] entries and two for
 * out[1] entries.  Synchronizes `stream`. */
hive_status hive_placement(hive_t h, uint64_t *out, void *stream);

/* Enqueue a copy of the table's key count into *host_dst (pinned host
 * memory) on `stream`, after the work already on it; no synchronization. */
hive_status hive_live_async(hive_t h, uint64_t *host_dst, void *stream);

/* Empty the table and restore its initial geometry (stream-ordered). */
hive_status hive_clear(hive_t h, void *stream);

/* A short English description of a status code (static storage). */
const char *hive_status_string(hive_status s);

/* ---- Phase timing (a measurement aid; off by default) --------------------
 * While enabled, every batch call records HIP events on its stream at the
 * boundaries of its phase groups (Section IV-A's insert steps map onto
 * them: steps 1 and 2 run in the probe launch, step 3 in the eviction
 * launch and step 4 in a launch of its own, which exists only while timing
 * is on; without timing the eviction launch also places the stash
 * entries).  hive_phase_times waits for the recorded events and
 * writes, per group, the milliseconds spent since the previous
 * hive_phase_times call, then starts over: ms_out is a caller-owned host
 * array of HIVE_PHASE_KINDS doubles.  The events are ordered on each call's
 * own stream only.  HIVE_ERR_HIP if waiting for the events failed. */
enum {
  HIVE_PHASE_DEDUPE = 0,  /* dedupe of the batch's repeated keys (by hash
                             partitions: collect, sums, scan, scatter, resolve) */
  HIVE_PHASE_PROBE = 1,   /* probe launch: replace, claim (steps 1-2), lookup, delete */
  HIVE_PHASE_EVICT = 2,   /* eviction chains (step 3); with 16-slot buckets and
                             the BitHash pair, step 4 is timed apart below,
                             otherwise it is included here */
  HIVE_PHASE_RESIZE = 3,  /* load-factor plans and split/merge passes */
  HIVE_PHASE_DRAIN = 4,   /* stash drain after splits and its re-placement */
  HIVE_PHASE_FINISH = 5,  /* counter folds after a batch */
  HIVE_PHASE_STASH = 6,   /* stash or pending placement of entries whose chain ran
                             out (step 4; 16-slot BitHash tables) */
  HIVE_PHASE_KINDS = 7
};
hive_status hive_phase_timing(hive_t h, int enable);
hive_status hive_phase_times(hive_t h, double *ms_out);

/* ---- Hash-function study (Section III-C) ----------------------------------
 * The spread of BitHash1/2 and of widely used hashes over m buckets.  Each
 * hash reads a key as its four little-endian bytes; a key's bucket is the
 * hash modulo m (all 64 bits for CRC-64):
 *   HIVE_HASH_CRC32    reflected 0xEDB88320, all-ones init and final xor;
 *   HIVE_HASH_CRC64    reflected 0xC96C5795D7870F42 (ECMA-182, as in xz),
 *                      all-ones init and final xor;
 *   HIVE_HASH_MURMUR3  MurmurHash3, x86 32-bit variant, seed 0;
 *   HIVE_HASH_CITY32   CityHash32 (its path for inputs of at most 4 bytes).
 * The CRCs are table-driven (tables in LDS), the others ALU only. */
enum {
  HIVE_HASH_BITHASH1 = 0,
  HIVE_HASH_BITHASH2 = 1,
  HIVE_HASH_CRC32 = 2,
  HIVE_HASH_CRC64 = 3,
  HIVE_HASH_MURMUR3 = 4,
  HIVE_HASH_CITY32 = 5,
  HIVE_HASH_KINDS = 6
};

/* d_out[i] = bucket of d_keys[i] under hash `kind` (device arrays of n
 * entries, caller-owned), stream-ordered, no synchronization.  HIVE_ERR_ARG
 * for an unknown kind, m = 0 or m > 2^32, or a null array with n > 0. */
hive_status hive_hash_buckets(uint32_t kind, const uint32_t *d_keys, uint64_t n, uint64_t m, uint32_t *d_out,
                              void *stream);

/* *y_out = sum over the m buckets of (load - 1)+ for the n keys of d_keys
 * under hash `kind`, the collision count Y of the uniform-hashing theorem
 * (Section III-C; equal to n minus the number of occupied buckets).
 * d_scratch: caller-owned device memory of at least 2 + ceil(m / 32) 32-bit
 * words, overwritten.  Synchronizes `stream`.  HIVE_ERR_ARG as for
 * hive_hash_buckets, or for a null d_scratch or y_out. */
hive_status hive_hash_collisions(uint32_t kind, const uint32_t *d_keys, uint64_t n, uint64_t m, uint32_t *d_scratch,
                                 uint64_t *y_out, void *stream);

/* ---- Gather ceiling (a measurement aid) ------------------------------------
 * Random 128-byte line reads, the access pattern of bucket probing, with the
 * probe kernel's shape and nothing else: d_out[i] = XOR of the 16 words of
 * line d_idx[i] of d_table (n_lines lines of 16 words; an index >= n_lines
 * reads nothing and gives 0).  All arrays are caller-owned device memory;
 * stream-ordered, no synchronization.  HIVE_ERR_ARG for null arrays with
 * n > 0, n_lines = 0 with n > 0, or n_lines > 2^32. */
hive_status hive_gather_lines(const uint64_t *d_table, uint64_t n_lines, const uint32_t *d_idx, uint64_t n,
                              uint64_t *d_out, void *stream);

/* ---- Persistent executor ------------------------------------------------
 * One resident grid drains a queue of batches in one launch (a hipGraph
 * captured once and replayed).  Each batch runs the same phases and gives
 * the same results as the batch call of its kind (hive_insert_batch,
 * hive_delete_batch, hive_lookup_batch, hive_mixed_batch, including the
 * table's pre/post load-factor rules); batches on one table run in
 * submission order, batches on different tables overlap.  While a table has
 * batches in an executor, no batch call may run on it. */
typedef struct hive_drain *hive_drain_t;

typedef struct {
  uint32_t op_mode;        /* HIVE_OP_INSERT, _DELETE, _LOOKUP, or _MIXED (d_ops) */
  uint32_t flags;          /* HIVE_UNIQUE */
  const uint8_t *d_ops;    /* HIVE_OP_MIXED: per-operation codes */
  const uint32_t *d_keys;
  const uint32_t *d_vals;  /* inserts */
  uint32_t *d_vals_out;    /* lookups; may be NULL */
  uint8_t *d_flags_out;    /* lookups (found), deletes (deleted); may be NULL */
  uint64_t n;
} hive_batch_desc;

/* Create an executor for tables of `slots_per_bucket` slots.  It holds a
 * ring of `ring_capacity` batches and up to `max_tables` tables;
 * `blocks_per_cu` = resident blocks per compute unit (0 = as many as fit);
 * `idle_timeout_us` = microseconds during which the queue makes no progress
 * (nothing new ingested, nothing retired) after which a resident block gives
 * up (0 = the default, 30 s), a watchdog in case the host never stops it. */
hive_status hive_drain_create(uint32_t slots_per_bucket, uint32_t blocks_per_cu, uint64_t ring_capacity,
                              uint32_t max_tables, uint64_t idle_timeout_us, hive_drain_t *out);

/* Append a batch (host only; no HIP call).  *ticket identifies it.  Returns
 * HIVE_ERR_BUDGET when the ring is full or max_tables tables are already
 * registered (retry after completions), and HIVE_ERR_ARG when the executor
 * is running and the batch would need more scratch than the table holds:
 * inserts and mixed batches need a worklist of n entries, batches without
 * HIVE_UNIQUE a dedupe set (create tables with max_batch to preallocate);
 * a stopped executor grows the scratch instead. */
hive_status hive_drain_submit(hive_drain_t d, hive_t table, const hive_batch_desc *b, uint64_t *ticket);

/* Launch the grid.  resident = 0: on `stream`; it exits once every batch it
 * has taken in is complete (batches submitted while it runs are taken in
 * until it has seen the last submission; a later launch serves the rest).
 * resident = 1: on the executor's own non-blocking stream, after the work
 * already enqueued on `stream`; it keeps serving batches submitted later
 * until hive_drain_stop, and holds up no other stream meanwhile (device
 * memory the batches use must be allocated before the launch).  A resident
 * grid leaves one block's room per compute unit free, so that other kernels
 * of the process (copies included) can run while it waits; when the worker
 * kernel's occupancy (queried at create) fits only one block per compute
 * unit, a resident launch returns HIVE_ERR_BUDGET and starts nothing. */
hive_status hive_drain_launch(hive_drain_t d, int resident, void *stream);

/* *done = 1 once the batch's outputs and table updates are complete and
 * visible to the host (no HIP call). */
hive_status hive_drain_poll(hive_drain_t d, uint64_t ticket, int *done);

/* Like hive_drain_poll, and once done *live_after = the table's key count
 * right after the batch (for admission control without a device sync).
 * Valid while the ticket's ring slot has not been reused. */
hive_status hive_drain_result(hive_drain_t d, uint64_t ticket, int *done, uint64_t *live_after);

/* hive_drain_result for n tickets in one call, for serving loops that poll
 * every batch in flight on each turn.  tickets, done and live_after are
 * host arrays of n entries owned by the caller: done[i] = 1 once tickets[i]
 * is complete, and then live_after[i] = the table's key count right after
 * it (0 while it runs).  HIVE_ERR_ARG, with nothing written, when a pointer
 * is null with n > 0, or any ticket was never submitted or has had its ring
 * slot reused. */
hive_status hive_drain_results(hive_drain_t d, const uint64_t *tickets, uint64_t n, uint8_t *done,
                               uint64_t *live_after);

/* Tell a resident grid to exit when its queue is empty and wait for it
 * (`stream` is unused).  Returns HIVE_ERR_HIP if a block gave up on its idle
 * watchdog. */
hive_status hive_drain_stop(hive_drain_t d, void *stream);

/* Stop (if needed), synchronize and free the executor. */
hive_status hive_drain_destroy(hive_drain_t d);

/* Host-callable copies of the device hash and reduction, for tests: the
 * full 32-bit BitHash1/BitHash2 mixes (Section III-C) and the bucket a mixed
 * hash maps to under the table's current geometry (reads the device
 * geometry; synchronizes the table's last stream). */
uint32_t hive_bithash1(uint32_t key);
uint32_t hive_bithash2(uint32_t key);
hive_status hive_bucket_of(hive_t h, uint32_t mixed_hash, uint64_t *bucket);

/* The remainder a % d by multiply-high with a precomputed magic number
 * (Lemire, Kaser, Kurz, "Faster remainder by direct computation", 2019), as
 * the FIXED addressing uses it on the device: exact for all 32-bit a and
 * 1 <= d < 2^32. */
uint64_t hive_fastmod_magic(uint32_t d);
uint32_t hive_fastmod(uint32_t a, uint64_t magic, uint32_t d);

#ifdef __cplusplus
}
#endif

#endif /* HIVE_H */
