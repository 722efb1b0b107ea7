// Hive hash table on MI355X (gfx950): kernels and the C ABI of include/hive.h.
//
// A batch runs as stream-ordered phases (launches):
//   dedupe  (optional) a scratch open-addressing set keeps, per key, the last
//           insert and the first delete of the batch; the others become
//           no-ops, so repeated keys cannot leave two copies (the paper does
//           not say what happens to repeats inside one batch);
//   P1      every operation: hash, match-and-elect over the first and then
//           the second candidate bucket (Section III-F), then replace
//           (Algorithm 1), lookup, delete (Algorithm 4) or claim-then-commit
//           of a free slot (Section III-E, Algorithm 2).  No entry moves in
//           P1, so lookups and deletes never miss a key in flight;
//   P3      inserts whose two buckets were full: bounded cuckoo eviction
//           (Algorithm 3), and after max_evictions displacements the item in
//           hand goes to the stash, or the pending list when the stash is
//           full (Section IV-A step 4; the stash here is an open-addressed
//           table rather than the paper's ring, so a search stops at the
//           first EMPTY slot of its key's probe run instead of scanning).
//
// gfx950 mapping of the warp protocols: with S = 16 a bucket is one 128-byte
// line probed by a 16-lane group, so one wave-wide load probes 4 buckets.
// Each wave owns 64 operations: lanes hash their own operation, the groups
// then issue all 16 bucket loads of the wave before consuming any (memory
// parallelism), ballot the key matches and the empty slots, and hand the
// per-operation result back through LDS.  The free mask of a bucket is the
// ballot of its EMPTY slots; claiming a slot and publishing the entry is one
// 64-bit CAS(EMPTY -> entry), issued lane-per-operation so a wave has 64
// CAS in flight.  A failed CAS returns the word it found, which corrects a
// stale view of the bucket (each XCD has its own L2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <type_traits>
#include <vector>

#include "hash_fns.hpp"
#include "hive.h"
#include "hive_device.hpp"

static_assert(hive::PAIR_BITHASH == HIVE_PAIR_BITHASH && hive::PAIR_CRC == HIVE_PAIR_CRC &&
                  hive::PAIR_MURMUR == HIVE_PAIR_MURMUR && hive::PAIR_TRIPLE == HIVE_PAIR_TRIPLE,
              "hash pair numbering");

namespace hive {

constexpr int WAVES = 4;  // waves per block
constexpr int BLOCK = 64 * WAVES;
#ifndef EVICT_SLOTS_PER_LANE
#define EVICT_SLOTS_PER_LANE 16  // 16-slot buckets: slots per lane of an eviction group (2, 4, 8, 16)
#endif
constexpr int EVICT_GRID = 2048;  // most blocks of the eviction phase (all resident at once)
constexpr int RESIZE_GRID = 2048; // blocks of a resize pass (grid-stride over pairs)
// Most blocks of a probe launch: larger batches stride over tiles, about
// eight tiles per block at 2^26 operations (bulk step +4% against one tile
// per block, measured over 2,048 .. 65,536 blocks: the launch pays less
// block setup, such as the coherent read of the control line)
constexpr uint64_t OPS_GRID = 32768;
constexpr int DRAIN_GRID = 2048;
constexpr int DRAIN_WORDS = 8;  // stash words per thread and trip of the drain
#ifndef OPS_WAVES_PER_EU
#define OPS_WAVES_PER_EU 4  // occupancy target of the probe kernel (waves per SIMD)
#endif

template <int S>
struct Traits {
  static_assert(S == 16 || S == 32 || S == 64, "slots per bucket must be 16, 32 or 64");
  static constexpr int G = 64 / S;  // buckets probed by one wave-wide load
  static constexpr int CH = 16;     // loads in flight per chunk of a probe round
  static constexpr int OPS_PER_CHUNK = CH * G;
  using Mask = typename std::conditional<(S <= 32), uint32_t, uint64_t>::type;
  static constexpr uint64_t FULL = (S == 64) ? ~0ull : ((1ull << S) - 1ull);
};

__device__ __forceinline__ int ctz_mask(uint32_t m) { return __builtin_ctz(m); }
__device__ __forceinline__ int ctz_mask(uint64_t m) { return __builtin_ctzll(m); }
__device__ __forceinline__ int popc_mask(uint32_t m) { return __builtin_popcount(m); }
__device__ __forceinline__ int popc_mask(uint64_t m) { return __builtin_popcountll(m); }

__device__ __forceinline__ uint64_t read_lane64(uint64_t x, int lane) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// Value of lane `src` of the wave, for a 64-bit word.
__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)x);
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(x >> 32));
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Sum over the 64 lanes of a wave (every lane active); every lane gets it.
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
  const int lane = threadIdx.x & 63;
  for (int o = 32; o > 0; o >>= 1) x += shfl64(x, lane ^ o);
  return x;
}

// Worklist segments.  The eviction worklist is NSHARD segments of seg_cap
// entries; tile t (256 operations, or 256 stash entries of a drain) appends
// to segment t % NSHARD through that shard's wl_count, so appends spread
// over NSHARD counters.  A segment receives at most 256 entries from each of
// ceil(tiles / NSHARD) tiles, which bounds seg_cap.
__device__ __forceinline__ uint64_t wl_append(const Ctl *c, uint64_t tile, uint64_t n) {
  return add64(&shard_of(c, tile % NSHARD)->wl_count, n);
}

// Exclusive prefix of the segment fills, pre[0..NSHARD] (pre[NSHARD] is the
// total); the whole block calls it, wave 0 loads and scans.
__device__ __forceinline__ void wl_prefix(const Ctl *c, uint64_t *pre) {
  if (threadIdx.x < NSHARD) {
    const int lane = threadIdx.x;
    uint64_t x = ld_ctl(&shard_of(c, lane)->wl_count);
    for (int o = 1; o < NSHARD; o <<= 1) {
      const uint64_t y = shfl64(x, lane >= o ? lane - o : lane);
      if (lane >= o) x += y;
    }
    pre[lane + 1] = x;
    if (lane == 0) pre[0] = 0;
  }
  __syncthreads();
}

// Position in the worklist of item k < pre[NSHARD] (items numbered segment
// by segment): the last segment whose prefix is <= k holds it.
__device__ __forceinline__ uint64_t wl_slot(const uint64_t *pre, uint64_t k, uint64_t seg_cap) {
  int s = 0;
  for (int step = NSHARD / 2; step > 0; step >>= 1)
    if (pre[s + step] <= k) s += step;
  return (uint64_t)s * seg_cap + (k - pre[s]);
}

// Fold the shards into the totals of Ctl line 1 (one full wave; nothing else
// may update this table's shards meanwhile).  With wl_done the worklist's
// items are counted and its segments emptied.  Returns the worklist size.
__device__ __forceinline__ uint64_t fold_shards_wave(Ctl *c, bool wl_done) {
  const int lane = threadIdx.x & 63;
  Shard *sh = shard_of(c, lane);
  // the last pair: stash placements made without a reservation join the
  // stash count here, after the launch (or executor phase) that made them
  constexpr int NF = 7;
  uint64_t *src[NF] = {&sh->live,          &sh->evictions,       &sh->full_chains,     &sh->invalid_keys,
                       &sh->stash_inserts, &sh->pending_inserts, &sh->stash_unreserved};
  uint64_t *dst[NF] = {&c->live,          &c->evictions,       &c->full_chains, &c->invalid_keys,
                       &c->stash_inserts, &c->pending_inserts, &c->stash_count};
  uint64_t v[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) v[f] = ld_ctl(src[f]);
  const uint64_t wl = ld_ctl(&sh->wl_count);
#pragma unroll
  for (int f = 0; f < NF; ++f)
    if (v[f]) __hip_atomic_store(src[f], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (wl_done && wl) __hip_atomic_store(&sh->wl_count, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
  for (int f = 0; f < NF; ++f) v[f] = wave_sum64(v[f]);
  const uint64_t total_wl = wave_sum64(wl);
  if (lane == 0) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
      if (v[f]) add64(dst[f], v[f]);
    if (wl_done && total_wl) add64(&c->evict_items, total_wl);
  }
  return total_wl;
}

// After a batch or a resize call (one wave of 64 threads).
__global__ __launch_bounds__(64) void finish_kernel(Ctl *c) {
  (void)fold_shards_wave(c, true);
}

// The counters folded with the worklist kept (one wave of 64 threads): the
// key count of a batch whose worklist is placed after its load-factor rule.
__global__ __launch_bounds__(64) void fold_kernel(Ctl *c) {
  (void)fold_shards_wave(c, false);
}

struct OpsArgs {
  uint64_t *buckets;
  uint32_t *hint;
  uint64_t *stash;
  uint64_t *pending;
  Ctl *ctl;
  uint64_t *wl;        // eviction worklist: NSHARD segments of wl_seg_cap entries
  uint64_t wl_seg_cap;
  const uint64_t *dd;  // dedupe set, or null
  uint64_t dd_mask;
  const uint8_t *ops;
  const uint32_t *keys;
  const uint32_t *vals;
  uint32_t *vals_out;
  uint8_t *flags_out;
  uint64_t n;
  uint64_t stash_cap;
  uint64_t pending_cap;
  const uint8_t *win;  // dedupe winner flag per operation (plain launches), or null
};

// ---------------------------------------------------------------------------
// Dedupe: per key, the largest index among inserts (last occurrence wins) and
// the smallest among deletes (the first occurrence reports the deletion).
// Entries are (key << 32 | index); EMPTY never collides since key
// 0xFFFFFFFF is reserved.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t v) {
  for (uint64_t t = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (uint64_t)gridDim.x * BLOCK) p[t] = v;
}

__global__ __launch_bounds__(BLOCK) void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v) {
  for (uint64_t t = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (uint64_t)gridDim.x * BLOCK) p[t] = v;
}

// Record entry e = (k << 32 | index) of an operation of type `op` in the
// set.  Plain loads come first: a key already present costs no CAS, and an
// index that cannot win costs no max/min atomic (a stale load is only ever
// an older value, which would already beat the index, so the skip is safe).
// Settle record e of key k whose claim of slot s found `cur` (not EMPTY):
// the same key keeps the larger insert index or the smaller delete index;
// another key sends the record on along the probe sequence.
__device__ __forceinline__ void dedupe_settle(uint64_t *dd, uint64_t mask, uint32_t op, uint32_t k, uint64_t e,
                                              uint64_t s, uint64_t cur) {
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    if ((uint32_t)(cur >> 32) == k) {
      if (op == OP_INSERT) {
        if (cur < e) __hip_atomic_fetch_max(&dd[s], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (cur > e) {
        __hip_atomic_fetch_min(&dd[s], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return;
    }
    s = (s + 1) & mask;
    cur = dd[s];
    if (cur == EMPTY) {
      cur = cas64(&dd[s], EMPTY, e);
      if (cur == EMPTY) return;
    }
  }
}

__device__ __forceinline__ void dedupe_record(uint64_t *dd, uint64_t mask, uint32_t op, uint32_t k, uint64_t e) {
  const uint64_t s = mix32(k) & mask;
  uint64_t cur = dd[s];
  if (cur == EMPTY) {
    cur = cas64(&dd[s], EMPTY, e);
    if (cur == EMPTY) return;
  }
  dedupe_settle(dd, mask, op, k, e, s, cur);
}

__device__ __forceinline__ void dedupe_insert(uint64_t *dd, uint64_t mask, uint32_t op, const uint32_t *keys,
                                              uint64_t i) {
  const uint32_t k = keys[i];
  if (valid_key(k)) dedupe_record(dd, mask, op, k, ((uint64_t)k << 32) | (uint32_t)i);
}

// Thread t records operation n-1-t if it is an insert and operation t if it
// is a delete: blocks start roughly in order, so inserts arrive in falling
// index order (the winner, the last, comes first) and deletes in rising
// order (the first comes first), and repeated hot keys mostly skip their
// atomics.
__device__ __forceinline__ void dedupe_thread(uint64_t *dd, uint64_t mask, uint32_t mode, const uint8_t *ops,
                                              const uint32_t *keys, uint64_t n, uint64_t t) {
  if (t >= n) return;
  const uint64_t ii = n - 1 - t;
  if (mode == OP_INSERT || (mode == OP_MIXED && ops[ii] == OP_INSERT)) dedupe_insert(dd, mask, OP_INSERT, keys, ii);
  if (mode == OP_DELETE || (mode == OP_MIXED && ops[t] == OP_DELETE)) dedupe_insert(dd, mask, OP_DELETE, keys, t);
}

// ---------------------------------------------------------------------------
// Dedupe of plain launches by hash partitions, with no global atomics.
//
// Device-scope atomics on random words run at about 26 G/s on this GPU
// however many are in flight (measured: 3.1 M CAS into a 64 MiB set take
// 119 us at one or at eight per thread), so a set in HBM costs at least one
// such atomic per distinct key of a chunk.  Instead, records
// (key << 32 | index) are partitioned by the top DDP_BITS bits of mix32(key),
// per operation type, and each partition is deduplicated in LDS:
//   1. collect, per chunk of DD_CHUNK operations and type: the chunk's
//      repeats collapse in an LDS table (a Zipf(0.99) hot key is about 5% of
//      the operations), its distinct records go to its staging area with a
//      histogram over the partitions, and the flags of the type's operations
//      are written: 1 for the chunk's winners, 0 for the rest;
//   2. segment sums: the histograms summed over segments of DDP_SEG chunks;
//   3. scan: per partition, exclusive prefixes over the segments and the
//      partition's total;
//   4. scatter: per segment, each record to its partition's run of `rec`;
//   5. resolve: per partition, an LDS table keeps per key the largest insert
//      index (the last occurrence wins) or the smallest delete index (the
//      first reports the deletion), and clears the flags of the records that
//      lose to another chunk's (random one-byte stores run at about 77 G/s:
//      one per distinct key took 30 us of a 2^22-operation batch).  A partition
//      with more distinct keys than the table takes falls back to a table of
//      its own in HBM (twice its records, in the staging area), by atomics.
// P1 then reads one flag byte per operation, coalesced, instead of looking
// the key up in a set.
// ---------------------------------------------------------------------------
constexpr int DD_PER_THREAD = 8;
constexpr uint64_t DD_CHUNK = (uint64_t)BLOCK * DD_PER_THREAD;
constexpr int DD_LDS = 2 * (int)DD_CHUNK;
constexpr int DDP_BITS = 9;
constexpr int DDP_BINS = 1 << DDP_BITS;  // partitions per operation type
constexpr uint64_t DDP_SEG = 8;          // chunks per segment
constexpr int DDP_SCATTER_LOADS = 8;     // staged records per thread in flight (scatter)
constexpr int DDP_RESOLVE_LOADS = 8;     // records per thread in flight (resolve)
constexpr int DDP_TAB = 8192;            // entries of a resolve table (64 KiB)
constexpr uint32_t DDP_CAP = DDP_TAB * 3 / 4;
static_assert(DDP_BINS % 64 == 0 && DDP_BINS <= BLOCK * 2, "partition counts per block");

__device__ __forceinline__ uint32_t ddp_bin(uint32_t k) { return mix32(k) >> (32 - DDP_BITS); }

struct DdpArgs {
  const uint8_t *ops;
  const uint32_t *keys;
  uint64_t n, nch, nseg;
  uint32_t mode, nt;  // nt: operation types recorded (2 for mixed batches)
  uint64_t *stage;    // max(nt, 2) * nch * DD_CHUNK words: staged records, then fallback tables
  uint64_t *rec;      // n words, partition by partition
  uint8_t *win;       // nch * DD_CHUNK flags, one per operation
  uint16_t *hist;     // nt * nch * DDP_BINS
  uint32_t *cnt;      // nt * nch: staged records per chunk
  uint32_t *seg;      // nt * nseg * DDP_BINS: segment sums, then exclusive prefixes over segments
  uint32_t *tot;      // nt * DDP_BINS: records per partition
};

// Operation type ti of a batch (0 and 1: inserts and deletes of a mixed one).
__device__ __forceinline__ uint32_t ddp_op(const DdpArgs &d, uint32_t ti) {
  return d.mode == OP_MIXED ? (ti == 0 ? OP_INSERT : OP_DELETE) : d.mode;
}

// Step 1.  Block c: chunk c, every recorded operation type at once (a mixed
// batch's inserts and deletes share the block's loads and table: their keys
// are disjoint by contract, so one table collapses both).  A table entry
// holds the key, the operation's type in bit 31 and its index within the
// chunk: a key's entries share one type, so the per-type rule (inserts keep
// the last occurrence, deletes the first) compares their indices alone.
__global__ __launch_bounds__(BLOCK) void ddp_collect_kernel(DdpArgs d) {
  __shared__ uint64_t tab[DD_LDS];
  const uint64_t c = blockIdx.x;
  const uint64_t base = c * DD_CHUNK;
  static_assert(DD_CHUNK <= (1ull << 31), "chunk indices share a word with the type bit");
  // the chunk's operands first, all loads in flight together; ty: the
  // operation's type (0 or 1), or -1 when it is not recorded
  uint32_t kk[DD_PER_THREAD];
  int ty[DD_PER_THREAD];
#pragma unroll
  for (int j = 0; j < DD_PER_THREAD; ++j) {
    const uint64_t i = base + (uint64_t)j * BLOCK + threadIdx.x;
    ty[j] = -1;
    if (i < d.n) {
      if (d.mode != OP_MIXED) ty[j] = 0;
      else {
        const uint8_t o = d.ops[i];
        ty[j] = o == OP_INSERT ? 0 : (o == OP_DELETE ? 1 : -1);
      }
    }
    kk[j] = i < d.n ? d.keys[i] : 0u;
  }
  // the flags of recorded operations start cleared; the chunk's winners set
  // theirs below (after barriers of this block), and the resolve step clears
  // those that lose to another chunk
#pragma unroll
  for (int j = 0; j < DD_PER_THREAD; ++j)
    if (ty[j] >= 0) d.win[base + (uint64_t)j * BLOCK + threadIdx.x] = 0;
  for (int j = threadIdx.x; j < DD_LDS; j += BLOCK) tab[j] = EMPTY;
  __syncthreads();
  // slot[j]: the table slot whose key operation j's thread claimed (the
  // key's first record in this chunk), DD_LDS when it claimed none
  uint32_t slot[DD_PER_THREAD];
#pragma unroll
  for (int j = 0; j < DD_PER_THREAD; ++j) {
    slot[j] = DD_LDS;
    const uint32_t k = kk[j];
    if (ty[j] < 0 || !valid_key(k)) continue;
    const bool keep_last = ddp_op(d, (uint32_t)ty[j]) == OP_INSERT;
    const uint64_t e = ((uint64_t)k << 32) | ((uint32_t)ty[j] << 31) | (uint32_t)(j * BLOCK + threadIdx.x);
    for (uint32_t s = mix32(k) & (DD_LDS - 1);; s = (s + 1) & (DD_LDS - 1)) {
      uint64_t cur = tab[s];
      if (cur == EMPTY) {
        cur = atomicCAS((unsigned long long *)&tab[s], (unsigned long long)EMPTY, (unsigned long long)e);
        if (cur == EMPTY) {
          slot[j] = s;
          break;
        }
      }
      if ((uint32_t)(cur >> 32) == k) {
        // only an update that can change the word (a hot key's later
        // occurrences mostly lose, and atomics on one word serialize)
        if (keep_last) {
          if (cur < e) atomicMax((unsigned long long *)&tab[s], (unsigned long long)e);
        } else if (cur > e) {
          atomicMin((unsigned long long *)&tab[s], (unsigned long long)e);
        }
        break;
      }
    }
  }
  __syncthreads();
  // each distinct key's record, as the collapse left it, is staged by the
  // thread that claimed its slot: the claimants' records are read, the
  // table is then free, and block-wide offsets per type come from a scan of
  // the per-thread counts (records of a type in thread order)
  uint64_t rec[DD_PER_THREAD];
  uint32_t mine0 = 0, mine1 = 0;
#pragma unroll
  for (int j = 0; j < DD_PER_THREAD; ++j) {
    rec[j] = slot[j] < DD_LDS ? tab[slot[j]] : EMPTY;
    if (rec[j] != EMPTY) {
      if (((uint32_t)rec[j] >> 31) != 0) ++mine1;
      else ++mine0;
    }
  }
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t in0 = mine0, in1 = mine1;  // inclusive prefixes within the wave
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y0 = __shfl_up(in0, o, 64), y1 = __shfl_up(in1, o, 64);
    if (lane >= o) {
      in0 += y0;
      in1 += y1;
    }
  }
  __syncthreads();  // every claimant holds its records: tab may be overwritten
  // the waves' totals in the table's last words, the partition histograms
  // (one per type) at its front
  static_assert(2 * DDP_BINS + 2 * WAVES <= 2 * DD_LDS, "histogram room");
  uint32_t *words = (uint32_t *)tab;
  if (lane == 63) {
    words[2 * DD_LDS - 1 - wv] = in0;
    words[2 * DD_LDS - 1 - WAVES - wv] = in1;
  }
  uint32_t *bins = words;
  for (int b = threadIdx.x; b < 2 * DDP_BINS; b += BLOCK) bins[b] = 0u;
  __syncthreads();
  uint32_t off0 = in0 - mine0, off1 = in1 - mine1, cnt0 = 0, cnt1 = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    const uint32_t c0w = words[2 * DD_LDS - 1 - w], c1w = words[2 * DD_LDS - 1 - WAVES - w];
    off0 += w < wv ? c0w : 0u;
    off1 += w < wv ? c1w : 0u;
    cnt0 += c0w;
    cnt1 += c1w;
  }
  uint64_t *st0 = d.stage + c * DD_CHUNK, *st1 = d.stage + ((uint64_t)d.nch + c) * DD_CHUNK;
#pragma unroll
  for (int j = 0; j < DD_PER_THREAD; ++j) {
    if (rec[j] == EMPTY) continue;
    const uint64_t t = rec[j];
    const uint32_t k = (uint32_t)(t >> 32), i = (uint32_t)(base + ((uint32_t)t & (DD_CHUNK - 1)));
    const uint64_t e = ((uint64_t)k << 32) | i;
    const bool t1 = ((uint32_t)t >> 31) != 0;
    if (t1) st1[off1++] = e;
    else st0[off0++] = e;
    d.win[i] = 1;  // within this chunk's flags
    atomicAdd(&bins[(t1 ? DDP_BINS : 0) + ddp_bin(k)], 1u);
  }
  __syncthreads();
  for (uint32_t ti = 0; ti < d.nt; ++ti) {
    uint16_t *h = d.hist + ((uint64_t)ti * d.nch + c) * DDP_BINS;
    for (int b = threadIdx.x; b < DDP_BINS; b += BLOCK) h[b] = (uint16_t)bins[ti * DDP_BINS + b];
  }
  if (threadIdx.x == 0) {
    d.cnt[c] = cnt0;
    if (d.nt > 1) d.cnt[(uint64_t)d.nch + c] = cnt1;
  }
}

// Step 2.  Block (ti, s): the histograms of segment s summed.
__global__ __launch_bounds__(BLOCK) void ddp_segsum_kernel(DdpArgs d) {
  const uint32_t ti = (uint32_t)(blockIdx.x / d.nseg);
  const uint64_t s = blockIdx.x % d.nseg;
  const uint64_t c0 = s * DDP_SEG, c1 = min(c0 + DDP_SEG, d.nch);
  for (int b = threadIdx.x; b < DDP_BINS; b += BLOCK) {
    uint32_t v[DDP_SEG], sum = 0;  // the segment's loads in flight together
#pragma unroll
    for (int j = 0; j < (int)DDP_SEG; ++j)
      v[j] = c0 + j < c1 ? d.hist[((uint64_t)ti * d.nch + c0 + j) * DDP_BINS + b] : 0u;
#pragma unroll
    for (int j = 0; j < (int)DDP_SEG; ++j) sum += v[j];
    d.seg[((uint64_t)ti * d.nseg + s) * DDP_BINS + b] = sum;
  }
}

// Step 3.  Block (ti, g): partitions g * 64 .. g * 64 + 63 of type ti, one per
// lane; its DDP_SCAN_WAVES waves take consecutive ranges of segments, eight
// loads in flight at a time.
constexpr int DDP_SCAN_WAVES = 16;
__global__ __launch_bounds__(DDP_SCAN_WAVES * 64) void ddp_scan_kernel(DdpArgs d) {
  __shared__ uint32_t part[DDP_SCAN_WAVES][64];
  constexpr int GROUPS = DDP_BINS / 64;
  const uint32_t ti = blockIdx.x / GROUPS;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = (blockIdx.x % GROUPS) * 64 + lane;
  const uint64_t q = (d.nseg + DDP_SCAN_WAVES - 1) / DDP_SCAN_WAVES;
  const uint64_t s0 = min((uint64_t)wv * q, d.nseg), s1 = min(s0 + q, d.nseg);
  uint32_t *col = d.seg + (uint64_t)ti * d.nseg * DDP_BINS + b;
  uint32_t sum = 0;
  for (uint64_t s = s0; s < s1; s += 8) {
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = s + j < s1 ? col[(s + j) * DDP_BINS] : 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j) sum += v[j];
  }
  part[wv][lane] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (int w = 0; w < wv; ++w) run += part[w][lane];
  for (uint64_t s = s0; s < s1; s += 8) {
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = s + j < s1 ? col[(s + j) * DDP_BINS] : 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (s + j < s1) {
        col[(s + j) * DDP_BINS] = run;
        run += v[j];
      }
  }
  if (wv == DDP_SCAN_WAVES - 1) d.tot[ti * DDP_BINS + b] = run;
}

// Start of every partition in `rec` (exclusive prefix of the totals over
// (type, partition)) into out[0 .. nt * DDP_BINS); the whole block (NT
// threads) calls it.
template <int NT>
__device__ __forceinline__ void ddp_starts(const DdpArgs &d, uint32_t *out) {
  __shared__ uint32_t s_wave[NT / 64];
  constexpr int PER = 2 * DDP_BINS / NT;  // values per thread (up to two types)
  static_assert(PER >= 1 && PER * NT == 2 * DDP_BINS, "partition counts per block");
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t total = d.nt * DDP_BINS;
  uint32_t v[PER], mine = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const uint32_t x = threadIdx.x * PER + j;
    v[j] = x < total ? d.tot[x] : 0u;
    mine += v[j];
  }
  uint32_t incl = mine;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_wave[wv] = incl;
  __syncthreads();
  uint32_t run = incl - mine;
  for (int w = 0; w < wv; ++w) run += s_wave[w];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const uint32_t x = threadIdx.x * PER + j;
    if (x < total) out[x] = run;
    run += v[j];
  }
  __syncthreads();
}

// The scatter and resolve steps wait on dependent loads and LDS atomics with
// few blocks per CU (a grid of a few hundred, and the resolve table's 64 KiB
// of LDS), so their blocks are 16 waves wide.
constexpr int DDP_WIDE = 1024;

// Step 4.  Block (ti, s): the records of segment s to their partitions' runs.
// A record's place in its partition's run is free, so each round of up to
// DDP_SCATTER_ROUND records is first sorted by partition in LDS (a counting
// sort) and then written run by run: consecutive lanes store consecutive
// words of one run, where one scattered 8-byte store per record had been
// bound by the memory system's rate of random stores.
constexpr int DDP_SCATTER_ROUND = DDP_WIDE * DDP_SCATTER_LOADS;
__global__ __launch_bounds__(DDP_WIDE) void ddp_scatter_kernel(DdpArgs d) {
  __shared__ uint32_t starts[2 * DDP_BINS];
  __shared__ uint32_t lcnt[DDP_BINS], lbase[DDP_BINS], s_sum[DDP_BINS / 64];
  __shared__ uint64_t sorted[DDP_SCATTER_ROUND];
  const uint32_t ti = (uint32_t)(blockIdx.x / d.nseg);
  const uint64_t s = blockIdx.x % d.nseg;
  ddp_starts<DDP_WIDE>(d, starts);
  uint32_t *cur = starts + ti * DDP_BINS;  // this type's cursors
  static_assert(DDP_BINS <= DDP_WIDE, "one partition per thread");
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  if (tid < DDP_BINS) {
    cur[tid] += d.seg[((uint64_t)ti * d.nseg + s) * DDP_BINS + tid];
    lcnt[tid] = 0;
  }
  __syncthreads();
  // the segment's staged records as one list (chunk j holds [pre[j],
  // pre[j + 1]))
  const uint64_t c0 = s * DDP_SEG, c1 = min(c0 + DDP_SEG, d.nch);
  uint32_t pre[DDP_SEG + 1];
  pre[0] = 0;
#pragma unroll
  for (int j = 0; j < (int)DDP_SEG; ++j) pre[j + 1] = pre[j] + (c0 + j < c1 ? d.cnt[(uint64_t)ti * d.nch + c0 + j] : 0u);
  const uint32_t total = pre[DDP_SEG];
  const uint64_t *st = d.stage + ((uint64_t)ti * d.nch + c0) * DD_CHUNK;
  constexpr int U = DDP_SCATTER_LOADS;
  for (uint32_t r0 = 0; r0 < total; r0 += DDP_SCATTER_ROUND) {  // the same rounds in every thread
    const uint32_t nr = min((uint32_t)DDP_SCATTER_ROUND, total - r0);
    uint64_t e[U];
    uint32_t bin[U], rk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t t = r0 + u * DDP_WIDE + tid;
      e[u] = EMPTY;
      if (t < total) {
        int j = 0;
#pragma unroll
        for (int x = 1; x < (int)DDP_SEG; ++x) j += t >= pre[x] ? 1 : 0;
        e[u] = st[(uint64_t)j * DD_CHUNK + (t - pre[j])];
      }
    }
    // each record's rank within its partition in this round
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e[u] != EMPTY) {
        bin[u] = ddp_bin((uint32_t)(e[u] >> 32));
        rk[u] = atomicAdd(&lcnt[bin[u]], 1u);
      }
    __syncthreads();
    // exclusive prefix of the round's partition counts
    uint32_t v = 0, incl = 0;
    if (tid < DDP_BINS) {
      v = lcnt[tid];
      incl = v;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      if (lane == 63) s_sum[wv] = incl;
    }
    __syncthreads();
    if (tid < DDP_BINS) {
      uint32_t run = incl - v;
      for (int w = 0; w < wv; ++w) run += s_sum[w];
      lbase[tid] = run;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e[u] != EMPTY) sorted[lbase[bin[u]] + rk[u]] = e[u];
    __syncthreads();
    // run by run to the partitions' places
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t p = u * DDP_WIDE + tid;
      if (p < nr) {
        const uint64_t x = sorted[p];
        const uint32_t b = ddp_bin((uint32_t)(x >> 32));
        d.rec[cur[b] + (p - lbase[b])] = x;
      }
    }
    __syncthreads();
    if (tid < DDP_BINS) {
      cur[tid] += lcnt[tid];
      lcnt[tid] = 0;
    }
    __syncthreads();
  }
}

// Step 5.  Block (ti, b): partition b of type ti.
__global__ __launch_bounds__(DDP_WIDE) void ddp_resolve_kernel(DdpArgs d) {
  __shared__ uint64_t tab[DDP_TAB];
  __shared__ uint32_t starts[2 * DDP_BINS];
  __shared__ uint32_t s_claims, s_over;
  const uint32_t ti = blockIdx.x / DDP_BINS, b = blockIdx.x % DDP_BINS;
  const uint32_t op = ddp_op(d, ti);
  ddp_starts<DDP_WIDE>(d, starts);
  const uint64_t start = starts[ti * DDP_BINS + b], count = d.tot[ti * DDP_BINS + b];
  if (count == 0) return;  // the same in the whole block
  for (int j = threadIdx.x; j < DDP_TAB; j += DDP_WIDE) tab[j] = EMPTY;
  if (threadIdx.x == 0) {
    s_claims = 0;
    s_over = 0;
  }
  __syncthreads();
  const uint64_t *rec = d.rec + start;
  // at most DDP_WIDE claims land after the one that crosses DDP_CAP (one per
  // thread in flight), so the table never fills and every probe ends
  static_assert(DDP_CAP + DDP_WIDE < DDP_TAB, "resolve table headroom");
  // records DDP_RESOLVE_LOADS at a time per thread, all loads in flight.
  // New keys are counted per wave and record step (one LDS atomic for the
  // wave's claims: one per claim serialized the block on a single word),
  // and the overflow flag is checked before every insert, so each thread
  // claims at most one slot after the count crosses DDP_CAP
  constexpr int U = DDP_RESOLVE_LOADS;
  const int lane = threadIdx.x & 63;
  uint64_t es[U];
#pragma unroll
  for (int u = 0; u < U; ++u) es[u] = EMPTY;
  for (uint64_t r0 = threadIdx.x; r0 < count; r0 += (uint64_t)U * DDP_WIDE) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t r = r0 + (uint64_t)u * DDP_WIDE;
      es[u] = r < count ? rec[r] : EMPTY;
    }
    bool over = false;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t e = es[u];
      over = over || *(volatile uint32_t *)&s_over != 0;
      bool claimed = false;
      if (e != EMPTY && !over) {
        const uint32_t k = (uint32_t)(e >> 32);
        for (uint32_t sl = mix32(k) & (DDP_TAB - 1);; sl = (sl + 1) & (DDP_TAB - 1)) {
          uint64_t cur = tab[sl];
          if (cur == EMPTY) {
            cur = atomicCAS((unsigned long long *)&tab[sl], (unsigned long long)EMPTY, (unsigned long long)e);
            if (cur == EMPTY) {
              claimed = true;
              break;
            }
          }
          if ((uint32_t)(cur >> 32) == k) {
            if (op == OP_INSERT) {
              if (cur < e) atomicMax((unsigned long long *)&tab[sl], (unsigned long long)e);
            } else if (cur > e) {
              atomicMin((unsigned long long *)&tab[sl], (unsigned long long)e);
            }
            break;
          }
        }
      }
      const uint64_t cm = ballot(claimed);
      if (cm && lane == __builtin_ctzll(cm)) {
        const uint32_t c = (uint32_t)__popcll(cm);
        if (atomicAdd(&s_claims, c) + c > DDP_CAP) s_over = 1;
      }
    }
    if (over) break;
  }
  __syncthreads();
  if (!s_over) {
    // every record's flag was set by its chunk: clear the losers' (a key
    // recorded by several chunks), a few scattered stores instead of one
    // per distinct key.  A partition of at most U * DDP_WIDE records was
    // read in one step, and each thread still holds its records.
    const bool held = count <= (uint64_t)U * DDP_WIDE;
    for (uint64_t r0 = threadIdx.x; r0 < count; r0 += (uint64_t)U * DDP_WIDE) {
      if (!held) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint64_t r = r0 + (uint64_t)u * DDP_WIDE;
          es[u] = r < count ? rec[r] : EMPTY;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t e = es[u];
        if (e == EMPTY) continue;
        const uint32_t k = (uint32_t)(e >> 32);
        uint32_t sl = mix32(k) & (DDP_TAB - 1);
        while ((uint32_t)(tab[sl] >> 32) != k) sl = (sl + 1) & (DDP_TAB - 1);
        if (tab[sl] != e) d.win[(uint32_t)e] = 0;
      }
    }
    return;
  }
  // more distinct keys than the table takes: an open-addressed table of
  // 2 x count words in HBM, in the staging area (free after the scatter;
  // partitions' tables are disjoint: [2 start, 2 (start + count))), by
  // atomics (stores written through, so that the claims see them)
  uint64_t *ft = d.stage + 2 * start;
  const uint64_t m = 2 * count;
  for (uint64_t j = threadIdx.x; j < m; j += DDP_WIDE)
    __hip_atomic_store(&ft[j], EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (uint64_t r = threadIdx.x; r < count; r += DDP_WIDE) {
    const uint64_t e = rec[r];
    const uint32_t k = (uint32_t)(e >> 32);
    for (uint64_t sl = mix32(k) % m;; sl = (sl + 1 == m) ? 0 : sl + 1) {
      const uint64_t cur = cas64(&ft[sl], EMPTY, e);
      if (cur == EMPTY) break;
      if ((uint32_t)(cur >> 32) == k) {
        if (op == OP_INSERT) {
          if (cur < e) __hip_atomic_fetch_max(&ft[sl], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (cur > e) {
          __hip_atomic_fetch_min(&ft[sl], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        break;
      }
    }
  }
  __syncthreads();
  // the record left in its key's word is the winner; clear the others' flags
  for (uint64_t r = threadIdx.x; r < count; r += DDP_WIDE) {
    const uint64_t e = rec[r];
    const uint32_t k = (uint32_t)(e >> 32);
    for (uint64_t sl = mix32(k) % m;; sl = (sl + 1 == m) ? 0 : sl + 1) {
      const uint64_t cur = __hip_atomic_load(&ft[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((uint32_t)(cur >> 32) == k) {
        if (cur != e) d.win[(uint32_t)e] = 0;
        break;
      }
    }
  }
}

__device__ __forceinline__ bool dedupe_winner(const uint64_t *dd, uint64_t mask, uint32_t k, uint32_t i) {
  uint64_t s = mix32(k) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const uint64_t cur = dd[s];
    if ((uint32_t)(cur >> 32) == k) return (uint32_t)cur == i;
    if (cur == EMPTY) return true;
    s = (s + 1) & mask;
  }
  return true;
}

// ---------------------------------------------------------------------------
// P1 helpers
// ---------------------------------------------------------------------------

// One probe round of match-and-elect.  Operations t < count of the round
// have their key and bucket in keys[t], bkts[t] and their owning lane in
// list[t] (t itself when list is null).  Each 16-lane group loads one bucket
// per wave-wide load and publishes, through LDS and indexed by the owning
// lane, the match mask, the empty-slot mask and the word of the lowest
// matching slot.  All loads of a chunk are issued before any is consumed.
// bkts[] holds 64 entries: entries from `count` on repeat the round's last
// bucket (the caller pads them), so idle group slots re-load a line that is
// loaded anyway, their result is ignored, and the loads need neither
// control flow nor clamped indices.
// PIPE: wave-wide loads in flight per chunk (the probe's pipelining depth).
template <int S, int PIPE = Traits<S>::CH>
__device__ __forceinline__ void probe_round(const uint64_t *__restrict__ buckets, const uint32_t *keys,
                                            const uint32_t *bkts, const uint8_t *list, int count,
                                            typename Traits<S>::Mask *m_out, typename Traits<S>::Mask *e_out,
                                            uint64_t *w_out, int g, int sl) {
  using T = Traits<S>;
  using Mask = typename T::Mask;
  for (int base = 0; base < count; base += PIPE * T::G) {
    uint64_t w[PIPE];
#pragma unroll
    for (int j = 0; j < PIPE; ++j) w[j] = buckets[(uint64_t)bkts[base + j * T::G + g] * S + sl];
    // keep the operands of the consume loop from being read (and held in
    // registers) while the loads are in flight
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < PIPE; ++j) {
      const int t = base + j * T::G + g;
      const bool mine = t < count;
      const uint32_t ko = keys[t];
      const uint64_t mm = ballot(mine && ko != 0u && key_of(w[j]) == ko);
      const uint64_t ee = ballot(w[j] == EMPTY);
      const Mask gm = (Mask)((mm >> (g * S)) & T::FULL);
      const Mask ge = (Mask)((ee >> (g * S)) & T::FULL);
      if (mine) {
        const int o = list ? list[t] : t;
        if (sl == 0) {
          m_out[o] = gm;
          e_out[o] = ge;
        }
        if (gm != 0 && sl == ctz_mask(gm)) w_out[o] = w[j];
      }
    }
  }
}

// Both probe rounds of an insert batch at once (S = 16): PIPE loads for the
// first candidates and PIPE for the second are in flight together (with
// PIPE = 16 one chunk covers the wave's 64 operations).
template <int S, int PIPE = Traits<S>::CH>
__device__ __forceinline__ void probe_round_pair(const uint64_t *__restrict__ buckets, const uint32_t *keys1,
                                                 const uint32_t *bkts1, typename Traits<S>::Mask *m1_out,
                                                 typename Traits<S>::Mask *e1_out, uint64_t *w1_out,
                                                 const uint32_t *keys2, const uint32_t *bkts2, const uint8_t *list2,
                                                 int count2, typename Traits<S>::Mask *m2_out,
                                                 typename Traits<S>::Mask *e2_out, uint64_t *w2_out, int g, int sl) {
  using T = Traits<S>;
  using Mask = typename T::Mask;
  static_assert(S == 16, "the fused round is built for 16-slot buckets");
  for (int base = 0; base < 64; base += PIPE * T::G) {
    uint64_t wa[PIPE], wb[PIPE];
#pragma unroll
    for (int j = 0; j < PIPE; ++j) wa[j] = buckets[(uint64_t)bkts1[base + j * T::G + g] * S + sl];
#pragma unroll
    for (int j = 0; j < PIPE; ++j) wb[j] = buckets[(uint64_t)bkts2[base + j * T::G + g] * S + sl];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < PIPE; ++j) {
      const int t = base + j * T::G + g;
      const uint32_t ko = keys1[t];
      const uint64_t mm = ballot(ko != 0u && key_of(wa[j]) == ko);
      const uint64_t ee = ballot(wa[j] == EMPTY);
      const Mask gm = (Mask)((mm >> (g * S)) & T::FULL);
      if (sl == 0) {
        m1_out[t] = gm;
        e1_out[t] = (Mask)((ee >> (g * S)) & T::FULL);
      }
      if (gm != 0 && sl == ctz_mask(gm)) w1_out[t] = wa[j];
    }
#pragma unroll
    for (int j = 0; j < PIPE; ++j) {
      const int t = base + j * T::G + g;
      const bool mine = t < count2;
      const uint32_t ko = mine ? keys2[t] : 0u;
      const uint64_t mm = ballot(mine && ko != 0u && key_of(wb[j]) == ko);
      const uint64_t ee = ballot(wb[j] == EMPTY);
      const Mask gm = (Mask)((mm >> (g * S)) & T::FULL);
      if (mine) {
        const int o = list2[t];
        if (sl == 0) {
          m2_out[o] = gm;
          e2_out[o] = (Mask)((ee >> (g * S)) & T::FULL);
        }
        if (gm != 0 && sl == ctz_mask(gm)) w2_out[o] = wb[j];
      }
    }
  }
}

__device__ __forceinline__ bool hinted(const uint32_t *hint, uint32_t c1, uint32_t c2) {
  return ((hint[c1 >> 5] >> (c1 & 31)) & 1u) | ((hint[c2 >> 5] >> (c2 & 31)) & 1u);
}

// Lane-wise search of the stash and the pending list.  The stash is an
// open-addressed table (linear probing from mix32(key)); a search ends at
// the key or at an EMPTY word (tombstones keep probe runs intact).
__device__ __forceinline__ uint64_t *overflow_find(uint64_t *stash, uint64_t stash_cap, uint64_t n_stash,
                                                   uint64_t *pending, uint64_t n_pend, uint32_t k, uint64_t *word,
                                                   bool fresh) {
  if (n_stash) {
    const uint64_t mask = stash_slots_for(stash_cap) - 1;
    for (uint64_t i = 0, p = mix32(k) & mask; i <= mask; ++i, p = (p + 1) & mask) {
      const uint64_t x = fresh ? load_fresh(stash + p) : stash[p];
      if (x == EMPTY) break;
      if (key_of(x) == k) {
        *word = x;
        return stash + p;
      }
    }
  }
  for (uint64_t p = 0; p < n_pend; ++p) {
    const uint64_t x = fresh ? load_fresh(pending + p) : pending[p];
    if (key_of(x) == k) {
      *word = x;
      return pending + p;
    }
  }
  return nullptr;
}

// The second-candidate round's operand list: the operations that need it,
// compacted in lane order (key, bucket, owning lane), and the rest of the 64
// entries padded with the last listed bucket (with lane 0's first bucket when
// the list is empty).
__device__ __forceinline__ void compact_second(bool need2, uint64_t need2_mask, int n2, uint32_t k, uint32_t c2,
                                               uint32_t c1, int lane, uint32_t *k2, uint32_t *b2, uint8_t *list) {
  const uint32_t pad = n2 > 0 ? (uint32_t)__builtin_amdgcn_readlane((int)c2, 63 - __builtin_clzll(need2_mask))
                              : (uint32_t)__builtin_amdgcn_readlane((int)c1, 0);
  if (need2) {
    const uint32_t r = rank_below(need2_mask);
    k2[r] = k;
    b2[r] = c2;
    list[r] = (uint8_t)lane;
  }
  if (lane >= n2) b2[lane] = pad;
}

// ---------------------------------------------------------------------------
// P1: hash, probe, and replace / lookup / delete / claim.
// ---------------------------------------------------------------------------
// LDS of one block of the probe phase (per wave: 64 operations).
// D: candidate buckets per key (a round of results per candidate).
template <int S, int D = 2>
struct OpsShared {
  using Mask = typename Traits<S>::Mask;
  uint32_t key[WAVES][64];
  uint32_t b1[WAVES][64];
  uint32_t k2[WAVES][64];  // rounds 2 (and 3), compacted: key, bucket, owner
  uint32_t b2[WAVES][64];
  uint8_t list[WAVES][64];
  Mask m[D][WAVES][64];
  Mask e[D][WAVES][64];
  uint64_t w[D][WAVES][64];
};

// The table state a probe tile needs, read once per launch (or per chunk of
// the persistent executor).
struct OpsView {
  Geo geo;
  uint64_t n_stash, n_pend;
};

__device__ __forceinline__ OpsView read_view(const Ctl *c, uint64_t stash_cap, uint64_t pending_cap) {
  OpsView v;
  v.geo = read_geo(c);
  v.n_stash = min(ld_ctl(&c->stash_count), stash_cap);
  v.n_pend = min(ld_ctl(&c->pending_count), pending_cap);
  return v;
}

// A wave's key-count change and reserved-key count, added to shard
// unit % NSHARD by its first lane.
__device__ __forceinline__ void ops_counts_add(Ctl *c, uint64_t unit, int64_t live_acc, uint64_t bad_acc) {
  if ((threadIdx.x & 63) == 0) {
    Shard *shd = shard_of(c, unit % NSHARD);
    if (live_acc != 0) add64(&shd->live, (uint64_t)live_acc);
    if (bad_acc) add64(&shd->invalid_keys, bad_acc);
  }
}

// P1 for one tile of WAVES x 64 operations [tile * 256, tile * 256 + 256).
// BOTH: probe both candidates in one round for every operation (inserts of
// new keys always need both; for lookups and deletes it trades bytes for one
// memory round trip fewer).
// PAIR: the table's candidate hashes (HashPair); BitHash1/2 by default.
// With three candidates (PAIR_TRIPLE) the third is probed in a third round
// by the operations that found their key in neither of the first two.
template <int S, uint32_t MODE, bool BOTH, int PAIR = PAIR_BITHASH, int PIPE = Traits<S>::CH>
__device__ __forceinline__ void ops_tile(const OpsArgs &a, const OpsView &view, uint64_t tile,
                                         OpsShared<S, PairArity<PAIR>::D> &sh, int64_t &live_acc,
                                         uint64_t &bad_acc) {
  using T = Traits<S>;
  using Mask = typename T::Mask;
  constexpr bool D3 = PairArity<PAIR>::D == 3;
  auto &s_key = sh.key;
  auto &s_b1 = sh.b1;
  auto &s_k2 = sh.k2;
  auto &s_b2 = sh.b2;
  auto &s_list = sh.list;
  auto &s_m = sh.m;
  auto &s_e = sh.e;
  auto &s_w = sh.w;

  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / S, sl = lane % S;
  const uint64_t i = (tile * WAVES + wv) * 64 + lane;
  const bool active = i < a.n;
  const Geo &geo = view.geo;
  const uint64_t n_stash = view.n_stash, n_pend = view.n_pend;
  const bool overflow_used = (n_stash | n_pend) != 0;

  uint32_t op = OP_NONE, k = 0, v = 0;
  if (active) {
    // the batch's inputs and outputs are touched once: non-temporal, so they
    // do not displace bucket lines from the caches (bulk step +0.7%)
    op = (MODE == OP_MIXED) ? (uint32_t)__builtin_nontemporal_load(&a.ops[i]) : MODE;
    k = __builtin_nontemporal_load(&a.keys[i]);
    if (op == OP_INSERT) v = __builtin_nontemporal_load(&a.vals[i]);
  }
  const bool valid = active && op <= OP_LOOKUP && valid_key(k);
  bool work = valid;
  if (work && op != OP_LOOKUP) {
    if (a.win)
      work = __builtin_nontemporal_load(&a.win[i]) != 0;
    else if (a.dd)
      work = dedupe_winner(a.dd, a.dd_mask, k, (uint32_t)i);
  }
  uint32_t c1 = 0, c2 = 0, c3 = 0;
  if (work) {
    c1 = address(geo, HashPair<PAIR>::h1(k));
    c2 = address(geo, HashPair<PAIR>::h2(k));
    if constexpr (D3) c3 = address(geo, HashPair<PAIR>::h3(k));
  }
  s_key[wv][lane] = work ? k : 0u;
  s_b1[wv][lane] = c1;
  wave_lds_sync();

  // Inserts of new keys need both candidates (absence check and two-choice
  // placement), so insert batches probe both in one round; lookups and
  // deletes probe the second candidate only after a miss in the first.
  constexpr bool kFused = (MODE == OP_INSERT || BOTH) && (S == 16);
  Mask m1;
  bool need2;
  if constexpr (kFused) {
    need2 = work && c2 != c1;
    const uint64_t need2_mask = ballot(need2);
    const int n2 = __popcll(need2_mask);
    compact_second(need2, need2_mask, n2, k, c2, c1, lane, s_k2[wv], s_b2[wv], s_list[wv]);
    wave_lds_sync();
    probe_round_pair<S, PIPE>(a.buckets, s_key[wv], s_b1[wv], s_m[0][wv], s_e[0][wv], s_w[0][wv], s_k2[wv],
                              s_b2[wv], s_list[wv], n2, s_m[1][wv], s_e[1][wv], s_w[1][wv], g, sl);
    wave_lds_sync();
    m1 = s_m[0][wv][lane];
  } else {
    // round 1: first candidate of every operation
    probe_round<S, PIPE>(a.buckets, s_key[wv], s_b1[wv], nullptr, 64, s_m[0][wv], s_e[0][wv], s_w[0][wv], g, sl);
    wave_lds_sync();
    m1 = s_m[0][wv][lane];
    need2 = work && m1 == 0 && c2 != c1;
    const uint64_t need2_mask = ballot(need2);
    const int n2 = __popcll(need2_mask);
    compact_second(need2, need2_mask, n2, k, c2, c1, lane, s_k2[wv], s_b2[wv], s_list[wv]);
    wave_lds_sync();
    // round 2: second candidate of the operations that missed in the first
    if (n2 > 0)
      probe_round<S, PIPE>(a.buckets, s_k2[wv], s_b2[wv], s_list[wv], n2, s_m[1][wv], s_e[1][wv], s_w[1][wv], g,
                           sl);
    wave_lds_sync();
  }
  const Mask e1 = s_e[0][wv][lane];
  // with the fused round a match in the first candidate makes the second's
  // result irrelevant; otherwise the second round ran only without one
  const Mask m2 = (need2 && m1 == 0) ? s_m[1][wv][lane] : (Mask)0;
  const Mask e2 = need2 ? s_e[1][wv][lane] : (Mask)0;
  Mask m3 = 0, e3 = 0;
  bool need3 = false;
  if constexpr (D3) {
    // round 3: the third candidate of the operations without a match so far
    need3 = work && m1 == 0 && m2 == 0 && c3 != c1 && c3 != c2;
    const uint64_t need3_mask = ballot(need3);
    const int n3 = __popcll(need3_mask);
    compact_second(need3, need3_mask, n3, k, c3, c1, lane, s_k2[wv], s_b2[wv], s_list[wv]);
    wave_lds_sync();
    if (n3 > 0)
      probe_round<S, PIPE>(a.buckets, s_k2[wv], s_b2[wv], s_list[wv], n3, s_m[2][wv], s_e[2][wv], s_w[2][wv], g,
                           sl);
    wave_lds_sync();
    if (need3) {
      m3 = s_m[2][wv][lane];
      e3 = s_e[2][wv][lane];
    }
  }

  uint32_t out_v = NO_VALUE;
  uint8_t out_f = 0;
  int dl = 0;
  bool to_wl = false;
  const uint64_t kv = pack(k, v);
  if (work) {
    uint64_t *slot = nullptr, word = 0;
    bool in_bucket = false;
    if (m1) {
      slot = a.buckets + (uint64_t)c1 * S + ctz_mask(m1);
      word = s_w[0][wv][lane];
      in_bucket = true;
    } else if (m2) {
      slot = a.buckets + (uint64_t)c2 * S + ctz_mask(m2);
      word = s_w[1][wv][lane];
      in_bucket = true;
    } else if (D3 && m3) {
      slot = a.buckets + (uint64_t)c3 * S + ctz_mask(m3);
      word = s_w[D3 ? 2 : 0][wv][lane];
      in_bucket = true;
    } else if (overflow_used && (hinted(a.hint, c1, c2) || (D3 && hinted(a.hint, c3, c3)))) {
      slot = overflow_find(a.stash, a.stash_cap, n_stash, a.pending, n_pend, k, &word, false);
    }
    if (op == OP_LOOKUP) {
      if (slot) {
        out_v = value_of(word);
        out_f = 1;
      }
    } else if (slot && in_bucket) {
      // replace (Algorithm 1) or delete (Algorithm 4).  The paper publishes
      // both with one CAS from the word seen; here the word of key k can
      // change only through this operation (no entry moves in this phase,
      // claims only fill EMPTY slots, and a batch gives each key one such
      // operation), so that CAS cannot fail and one 64-bit store does the
      // same: the whole entry is replaced at once and nothing waits for an
      // atomic's return.  The store is an agent-scope atomic one: claims of
      // other XCDs change the same bucket lines in this phase, and a plain
      // store leaves the line dirty in this XCD's L2, whose write-back
      // carries this XCD's stale copy of the neighbouring slots and
      // overwrote such claims (keys inserted by a mixed batch went missing).
      __hip_atomic_store(slot, (op == OP_INSERT) ? kv : EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (op == OP_DELETE) {
        out_f = 1;
        dl = -1;
      }
    } else if (slot) {
      // stash or pending entry: the same single-word update, by CAS (rare)
      const uint64_t desired = (op == OP_INSERT) ? kv : TOMB;
      bool done = false;
      for (int attempt = 0; attempt < 4 && slot; ++attempt) {
        if (cas64(slot, word, desired) == word) {
          done = true;
          break;
        }
        atomicOr(&a.ctl->error, ERR_CAS_RETRY);
        slot = overflow_find(a.stash, a.stash_cap, n_stash, a.pending, n_pend, k, &word, true);
      }
      if (op == OP_DELETE && done) {
        out_f = 1;
        dl = -1;
      }
    } else if (op == OP_INSERT) {
      // claim-then-commit (Algorithm 2) in the candidate with more empty
      // slots first, ties to the first hash: bucketed two-choice placement
      // (three-choice with three candidates)
      dl = 1;
      Mask f_first = e1, f_second = (c2 != c1) ? e2 : (Mask)0;
      uint32_t b_first = c1, b_second = c2;
      if (popc_mask(f_second) > popc_mask(f_first)) {
        const Mask tm = f_first;
        f_first = f_second;
        f_second = tm;
        b_first = c2;
        b_second = c1;
      }
      Mask f_third = 0;
      uint32_t b_third = c3;
      if constexpr (D3) {
        f_third = need3 ? e3 : (Mask)0;
        if (popc_mask(f_third) > popc_mask(f_second)) {
          const Mask tm = f_second;
          f_second = f_third;
          f_third = tm;
          b_third = b_second;
          b_second = c3;
          if (popc_mask(f_second) > popc_mask(f_first)) {
            const Mask t2 = f_first;
            f_first = f_second;
            f_second = t2;
            const uint32_t bt = b_first;
            b_first = b_second;
            b_second = bt;
          }
        }
      }
      bool placed = false;
      while (!placed && (f_first | f_second | f_third)) {
        if (f_first == 0) {
          f_first = f_second;
          b_first = b_second;
          f_second = f_third;
          b_second = b_third;
          f_third = 0;
          continue;
        }
        const int s = ctz_mask(f_first);
        if (cas64(a.buckets + (uint64_t)b_first * S + s, EMPTY, kv) == EMPTY)
          placed = true;
        else
          f_first &= (Mask)(f_first - 1);
      }
      to_wl = !placed;
    }
  }

  // eviction worklist: one atomic per wave, on the tile's segment counter
  const uint64_t wl_mask = ballot(to_wl);
  if (wl_mask) {
    const int leader = __builtin_ctzll(wl_mask);
    uint64_t base = 0;
    if (lane == leader) base = wl_append(a.ctl, tile, (uint64_t)__popcll(wl_mask));
    base = read_lane64(base, leader);
    if (to_wl) a.wl[(tile % NSHARD) * a.wl_seg_cap + base + rank_below(wl_mask)] = kv;
  }
  // key count and reserved keys: summed per wave in registers over the
  // wave's tiles (the caller adds them to its shard once: device atomics
  // run at about 26 G/s, and an insert batch already spends one per
  // operation; aggregating the block's waves per tile instead measured 2-4%
  // slower, its two block barriers costing more than the atomics)
  const uint64_t up = ballot(dl > 0), down = ballot(dl < 0), bad = ballot(active && !valid);
  live_acc += (int64_t)__popcll(up) - (int64_t)__popcll(down);
  bad_acc += (uint64_t)__popcll(bad);
  if (active) {
    if (MODE == OP_LOOKUP || MODE == OP_MIXED) {
      if (a.vals_out) __builtin_nontemporal_store(out_v, &a.vals_out[i]);
      if (a.flags_out) __builtin_nontemporal_store(out_f, &a.flags_out[i]);
    } else if (MODE == OP_DELETE) {
      if (a.flags_out) __builtin_nontemporal_store(out_f, &a.flags_out[i]);
    }
  }
}

// WPE: the occupancy target (waves per SIMD) the registers are allocated
// for; PIPE: loads in flight per probe chunk.  Tuned variants of the
// 16-slot BitHash kernels are picked per table (hive_config.probe_tuning).
template <int S, uint32_t MODE, bool BOTH, int PAIR = PAIR_BITHASH, int WPE = OPS_WAVES_PER_EU,
          int PIPE = Traits<S>::CH>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) void ops_kernel(OpsArgs a) {
  __shared__ OpsShared<S, PairArity<PAIR>::D> sh;
  const OpsView view = read_view(a.ctl, a.stash_cap, a.pending_cap);
  const uint64_t ntiles = (a.n + BLOCK - 1) / BLOCK;
  int64_t live_acc = 0;
  uint64_t bad_acc = 0;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    ops_tile<S, MODE, BOTH, PAIR, PIPE>(a, view, tile, sh, live_acc, bad_acc);
  ops_counts_add(a.ctl, (uint64_t)blockIdx.x * WAVES + (threadIdx.x >> 6), live_acc, bad_acc);
}

// ---------------------------------------------------------------------------
// P3: bounded cuckoo eviction (Algorithm 3) and the stash (Section IV-A step 4)
// ---------------------------------------------------------------------------
struct EvictArgs {
  uint64_t *buckets;
  uint32_t *hint;
  uint64_t *stash;
  uint64_t *pending;
  Ctl *ctl;
  uint64_t *wl;
  uint64_t wl_seg_cap;
  uint64_t stash_cap;
  uint64_t pending_cap;
  uint32_t max_evictions;
};

__device__ __forceinline__ void set_hint(uint32_t *hint, uint32_t b) { or32(&hint[b >> 5], 1u << (b & 31)); }

// Step 4: the item goes to the stash, or to the pending list when the stash
// is full.  Room is reserved by a fetch-add on the count, one per wave for
// all of its pushes (the counts may pass their capacities; every reader
// clamps them); given its reserved position c (c >= capacity: pending), the
// entry claims the first EMPTY or TOMB word of its probe run by CAS (an
// EMPTY one exists: the table has at least twice the capacity).  A TOMB word
// is reused: it already counts as used, and searches pass it, so the entry
// is found at the first free word of its run either way (no key is stashed
// twice: items here are keys absent from the table, and a word taken by
// another placement meanwhile holds a live entry).  Returns where it went:
// 0 stash (an EMPTY word), 3 stash (a TOMB word), 1 pending, 2 lost (the
// pending list was full too; latched as an error).
template <int PAIR = PAIR_BITHASH>
__device__ __forceinline__ int overflow_place(const EvictArgs &a, const Geo &geo, uint64_t kv, uint64_t c) {
  int where = -1;
  if (c < a.stash_cap) {
    const uint64_t mask = stash_slots_for(a.stash_cap) - 1;
    for (uint64_t i = 0, p = mix32(key_of(kv)) & mask; i <= mask; ++i, p = (p + 1) & mask) {
      const uint64_t cur = cas64(a.stash + p, EMPTY, kv);
      if (cur == EMPTY) {
        where = 0;
        break;
      }
      if (cur == TOMB && cas64(a.stash + p, TOMB, kv) == TOMB) {
        where = 3;
        break;
      }
    }
  }
  if (where < 0) {
    const uint64_t p = add64(&a.ctl->pending_count, 1);
    if (p < a.pending_cap) {
      __hip_atomic_store(a.pending + p, kv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      where = 1;
    } else {
      atomicOr(&a.ctl->error, ERR_PENDING_LOST);
      where = 2;
    }
  }
  const uint32_t k = key_of(kv);
  set_hint(a.hint, address(geo, HashPair<PAIR>::h1(k)));
  set_hint(a.hint, address(geo, HashPair<PAIR>::h2(k)));
  if constexpr (PairArity<PAIR>::D == 3) set_hint(a.hint, address(geo, HashPair<PAIR>::h3(k)));
  return where;
}

// Eviction group shape.  A group of L lanes works on one item and sees a
// bucket as P adjacent slots per lane (L x P = S).  A chain is a sequence of
// dependent memory round trips, so the number of chains in flight sets the
// eviction rate: for S = 16 each lane holds a whole bucket (P = 16, measured
// best against 8, 4 and 2: mixed Zipf batches at 95% load 1.2 ms against
// 1.5, 1.9 and 2.4 ms), so a wave runs 64 chains at once; wider buckets keep
// one slot per lane.
template <int S>
struct EvictShape {
  static constexpr int P = (S == 16) ? EVICT_SLOTS_PER_LANE : 1;
  static constexpr int L = S / P;
  static constexpr int G = 64 / L;  // items per wave
  static constexpr uint64_t LANES = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
};

__host__ __device__ __forceinline__ int evict_groups_per_wave(uint32_t S) {
  return S == 16 ? 64 / (16 / EVICT_SLOTS_PER_LANE) : (int)(64 / S);
}

// Bits of slots s = l * P + p from per-word masks (bit l of m[p]).
template <int P, typename Mask>
__device__ __forceinline__ Mask interleave_slots(const uint64_t *m) {
  if constexpr (P == 1) {
    return (Mask)m[0];
  } else if constexpr (P == 2) {
    uint32_t a = (uint32_t)m[0], b = (uint32_t)m[1];  // 8 bits each
    a = (a | (a << 4)) & 0x0F0Fu;
    a = (a | (a << 2)) & 0x3333u;
    a = (a | (a << 1)) & 0x5555u;
    b = (b | (b << 4)) & 0x0F0Fu;
    b = (b | (b << 2)) & 0x3333u;
    b = (b | (b << 1)) & 0x5555u;
    return (Mask)(a | (b << 1));
  } else if constexpr (P == 4) {
    uint32_t r = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      uint32_t x = (uint32_t)m[p];  // 4 bits
      x = (x | (x << 6)) & 0x0303u;
      x = (x | (x << 3)) & 0x1111u;
      r |= x << p;
    }
    return (Mask)r;
  } else if constexpr (P == 8) {
    uint32_t r = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const uint32_t x = (uint32_t)m[p];  // 2 bits
      r |= ((x & 1u) | ((x & 2u) << 7)) << p;
    }
    return (Mask)r;
  } else {
    static_assert(P == 16, "two, four, eight or sixteen slots per lane");
    uint32_t r = 0;
#pragma unroll
    for (int p = 0; p < 16; ++p) r |= ((uint32_t)m[p] & 1u) << p;
    return (Mask)r;
  }
}

// One lane's fresh copy of a whole 16-slot bucket (128 bytes, 128-byte
// aligned) in eight 16-byte loads with the cache policy of an agent-scope
// relaxed atomic load (sc1: served coherently, not from a stale vector-cache
// line).  Atomic loads are at most 8 bytes wide; in the one-lane-per-item
// shape sixteen of them cost each wave instruction 64 scattered lines, eight
// wide ones half the instructions (bulk eviction 205 -> 162 us).  The block
// ends in its own wait for the loads, so the registers are complete when it
// returns.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void load_bucket16_fresh(const uint64_t *b, uint64_t *w) {
  u32x4 x0, x1, x2, x3, x4, x5, x6, x7;
  asm volatile(
      "global_load_dwordx4 %0, %8, off sc1\n"
      "global_load_dwordx4 %1, %8, off offset:16 sc1\n"
      "global_load_dwordx4 %2, %8, off offset:32 sc1\n"
      "global_load_dwordx4 %3, %8, off offset:48 sc1\n"
      "global_load_dwordx4 %4, %8, off offset:64 sc1\n"
      "global_load_dwordx4 %5, %8, off offset:80 sc1\n"
      "global_load_dwordx4 %6, %8, off offset:96 sc1\n"
      "global_load_dwordx4 %7, %8, off offset:112 sc1\n"
      "s_waitcnt vmcnt(0)\n"
      : "=&v"(x0), "=&v"(x1), "=&v"(x2), "=&v"(x3), "=&v"(x4), "=&v"(x5), "=&v"(x6), "=&v"(x7)
      : "v"(b)
      : "memory");
  const u32x4 xs[8] = {x0, x1, x2, x3, x4, x5, x6, x7};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    w[2 * j] = ((uint64_t)xs[j][1] << 32) | xs[j][0];
    w[2 * j + 1] = ((uint64_t)xs[j][3] << 32) | xs[j][2];
  }
}

// Two whole buckets per lane, all sixteen loads in flight before the one
// wait (the same loads as load_bucket16_fresh).
__device__ __forceinline__ void load_bucket16x2_fresh(const uint64_t *b1, const uint64_t *b2, uint64_t *w1,
                                                      uint64_t *w2) {
  u32x4 x0, x1, x2, x3, x4, x5, x6, x7, y0, y1, y2, y3, y4, y5, y6, y7;
  asm volatile(
      "global_load_dwordx4 %0, %16, off sc1\n"
      "global_load_dwordx4 %1, %16, off offset:16 sc1\n"
      "global_load_dwordx4 %2, %16, off offset:32 sc1\n"
      "global_load_dwordx4 %3, %16, off offset:48 sc1\n"
      "global_load_dwordx4 %4, %16, off offset:64 sc1\n"
      "global_load_dwordx4 %5, %16, off offset:80 sc1\n"
      "global_load_dwordx4 %6, %16, off offset:96 sc1\n"
      "global_load_dwordx4 %7, %16, off offset:112 sc1\n"
      "global_load_dwordx4 %8, %17, off sc1\n"
      "global_load_dwordx4 %9, %17, off offset:16 sc1\n"
      "global_load_dwordx4 %10, %17, off offset:32 sc1\n"
      "global_load_dwordx4 %11, %17, off offset:48 sc1\n"
      "global_load_dwordx4 %12, %17, off offset:64 sc1\n"
      "global_load_dwordx4 %13, %17, off offset:80 sc1\n"
      "global_load_dwordx4 %14, %17, off offset:96 sc1\n"
      "global_load_dwordx4 %15, %17, off offset:112 sc1\n"
      "s_waitcnt vmcnt(0)\n"
      : "=&v"(x0), "=&v"(x1), "=&v"(x2), "=&v"(x3), "=&v"(x4), "=&v"(x5), "=&v"(x6), "=&v"(x7), "=&v"(y0),
        "=&v"(y1), "=&v"(y2), "=&v"(y3), "=&v"(y4), "=&v"(y5), "=&v"(y6), "=&v"(y7)
      : "v"(b1), "v"(b2)
      : "memory");
  const u32x4 xs[8] = {x0, x1, x2, x3, x4, x5, x6, x7};
  const u32x4 ys[8] = {y0, y1, y2, y3, y4, y5, y6, y7};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    w1[2 * j] = ((uint64_t)xs[j][1] << 32) | xs[j][0];
    w1[2 * j + 1] = ((uint64_t)xs[j][3] << 32) | xs[j][2];
    w2[2 * j] = ((uint64_t)ys[j][1] << 32) | ys[j][0];
    w2[2 * j + 1] = ((uint64_t)ys[j][3] << 32) | ys[j][2];
  }
}

// EMPTY-slot mask of a whole bucket held by one lane.
__device__ __forceinline__ uint32_t empty_mask16(const uint64_t *w) {
  uint32_t m = 0;
#pragma unroll
  for (int p = 0; p < 16; ++p) m |= (w[p] == EMPTY ? 1u : 0u) << p;
  return m;
}

// The group's fresh view of bucket `bkt`: words w[p] of slots sl * P + p,
// and its EMPTY-slot mask.
template <int S>
__device__ __forceinline__ typename Traits<S>::Mask load_view(const uint64_t *bkt, int g, int sl, uint64_t *w) {
  using E = EvictShape<S>;
  uint64_t m[E::P];
  if constexpr (E::L == 1 && E::P == 16) {
    load_bucket16_fresh(bkt, w);
  } else {
#pragma unroll
    for (int p = 0; p < E::P; ++p) w[p] = load_fresh(bkt + sl * E::P + p);
  }
  if constexpr (E::L == 1) {  // the lane holds the whole bucket
#pragma unroll
    for (int p = 0; p < E::P; ++p) m[p] = w[p] == EMPTY;
  } else {
#pragma unroll
    for (int p = 0; p < E::P; ++p) m[p] = (ballot(w[p] == EMPTY) >> (g * E::L)) & E::LANES;
  }
  return interleave_slots<E::P, typename Traits<S>::Mask>(m);
}

// Claim-then-commit by one group (WABC): `free_mask` holds the group's view
// of the bucket's EMPTY slots; the lowest one is claimed with one CAS by the
// lane holding it, and a failed CAS (the view was stale) drops that slot and
// tries the next.  Returns true when the entry was committed.
template <int S>
__device__ __forceinline__ bool group_claim(uint64_t *bkt, typename Traits<S>::Mask free_mask, uint64_t kv, int g,
                                            int sl) {
  using E = EvictShape<S>;
  using Mask = typename Traits<S>::Mask;
  while (free_mask) {
    const int s = ctz_mask(free_mask);
    bool won = false;
    if (sl == s / E::P) won = cas64(bkt + s, EMPTY, kv) == EMPTY;
    if ((ballot(won) >> (g * E::L)) & E::LANES) return true;
    free_mask &= (Mask)(free_mask - 1);
  }
  return false;
}

// P3: items whose two buckets were full in P1 (or stash entries re-placed
// after a split), one group per item (a group of the eviction shape: one
// lane for 16-slot buckets).  Step 2 is tried again with a fresh view of
// both buckets (two-choice), then the bounded cuckoo chain of Algorithm 3:
// each round claims a free slot of the current bucket or displaces a victim
// by CAS and carries the victim to its alternate bucket.  Returns whether
// the item was placed; if not, the caller sends the entry in hand to the
// stash (or the pending list when the stash is full).
template <int S, int PAIR = PAIR_BITHASH>
__device__ __forceinline__ bool evict_chain(const EvictArgs &a, const Geo &geo, uint64_t &kv, uint32_t max_kicks,
                                            int g, int sl, uint64_t &n_evict) {
  using T = Traits<S>;
  using Mask = typename T::Mask;
  using E = EvictShape<S>;
  const uint32_t c1 = address(geo, HashPair<PAIR>::h1(key_of(kv))), c2 = address(geo, HashPair<PAIR>::h2(key_of(kv)));
  // step 2 with fresh loads (fresh: other items of this phase change buckets)
  uint64_t w[E::P], w2v[E::P];
  // one lane holding whole buckets: both candidates in one round trip
  constexpr bool kLaneBucket = E::L == 1 && E::P == 16;
  Mask f1, f2;
  if constexpr (kLaneBucket) {
    load_bucket16x2_fresh(a.buckets + (uint64_t)c1 * S, a.buckets + (uint64_t)c2 * S, w, w2v);
    f1 = (Mask)empty_mask16(w);
    f2 = (Mask)empty_mask16(w2v) & (Mask)((c2 != c1) ? ~0ull : 0ull);
  } else {
    f1 = load_view<S>(a.buckets + (uint64_t)c1 * S, g, sl, w);
    f2 = load_view<S>(a.buckets + (uint64_t)c2 * S, g, sl, w2v) & (Mask)((c2 != c1) ? ~0ull : 0ull);
  }
  bool placed;
  if constexpr (PairArity<PAIR>::D == 3) {
    // three-choice: the emptiest candidate first, ties to the lower hash
    const uint32_t c3 = address(geo, HashPair<PAIR>::h3(key_of(kv)));
    const Mask f3 = load_view<S>(a.buckets + (uint64_t)c3 * S, g, sl, w) &
                    (Mask)((c3 != c1 && c3 != c2) ? ~0ull : 0ull);
    Mask f[3] = {f1, f2, f3};
    uint32_t c[3] = {c1, c2, c3};
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2 - x; ++y)
        if (popc_mask(f[y + 1]) > popc_mask(f[y])) {
          const Mask tf = f[y];
          f[y] = f[y + 1];
          f[y + 1] = tf;
          const uint32_t tc = c[y];
          c[y] = c[y + 1];
          c[y + 1] = tc;
        }
    placed = group_claim<S>(a.buckets + (uint64_t)c[0] * S, f[0], kv, g, sl) ||
             group_claim<S>(a.buckets + (uint64_t)c[1] * S, f[1], kv, g, sl) ||
             group_claim<S>(a.buckets + (uint64_t)c[2] * S, f[2], kv, g, sl);
  } else {
    if (popc_mask(f2) > popc_mask(f1))
      placed = group_claim<S>(a.buckets + (uint64_t)c2 * S, f2, kv, g, sl) ||
               group_claim<S>(a.buckets + (uint64_t)c1 * S, f1, kv, g, sl);
    else
      placed = group_claim<S>(a.buckets + (uint64_t)c1 * S, f1, kv, g, sl) ||
               group_claim<S>(a.buckets + (uint64_t)c2 * S, f2, kv, g, sl);
  }
  uint32_t b = c1;  // chains start at the first candidate
  // look-ahead chains keep the view of the bucket they move to: w holds
  // bucket b's words when `have_view` (first the view step 2 loaded; its
  // free slots were just tried)
  bool have_view = kLaneBucket && PairArity<PAIR>::D == 2;
  for (uint32_t kick = 1; kick <= max_kicks && !placed; ++kick) {
    uint64_t *bkt = a.buckets + (uint64_t)b * S;
    if (!have_view) {
      const Mask fm = load_view<S>(bkt, g, sl, w);
      if (group_claim<S>(bkt, fm, kv, g, sl)) {
        placed = true;
        break;
      }
    }
    have_view = false;
    if constexpr (kLaneBucket && PairArity<PAIR>::D == 2) {
      // Look ahead: two candidate victims at pseudo-random distinct slots;
      // both alternate buckets are loaded in one round trip, and a victim
      // whose alternate has an EMPTY slot is displaced and claims that slot
      // from the view just loaded.  At 95% load most chains then end after
      // one displacement instead of several, and far fewer run out of
      // rounds into the stash (mixed Zipf batches at 95%: 130 K stash
      // entries per 2^22 operations before, about 12 K with look-ahead);
      // with no room in either, the first is displaced and the chain goes
      // on from its alternate.  (Four candidates, loaded one after another,
      // stretched every chain that fails to four more round trips per
      // displacement.)
      constexpr int LA = 2;
      const uint32_t r = mix32(key_of(kv) ^ (kick * 0x9E3779B9u));
      int vs[LA];
      uint64_t vw[LA];
      uint32_t va[LA];
#pragma unroll
      for (int j = 0; j < LA; ++j) {
        vs[j] = (int)((r + 5u * (uint32_t)j) & 15u);
        vw[j] = w[vs[j]];
        const uint32_t a1 = address(geo, HashPair<PAIR>::h1(key_of(vw[j])));
        const uint32_t a2 = address(geo, HashPair<PAIR>::h2(key_of(vw[j])));
        va[j] = (b == a1) ? a2 : a1;
      }
      load_bucket16x2_fresh(a.buckets + (uint64_t)va[0] * S, a.buckets + (uint64_t)va[1] * S, w, w2v);
      const Mask fa = (Mask)empty_mask16(w) & (Mask)((va[0] != b) ? ~0ull : 0ull);
      const Mask fb = (Mask)empty_mask16(w2v) & (Mask)((va[1] != b) ? ~0ull : 0ull);
      const int pick = (fa == 0 && fb != 0) ? 1 : 0;
      const Mask fpick = pick ? fb : fa;
      const uint64_t victim = vw[pick];
      if (cas64(bkt + vs[pick], victim, kv) != victim) continue;  // the slot changed: count the round
      if (victim == EMPTY) {
        placed = true;  // the slot was empty after all: the CAS claimed it
        break;
      }
      ++n_evict;
      kv = victim;
      b = va[pick];
      if (fpick && group_claim<S>(a.buckets + (uint64_t)b * S, fpick, kv, g, sl)) {
        placed = true;
        break;
      }
      // no room there (or it was taken meanwhile): the next displacement
      // works from the view just loaded, one round trip fewer
      if (pick == 1) {
#pragma unroll
        for (int p = 0; p < 16; ++p) w[p] = w2v[p];
      }
      have_view = true;
      continue;
    }
    // victim: a pseudo-random slot (the paper's "first occupied" slot is
    // slot 0 of every full bucket, which lets two chains trade the same
    // pair of entries back and forth)
    const int s0 = (int)(mix32(key_of(kv) ^ (kick * 0x9E3779B9u)) & (S - 1));
    const uint64_t ws = w[s0 % E::P];  // this lane's word at the victim's position in its pair
    bool won = false;
    if (sl == s0 / E::P) won = cas64(bkt + s0, ws, kv) == ws;
    const bool ok = (ballot(won) >> (g * E::L)) & E::LANES;
    const uint64_t victim = shfl64(ws, g * E::L + s0 / E::P);
    if (!ok) continue;  // the slot changed under us: count the round, keep the item
    if (victim == EMPTY) {
      placed = true;  // the slot was empty after all: the CAS claimed it
      break;
    }
    ++n_evict;
    kv = victim;
    const uint32_t v1 = address(geo, HashPair<PAIR>::h1(key_of(kv)));
    const uint32_t v2 = address(geo, HashPair<PAIR>::h2(key_of(kv)));
    if constexpr (PairArity<PAIR>::D == 3) {
      // the victim's next candidate after b, in hash order, cyclically
      const uint32_t v3 = address(geo, HashPair<PAIR>::h3(key_of(kv)));
      b = (b == v1) ? v2 : (b == v2) ? v3 : v1;
    } else {
      b = (b == v1) ? v2 : v1;  // AltBucket: the victim's other candidate
    }
  }
  return placed;  // if not, kv is the entry in hand
}

// One item per group of the wave (`have`: the group has one, at worklist
// position `pos`); every lane of the wave calls it.  Each item takes step 2
// (two-choice claim on fresh loads) and the bounded chain of Algorithm 3;
// an entry still in hand goes to the stash.  `unreserved`: the launch cannot
// fill the stash (its count when the launch started plus the launch's items
// is within capacity), so entries take stash slots without touching the
// count, which every pushing wave would otherwise reserve from, one atomic
// each on a single address (thousands of waves queue there in a stash drain);
// their number is added per wave to the shards and folded into the count
// after the launch.  Otherwise one count reservation per wave.
//
// DEFER (phase timing of the plain path): step 4 is left to its own launch,
// stash_kernel, so that steps 3 and 4 are timed apart; the item's worklist
// word is overwritten with the entry still in hand, or EMPTY once placed.
template <int S, int PAIR = PAIR_BITHASH, bool DEFER = false>
__device__ __forceinline__ void evict_round(const EvictArgs &a, const Geo &geo, bool unreserved, bool have,
                                            uint64_t pos, int g, int sl, uint64_t &n_evict, uint64_t &n_full,
                                            uint64_t &n_side, uint64_t &n_fresh) {
  uint64_t kv = 0;
  bool placed = true;
  if (have) {
    kv = a.wl[pos];
    placed = evict_chain<S, PAIR>(a, geo, kv, a.max_evictions, g, sl, n_evict);
  }
  if constexpr (DEFER) {
    if (have && sl == 0) {
      a.wl[pos] = placed ? EMPTY : kv;
      n_full += !placed;
    }
    return;
  }
  const bool push = !placed && sl == 0;
  const uint64_t pm = ballot(push);
  if (pm) {
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(pm);
    uint64_t base = 0;
    if (!unreserved) {
      if (lane == leader) {
        const uint64_t n = (uint64_t)__popcll(pm);
        base = load_fresh(&a.ctl->stash_count) < a.stash_cap ? add64(&a.ctl->stash_count, n) : a.stash_cap;
      }
      base = read_lane64(base, leader);
    }
    if (push) {
      ++n_full;
      const int where = overflow_place<PAIR>(a, geo, kv, base + rank_below(pm));
      n_side += (where == 0 || where == 3) ? 1 : where == 1 ? (1ull << 32) : 0;
      n_fresh += where == 0;
    }
  }
}

// Chain statistics of a wave (per group, held by its lane 0) added to the
// wave's shard.  Every lane of the wave calls it.  n_side counts the lane's
// stash placements in its low half and pending ones in its high half (a
// wave places far fewer than 2^32 entries); n_fresh counts the stash
// placements that took an EMPTY word, the ones that add a used word to the
// count (when the launch reserved no room, they are added after it).
__device__ __forceinline__ void evict_counters(const EvictArgs &a, bool unreserved, uint64_t unit, uint64_t n_evict,
                                               uint64_t n_full, uint64_t n_side, uint64_t n_fresh, int sl) {
  const uint64_t e = wave_sum64(sl == 0 ? n_evict : 0), f = wave_sum64(n_full), sd = wave_sum64(n_side);
  const uint64_t fr = wave_sum64(n_fresh);
  if ((threadIdx.x & 63) == 0 && (e | f | sd)) {
    Shard *sh = shard_of(a.ctl, unit % NSHARD);
    if (e) add64(&sh->evictions, e);
    if (f) add64(&sh->full_chains, f);
    if ((uint32_t)sd) add64(&sh->stash_inserts, (uint32_t)sd);
    if (fr && unreserved) add64(&sh->stash_unreserved, fr);
    if (sd >> 32) add64(&sh->pending_inserts, sd >> 32);
  }
}

// P3 as a launch: every worklist item through evict_round (step 2 again,
// then the bounded chain of Algorithm 3, then the stash or the pending list),
// one item per group of the eviction shape, the grid striding over items.
// The worklist is emptied afterwards by finish_kernel (it also counts the
// items and folds unreserved stash placements into the stash count), so this
// kernel takes no ticket.
template <int S, int PAIR = PAIR_BITHASH, bool DEFER = false>
__global__ __launch_bounds__(BLOCK) void evict_kernel(EvictArgs a) {
  using E = EvictShape<S>;
  __shared__ uint64_t pre[NSHARD + 1];
  wl_prefix(a.ctl, pre);
  const uint64_t cnt = pre[NSHARD];
  if (cnt == 0) return;  // same in every block
  const Geo geo = read_geo(a.ctl);
  // the same in every block: an unreserved launch leaves the count alone
  const bool unreserved = ld_ctl(&a.ctl->stash_count) + cnt <= a.stash_cap;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / E::L, sl = lane % E::L;
  const uint64_t groups = (uint64_t)gridDim.x * WAVES * E::G;
  uint64_t n_evict = 0, n_full = 0, n_side = 0, n_fresh = 0;
  const uint64_t first = ((uint64_t)blockIdx.x * WAVES + wv) * E::G + g;
  // a uniform trip count per wave: every lane reaches the wave-wide steps
  const uint64_t wave_first = ((uint64_t)blockIdx.x * WAVES + wv) * E::G;
  for (uint64_t base = wave_first; base < cnt; base += groups) {
    const uint64_t t = base - wave_first + first;
    evict_round<S, PAIR, DEFER>(a, geo, unreserved, t < cnt, t < cnt ? wl_slot(pre, t, a.wl_seg_cap) : 0, g, sl,
                                n_evict, n_full, n_side, n_fresh);
  }
  evict_counters(a, unreserved, (uint64_t)blockIdx.x * WAVES + wv, n_evict, n_full, n_side, n_fresh, sl);
}

// P3 for 16-slot buckets with two candidates, as a launch whose lanes are
// refilled as their chains end.  Each wave owns a contiguous range of the
// worklist (at least 64 items); a lane takes the range's next item whenever
// it holds none, so a wave lasts about as long as its lanes' total work
// rather than one round per 64 items, each as long as its longest chain
// (at 95% load a few percent of the chains run all their rounds, and nearly
// every group of 64 items held one).  A lane steps through one memory round
// trip at a time:
//   FRESH   both candidates loaded (step 2 again, two-choice claim);
//   LOOK    one displacement round of the look-ahead chain: two victims of
//           the bucket in hand, both alternates loaded in one round trip,
//           a victim displaced by CAS and its slot claimed from that view;
//   RELOAD  the bucket in hand loaded again after a displacement CAS found
//           its slot changed, and its free slots tried.
// The rounds, the victims and the stash placement are those of evict_chain
// and evict_round (step 4 reserves room once per wave and step, as there);
// only the order in which a wave's items run differs.  The grid should be
// resident at once: a wave's range is not shared.
template <int PAIR>
__global__ __launch_bounds__(BLOCK) void evict_lanes_kernel(EvictArgs a) {
  static_assert(PairArity<PAIR>::D == 2, "two candidate buckets");
  constexpr int S = 16;
  using Mask = typename Traits<S>::Mask;
  __shared__ uint64_t pre[NSHARD + 1];
  wl_prefix(a.ctl, pre);
  const uint64_t cnt = pre[NSHARD];
  if (cnt == 0) return;  // same in every block
  const Geo geo = read_geo(a.ctl);
  // the same in every block: an unreserved launch leaves the count alone
  const bool unreserved = ld_ctl(&a.ctl->stash_count) + cnt <= a.stash_cap;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t nw = (uint64_t)gridDim.x * WAVES, wid = (uint64_t)blockIdx.x * WAVES + wv;
  const uint64_t q = max<uint64_t>(64, (cnt + nw - 1) / nw);
  const uint64_t end = min(cnt, (wid + 1) * q);
  uint64_t cursor = wid * q;  // the wave's next item (the same in every lane)
  const uint32_t max_kicks = a.max_evictions;
  uint64_t n_evict = 0, n_full = 0, n_side = 0, n_fresh = 0;
  constexpr int IDLE = 0, FRESH = 1, RELOAD = 2, LOOK = 3;
  int st = IDLE;
  uint64_t kv = 0;        // the entry in hand
  uint32_t b = 0;         // the bucket it is carried into
  uint32_t kick = 0;      // displacement rounds taken
  uint64_t w[16], w2v[16];  // LOOK, RELOAD: w holds bucket b's words
  while (cursor < end || ballot(st != IDLE)) {
    // lanes without an item take the range's next ones, in lane order
    const uint64_t nm = ballot(st == IDLE);
    if (nm && cursor < end) {
      const uint64_t t = cursor + rank_below(nm);
      if (st == IDLE && t < end) {
        kv = a.wl[wl_slot(pre, t, a.wl_seg_cap)];
        st = FRESH;
        kick = 0;
      }
      cursor += (uint64_t)__popcll(nm);
    }
    // this step's two bucket loads
    uint32_t x1 = 0, x2 = 0;
    int vs0 = 0, vs1 = 0;
    uint64_t vw0 = 0, vw1 = 0;
    if (st == FRESH) {
      x1 = address(geo, HashPair<PAIR>::h1(key_of(kv)));
      x2 = address(geo, HashPair<PAIR>::h2(key_of(kv)));
    } else if (st == RELOAD) {
      x1 = b;
      x2 = b;
    } else if (st == LOOK) {
      // two candidate victims at pseudo-random distinct slots (round kick + 1)
      const uint32_t r = mix32(key_of(kv) ^ ((kick + 1) * 0x9E3779B9u));
      vs0 = (int)(r & 15u);
      vs1 = (int)((r + 5u) & 15u);
      vw0 = w[vs0];
      vw1 = w[vs1];
      const uint32_t a1 = address(geo, HashPair<PAIR>::h1(key_of(vw0))), a2 = address(geo, HashPair<PAIR>::h2(key_of(vw0)));
      const uint32_t b1 = address(geo, HashPair<PAIR>::h1(key_of(vw1))), b2 = address(geo, HashPair<PAIR>::h2(key_of(vw1)));
      x1 = (b == a1) ? a2 : a1;
      x2 = (b == b1) ? b2 : b1;
    }
    if (st != IDLE) load_bucket16x2_fresh(a.buckets + (uint64_t)x1 * S, a.buckets + (uint64_t)x2 * S, w, w2v);
    bool fail = false;  // the chain ran out of rounds: step 4
    if (st == FRESH) {
      const Mask f1 = (Mask)empty_mask16(w);
      const Mask f2 = (Mask)empty_mask16(w2v) & (Mask)((x2 != x1) ? ~0ull : 0ull);
      bool placed;
      if (popc_mask(f2) > popc_mask(f1))
        placed = group_claim<S>(a.buckets + (uint64_t)x2 * S, f2, kv, lane, 0) ||
                 group_claim<S>(a.buckets + (uint64_t)x1 * S, f1, kv, lane, 0);
      else
        placed = group_claim<S>(a.buckets + (uint64_t)x1 * S, f1, kv, lane, 0) ||
                 group_claim<S>(a.buckets + (uint64_t)x2 * S, f2, kv, lane, 0);
      if (placed) {
        st = IDLE;
      } else if (max_kicks == 0) {
        fail = true;
      } else {
        b = x1;  // chains start at the first candidate, whose view w holds
        st = LOOK;
      }
    } else if (st == RELOAD) {
      st = group_claim<S>(a.buckets + (uint64_t)b * S, (Mask)empty_mask16(w), kv, lane, 0) ? IDLE : LOOK;
    } else if (st == LOOK) {
      ++kick;
      const Mask fa = (Mask)empty_mask16(w) & (Mask)((x1 != b) ? ~0ull : 0ull);
      const Mask fb = (Mask)empty_mask16(w2v) & (Mask)((x2 != b) ? ~0ull : 0ull);
      const int pick = (fa == 0 && fb != 0) ? 1 : 0;
      const Mask fpick = pick ? fb : fa;
      const uint64_t victim = pick ? vw1 : vw0;
      const int vsl = pick ? vs1 : vs0;
      if (cas64(a.buckets + (uint64_t)b * S + vsl, victim, kv) != victim) {
        // the slot changed: the round is spent, the item stays in hand
        if (kick < max_kicks) st = RELOAD;
        else fail = true;
      } else if (victim == EMPTY) {
        st = IDLE;  // the slot was empty after all: the CAS claimed it
      } else {
        ++n_evict;
        kv = victim;
        b = pick ? x2 : x1;
        if (fpick && group_claim<S>(a.buckets + (uint64_t)b * S, fpick, kv, lane, 0)) {
          st = IDLE;
        } else if (kick < max_kicks) {
          // the next round works from the view just loaded
          if (pick == 1) {
#pragma unroll
            for (int p = 0; p < 16; ++p) w[p] = w2v[p];
          }
        } else {
          fail = true;
        }
      }
    }
    // step 4 for the chains that ran out of rounds
    const uint64_t pm = ballot(fail);
    if (pm) {
      const int leader = __builtin_ctzll(pm);
      uint64_t base = 0;
      if (!unreserved) {
        if (lane == leader) {
          const uint64_t n = (uint64_t)__popcll(pm);
          base = load_fresh(&a.ctl->stash_count) < a.stash_cap ? add64(&a.ctl->stash_count, n) : a.stash_cap;
        }
        base = read_lane64(base, leader);
      }
      if (fail) {
        ++n_full;
        const int where = overflow_place<PAIR>(a, geo, kv, base + rank_below(pm));
        n_side += (where == 0 || where == 3) ? 1 : where == 1 ? (1ull << 32) : 0;
        n_fresh += where == 0;
        st = IDLE;
      }
    }
  }
  evict_counters(a, unreserved, wid, n_evict, n_full, n_side, n_fresh, 0);
}

// Step 4 as its own launch (after evict_kernel<.., DEFER>): every worklist
// word that still holds an entry goes to the stash or the pending list, one
// entry per lane, with the same room reservation as the fused path.
template <int PAIR = PAIR_BITHASH>
__global__ __launch_bounds__(BLOCK) void stash_kernel(EvictArgs a) {
  __shared__ uint64_t pre[NSHARD + 1];
  wl_prefix(a.ctl, pre);
  const uint64_t cnt = pre[NSHARD];
  if (cnt == 0) return;
  const Geo geo = read_geo(a.ctl);
  const bool unreserved = ld_ctl(&a.ctl->stash_count) + cnt <= a.stash_cap;
  const int lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  uint64_t n_side = 0, n_fresh = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * BLOCK + (threadIdx.x & ~63u); base < cnt; base += stride) {
    const uint64_t t = base + lane;
    const uint64_t kv = t < cnt ? a.wl[wl_slot(pre, t, a.wl_seg_cap)] : EMPTY;
    const bool push = kv != EMPTY;
    const uint64_t pm = ballot(push);
    if (!pm) continue;
    const int leader = __builtin_ctzll(pm);
    uint64_t room = 0;
    if (!unreserved) {
      if (lane == leader) {
        const uint64_t n = (uint64_t)__popcll(pm);
        room = load_fresh(&a.ctl->stash_count) < a.stash_cap ? add64(&a.ctl->stash_count, n) : a.stash_cap;
      }
      room = read_lane64(room, leader);
    }
    if (push) {
      const int where = overflow_place<PAIR>(a, geo, kv, room + rank_below(pm));
      n_side += (where == 0 || where == 3) ? 1 : where == 1 ? (1ull << 32) : 0;
      n_fresh += where == 0;
    }
  }
  evict_counters(a, unreserved, (uint64_t)blockIdx.x * WAVES + (threadIdx.x >> 6), 0, 0, n_side, n_fresh, 0);
}

// ---------------------------------------------------------------------------
// Linear-hashing resize (Section IV-C), decided on the device.
//
// A resize call is planned by resize_plan_kernel (pairs to split or merge),
// then runs as segments, one per hashing round: pass 1 splits the segment's
// pairs, or tests each merge pair for room; pass 2 moves the merge pairs that
// passed, from the top down to the first that did not.  The last block of
// each pass updates the geometry and plans the next segment, so the host
// launches a fixed number of segments and never reads the device.
// ---------------------------------------------------------------------------
enum : uint32_t { PLAN_PRE = 0, PLAN_PRE_MIXED = 1, PLAN_POST = 2, PLAN_SPLIT = 3, PLAN_MERGE = 4 };

struct ResizeArgs {
  uint64_t *buckets;
  uint32_t *hint;
  Ctl *ctl;
  uint32_t S;
  uint32_t K;
  uint32_t lf_expand_pct;
  uint32_t lf_contract_pct;
};

// Geometry of the next segment.  Splits first finish a round (sp == im+1 is
// the same addressing as the next round with sp == 0); merges first regress
// a round when sp == 0 (again the same addressing).
__device__ __forceinline__ void plan_next(volatile Ctl *c) {
  c->seg = 0;
  if (c->resize_todo == 0) {
    c->resize_dir = 0;
    return;
  }
  if (c->resize_dir > 0) {
    if (c->sp == c->im + 1) {
      c->im = 2 * c->im + 1;
      c->sp = 0;
    }
    const uint64_t room = c->max_buckets - c->n_buckets;
    if (room == 0) {
      c->resize_todo = 0;
      c->resize_dir = 0;
      return;
    }
    c->seg = min(min(c->resize_todo, c->im + 1 - c->sp), room);
  } else {
    if (c->n_buckets <= c->initial_buckets) {
      c->resize_todo = 0;
      c->resize_dir = 0;
      return;
    }
    if (c->sp == 0) {
      c->im >>= 1;
      c->sp = c->im + 1;
    }
    c->seg = min(min(c->resize_todo, c->sp), c->n_buckets - c->initial_buckets);
    c->merge_commit = c->seg;
  }
}

// Pairs the load-factor rule asks for, in whole K-pair steps: expansion
// while (live + extra) * 100 > lf_expand * buckets * S, contraction while
// live * 100 < lf_contract * buckets * S and the table is above its initial
// size.
__device__ __forceinline__ void plan_policy(volatile Ctl *c, const ResizeArgs &a, uint64_t extra,
                                            bool allow_contract) {
  const uint64_t S = a.S, K = a.K, nb = c->n_buckets, live = c->live;
  const uint64_t need = live + extra;
  if (need * 100 > (uint64_t)a.lf_expand_pct * nb * S) {
    const uint64_t den = (uint64_t)a.lf_expand_pct * S;
    const uint64_t r = (need * 100 + den - 1) / den;  // fewest buckets that satisfy the rule
    const uint64_t steps = (r - nb + K - 1) / K;
    c->resize_dir = 1;
    c->resize_todo = steps * K;
  } else if (allow_contract && live * 100 < (uint64_t)a.lf_contract_pct * nb * S && nb > c->initial_buckets) {
    const uint64_t q = live * 100 / ((uint64_t)a.lf_contract_pct * S);
    const uint64_t lim = max(q, c->initial_buckets);
    if (nb > lim) {
      const uint64_t steps = (nb - lim + K - 1) / K;
      const uint64_t fin = (nb > steps * K && nb - steps * K > c->initial_buckets) ? nb - steps * K
                                                                                  : c->initial_buckets;
      c->resize_dir = -1;
      c->resize_todo = nb - fin;
    }
  }
}

// Start a resize call (one thread): the pairs the call asks for, then the
// first segment.  `amount` is the insert count (PRE), or the pair count
// (SPLIT, MERGE).
__device__ __forceinline__ void plan_start(volatile Ctl *c, const ResizeArgs &a, uint32_t mode, uint64_t amount) {
  c->resize_dir = 0;
  c->resize_todo = 0;
  c->ticket = 0;
  if (c->mode != ADDR_LINEAR) {
    c->seg = 0;
    return;
  }
  switch (mode) {
    case PLAN_PRE:
    case PLAN_PRE_MIXED: plan_policy(c, a, amount, false); break;
    case PLAN_POST: plan_policy(c, a, 0, true); break;
    case PLAN_SPLIT:
      c->resize_dir = 1;
      c->resize_todo = amount;
      break;
    default:
      c->resize_dir = -1;
      c->resize_todo = amount;
      break;
  }
  plan_next(c);
}

// Insert operations of a mixed batch, for its pre-batch plan: one add per
// block to Ctl::plan_inserts, which the plan kernel reads and clears.
__global__ __launch_bounds__(BLOCK) void count_inserts_kernel(Ctl *c, const uint8_t *ops, uint64_t n) {
  __shared__ unsigned long long block_sum;
  if (threadIdx.x == 0) block_sum = 0;
  __syncthreads();
  unsigned long long mine = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (uint64_t)gridDim.x * BLOCK)
    mine += ops[i] == OP_INSERT;
  mine = wave_sum64(mine);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&block_sum, mine);
  __syncthreads();
  if (threadIdx.x == 0 && block_sum) add64(&c->plan_inserts, block_sum);
}

// A mixed batch's insert count and the plan in one block (batches of at most
// BLOCK * 16 operations: one launch fewer).
__global__ __launch_bounds__(BLOCK) void count_and_plan_kernel(ResizeArgs a, const uint8_t *ops, uint64_t n) {
  __shared__ unsigned long long block_sum;
  if (threadIdx.x == 0) block_sum = 0;
  __syncthreads();
  unsigned long long mine = 0;
  for (uint64_t i = threadIdx.x; i < n; i += BLOCK) mine += ops[i] == OP_INSERT;
  mine = wave_sum64(mine);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&block_sum, mine);
  __syncthreads();
  if (threadIdx.x == 0) plan_start(a.ctl, a, PLAN_PRE_MIXED, block_sum);
}

__global__ void resize_plan_kernel(ResizeArgs a, uint32_t mode, uint64_t amount) {
  uint64_t n = amount;
  if (mode == PLAN_PRE_MIXED) {
    n = ld_ctl(&a.ctl->plan_inserts);
    __hip_atomic_store(&a.ctl->plan_inserts, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  plan_start(a.ctl, a, mode, n);
}

// Ticket for "the last block of this launch": every block has finished its
// reads of the control block.  Two levels, so that no counter takes more
// than NSHARD atomics: block b counts on shard b % NSHARD, and the block
// completing a shard counts on Ctl::ticket.  The last block resets both
// levels for the next launch.
//
// No release fence before the count: the last block only rewrites control
// scalars (geometry, counts) that the other blocks read before they count
// (their loads have returned: the values bound the work they did), and the
// table words the other blocks wrote are read by later launches, which the
// kernel boundary orders.  An agent-scope release writes back the block's
// L2, one after another per XCD: with a 2,048-block grid the fences alone
// cost 26 us (43 us with dirty lines) against 7 us for the same launch
// without them.
__device__ __forceinline__ bool last_block(Ctl *c) {
  __shared__ bool last;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t grid = gridDim.x, s = blockIdx.x % NSHARD;
    const uint64_t in_shard = (grid - s + NSHARD - 1) / NSHARD;
    bool l = false;
    if (add64(&shard_of(c, s)->ticket, 1) + 1 == in_shard)
      l = add64(&c->ticket, 1) + 1 == min(grid, (uint64_t)NSHARD);
    last = l;
  }
  __syncthreads();
  if (last) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x < NSHARD)
      __hip_atomic_store(&shard_of(c, threadIdx.x)->ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) __hip_atomic_store(&c->ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return last;
}

__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t r) {
  for (uint32_t i = 0; i < r; ++i) m &= m - 1;
  return (uint32_t)__builtin_ctzll(m);
}

// One split pair (Section IV-C-1): pair j of the segment is (src, src + 2^m)
// with src = sp + j.  An entry stays when one of its candidate hashes still
// addresses src under the next round's mask, otherwise it moves; movers are
// compacted into the partner's first slots (the partner is EMPTY).
template <int S>
__device__ __forceinline__ void split_pair(const ResizeArgs &a, uint64_t im, uint64_t sp, uint64_t j, int g, int sl) {
  using T = Traits<S>;
  const uint64_t src = sp + j, dst = src + im + 1, next = 2 * im + 1;
  const uint64_t w = a.buckets[src * S + sl];
  bool move = false;
  if (w != EMPTY) {
    const uint32_t h1 = bithash1(key_of(w)), h2 = bithash2(key_of(w));
    const bool stay = ((h1 & im) == src && (h1 & next) == src) || ((h2 & im) == src && (h2 & next) == src);
    move = !stay;
  }
  const uint64_t mm = (ballot(move) >> (g * S)) & T::FULL;
  if (move) {
    const uint32_t rank = __builtin_popcountll(mm & ((1ull << sl) - 1ull));
    a.buckets[dst * S + rank] = w;
    a.buckets[src * S + sl] = EMPTY;
  }
}

// Merge pair j of the segment, walked from the top: (lo, lo + 2^m) with
// lo = sp - 1 - j.  It fits when hi's entries fit lo's EMPTY slots
// (Section IV-C-2); the first pair that does not fit bounds the commit.
template <int S>
__device__ __forceinline__ void merge_test_pair(const ResizeArgs &a, Ctl *c, uint64_t im, uint64_t sp, uint64_t j,
                                                int g, int sl) {
  using T = Traits<S>;
  const uint64_t lo = sp - 1 - j, hi = lo + im + 1;
  const uint64_t wl = a.buckets[lo * S + sl], wh = a.buckets[hi * S + sl];
  const uint64_t fl = (ballot(wl == EMPTY) >> (g * S)) & T::FULL;
  const uint64_t lh = (ballot(wh != EMPTY) >> (g * S)) & T::FULL;
  if (sl == 0 && __builtin_popcountll(lh) > __builtin_popcountll(fl))
    __hip_atomic_fetch_min(&c->merge_commit, j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Move a merge pair that fits: the r-th live entry of hi goes to the r-th
// EMPTY slot of lo; stash entries with a candidate in hi now address lo.
template <int S>
__device__ __forceinline__ void merge_move_pair(const ResizeArgs &a, uint64_t im, uint64_t sp, uint64_t j, int g,
                                                int sl) {
  using T = Traits<S>;
  const uint64_t lo = sp - 1 - j, hi = lo + im + 1;
  const uint64_t wl = a.buckets[lo * S + sl], wh = a.buckets[hi * S + sl];
  const uint64_t fl = (ballot(wl == EMPTY) >> (g * S)) & T::FULL;
  const uint64_t lh = (ballot(wh != EMPTY) >> (g * S)) & T::FULL;
  if (wh != EMPTY) {
    const uint32_t r = __builtin_popcountll(lh & ((1ull << sl) - 1ull));
    a.buckets[lo * S + nth_set_bit(fl, r)] = wh;
    a.buckets[hi * S + sl] = EMPTY;
  }
  if (sl == 0 && ((a.hint[hi >> 5] >> (hi & 31)) & 1u)) set_hint(a.hint, (uint32_t)lo);
}

// Geometry after a finished segment (run by one thread once every pair of
// the segment is done), then the plan of the next segment.
__device__ __forceinline__ void split_segment_done(volatile Ctl *c, uint64_t sp, uint64_t seg) {
  c->sp = sp + seg;
  c->n_buckets += seg;
  c->resize_todo -= seg;
  c->split_happened = 1;
  plan_next(c);
}

__device__ __forceinline__ void merge_segment_done(volatile Ctl *c, uint64_t sp, uint64_t seg, uint64_t commit) {
  c->sp = sp - commit;
  c->n_buckets -= commit;
  c->resize_todo -= commit;
  if (commit < seg) c->resize_todo = 0;  // a pair did not fit: the call stops here
  plan_next(c);
}

// Pass 1: split the segment's pairs, or test merge pairs.
template <int S>
__global__ __launch_bounds__(BLOCK) void resize_pass1_kernel(ResizeArgs a) {
  using T = Traits<S>;
  Ctl *c = a.ctl;
  const uint64_t seg = c->seg;
  if (seg == 0) return;  // same value in every block: nobody takes a ticket
  const int64_t dir = c->resize_dir;
  const uint64_t im = c->im, sp = c->sp;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / S, sl = lane % S;
  const uint64_t groups = (uint64_t)gridDim.x * WAVES * T::G;
  for (uint64_t j = ((uint64_t)blockIdx.x * WAVES + wv) * T::G + g; j < seg; j += groups) {
    if (dir > 0)
      split_pair<S>(a, im, sp, j, g, sl);
    else
      merge_test_pair<S>(a, c, im, sp, j, g, sl);
  }
  if (dir > 0 && last_block(c) && threadIdx.x == 0) split_segment_done(c, sp, seg);
}

// Pass 2: move the merge pairs that fit, top down.
template <int S>
__global__ __launch_bounds__(BLOCK) void resize_pass2_kernel(ResizeArgs a) {
  using T = Traits<S>;
  Ctl *c = a.ctl;
  const uint64_t seg = c->seg;
  if (seg == 0 || c->resize_dir > 0) return;
  const uint64_t commit = c->merge_commit;
  const uint64_t im = c->im, sp = c->sp;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / S, sl = lane % S;
  const uint64_t groups = (uint64_t)gridDim.x * WAVES * T::G;
  for (uint64_t j = ((uint64_t)blockIdx.x * WAVES + wv) * T::G + g; j < commit; j += groups)
    merge_move_pair<S>(a, im, sp, j, g, sl);
  if (last_block(c) && threadIdx.x == 0) merge_segment_done(c, sp, seg, commit);
}

// After splits: every stash and pending entry moves to the eviction worklist
// (the eviction phase re-places it under the new geometry) and the hint bits
// are cleared (Section III-B "Overflow Stash").  One wave-aggregated append
// per wave and item range; `t` indexes stash words (the whole table, which
// is reset to EMPTY on the way) then pending entries, and the 256-entry tile
// t / 256 picks the worklist segment.
__device__ __forceinline__ uint64_t drain_word(uint64_t t, uint64_t n_stash_words, uint64_t total,
                                               const uint64_t *stash, const uint64_t *pending) {
  return t < n_stash_words ? stash[t] : t < total ? pending[t - n_stash_words] : TOMB;
}

// Word w (drain_word of t) to the worklist; a used stash word is reset.
__device__ __forceinline__ void drain_append(uint64_t t, uint64_t w, uint64_t n_stash_words, uint64_t *stash,
                                             uint64_t *wl, uint64_t seg_cap, Ctl *c) {
  if (t < n_stash_words && w != EMPTY) stash[t] = EMPTY;
  const bool live = w != TOMB && w != EMPTY;
  const uint64_t m = ballot(live);
  if (m) {
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    uint64_t base = 0;
    const uint64_t tile = t / BLOCK;
    if (lane == leader) base = wl_append(c, tile, (uint64_t)__popcll(m));
    base = read_lane64(base, leader);
    if (live) wl[(tile % NSHARD) * seg_cap + base + rank_below(m)] = w;
  }
}

__device__ __forceinline__ void drain_collect(uint64_t t, uint64_t n_stash_words, uint64_t total, uint64_t *stash,
                                              const uint64_t *pending, uint64_t *wl, uint64_t seg_cap, Ctl *c) {
  drain_append(t, drain_word(t, n_stash_words, total, stash, pending), n_stash_words, stash, wl, seg_cap, c);
}

__device__ __forceinline__ void drain_done(volatile Ctl *c) {
  c->stash_count = 0;
  c->pending_count = 0;
  c->split_happened = 0;
}

__global__ __launch_bounds__(BLOCK) void drain_kernel(uint64_t *stash, uint64_t stash_cap, uint64_t *pending,
                                                      uint64_t pending_cap, uint32_t *hint, uint64_t hint_n,
                                                      uint64_t *wl, uint64_t seg_cap, Ctl *c) {
  if (!c->split_happened) return;
  const uint64_t n_stash = min(c->stash_count, stash_cap) ? stash_slots_for(stash_cap) : 0;
  const uint64_t n_pend = min(c->pending_count, pending_cap);
  const uint64_t total = n_stash + n_pend;
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  const uint64_t tid = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (total) {
    for (uint64_t t = tid; t < hint_n; t += stride) hint[t] = 0u;
  }
  // A trip of a block takes DRAIN_WORDS tiles of 256 words that share one
  // worklist segment (tiles T, T + NSHARD, ...: word t is in tile t / 256,
  // which appends to segment tile % NSHARD, so segment fills stay within the
  // capacity sized from the words walked), loads all of its words at once
  // (the walk of a mostly empty stash table is bound by load latency), and
  // appends its live words with one atomic: per-wave appends queued
  // thousands of atomics on each segment counter.
  __shared__ uint32_t s_wave[WAVES];
  __shared__ uint64_t s_base;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t tiles = (total + BLOCK - 1) / BLOCK;
  const uint64_t group = (uint64_t)NSHARD * DRAIN_WORDS;  // tiles of NSHARD trips
  const uint64_t trips = (tiles + group - 1) / group * NSHARD;
  for (uint64_t q = blockIdx.x; q < trips; q += gridDim.x) {
    const uint64_t seg = q % NSHARD, tile0 = (q / NSHARD) * group + seg;
    uint64_t w[DRAIN_WORDS];
#pragma unroll
    for (int j = 0; j < DRAIN_WORDS; ++j)
      w[j] = drain_word((tile0 + (uint64_t)j * NSHARD) * BLOCK + threadIdx.x, n_stash, total, stash, pending);
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < DRAIN_WORDS; ++j) {
      const uint64_t t = (tile0 + (uint64_t)j * NSHARD) * BLOCK + threadIdx.x;
      if (t < n_stash && w[j] != EMPTY) stash[t] = EMPTY;
      mine += (w[j] != TOMB && w[j] != EMPTY) ? 1u : 0u;
    }
    // block-wide exclusive prefix of the live counts
    uint32_t incl = mine;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    uint32_t before = 0, sum = 0;
#pragma unroll
    for (int x = 0; x < WAVES; ++x) {
      before += x < wv ? s_wave[x] : 0u;
      sum += s_wave[x];
    }
    if (threadIdx.x == 0 && sum) s_base = wl_append(c, seg, sum);
    __syncthreads();
    if (sum) {
      uint64_t pos = seg * seg_cap + s_base + before + incl - mine;
#pragma unroll
      for (int j = 0; j < DRAIN_WORDS; ++j)
        if (w[j] != TOMB && w[j] != EMPTY) wl[pos++] = w[j];
    }
    __syncthreads();  // s_wave and s_base of the next trip
  }
  if (last_block(c) && threadIdx.x == 0) drain_done(c);
}

// ---------------------------------------------------------------------------
// Dump: every live word with its place (bucket, -1 stash, -2 pending).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void dump_kernel(const uint64_t *buckets, uint32_t S, const uint64_t *stash,
                                                     const uint64_t *pending, Ctl *ctl, uint64_t stash_cap,
                                                     uint64_t pending_cap, uint64_t *out, int64_t *where,
                                                     uint64_t cap) {
  const uint64_t nb = ctl->n_buckets;
  const uint64_t n_stash = min(ctl->stash_count, stash_cap) ? stash_slots_for(stash_cap) : 0;
  const uint64_t n_pend = min(ctl->pending_count, pending_cap);
  const uint64_t n_slots = nb * S, total = n_slots + n_stash + n_pend;
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  const uint64_t span = (total + stride - 1) / stride * stride;  // uniform trip count
  const int lane = threadIdx.x & 63;
  for (uint64_t t = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; t < span; t += stride) {
    uint64_t w = EMPTY;
    int64_t pl = 0;
    if (t < n_slots) {
      w = buckets[t];
      pl = (int64_t)(t / S);
    } else if (t < n_slots + n_stash) {
      w = stash[t - n_slots];
      pl = -1;
    } else if (t < total) {
      w = pending[t - n_slots - n_stash];
      pl = -2;
    }
    const bool live = t < total && w != EMPTY && w != TOMB;
    const uint64_t m = ballot(live);
    if (m) {
      const int leader = __builtin_ctzll(m);
      uint64_t base = 0;
      if (lane == leader) base = add64(&ctl->dump_count, (uint64_t)__popcll(m));
      base = read_lane64(base, leader);
      const uint64_t pos = base + rank_below(m);
      if (live && pos < cap) {
        out[pos] = w;
        if (where) where[pos] = pl;
      }
    }
  }
}

// Placement census: live bucket entries in their first candidate bucket and
// in their second one (the two differ).
// SET32: buckets of 32-bit entries (the key itself; EMPTY is all ones).
template <bool SET32>
__global__ __launch_bounds__(BLOCK) void placement_kernel(const void *bucket_words, uint32_t S, Ctl *ctl) {
  __shared__ unsigned long long s_first, s_second;
  if (threadIdx.x == 0) s_first = s_second = 0;
  __syncthreads();
  unsigned long long n_first = 0, n_second = 0;
  const Geo geo = read_geo(ctl);
  const uint64_t n_slots = geo.n_buckets * S;
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  const uint64_t span = (n_slots + stride - 1) / stride * stride;
  for (uint64_t t = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; t < span; t += stride) {
    uint64_t w = EMPTY;
    if (t < n_slots) {
      if constexpr (SET32) {
        const uint32_t x = ((const uint32_t *)bucket_words)[t];
        w = x == 0xFFFFFFFFu ? EMPTY : x;
      } else {
        w = ((const uint64_t *)bucket_words)[t];
      }
    }
    const bool live = w != EMPTY;
    const bool first = live && address(geo, bithash1(key_of(w))) == (uint32_t)(t / S);
    const uint64_t mf = ballot(first), ms = ballot(live && !first);
    if ((threadIdx.x & 63) == 0) {
      n_first += (uint64_t)__popcll(mf);
      n_second += (uint64_t)__popcll(ms);
    }
  }
  // one pair of atomics per block
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&s_first, n_first);
    atomicAdd(&s_second, n_second);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_first) add64(&ctl->place_first, s_first);
    if (s_second) add64(&ctl->place_second, s_second);
  }
}

__global__ void ctl_zero_placement_kernel(Ctl *ctl) {
  ctl->place_first = 0;
  ctl->place_second = 0;
}

__global__ void ctl_reset_kernel(Ctl *ctl, Ctl init) { *ctl = init; }
__global__ void ctl_zero_dump_kernel(Ctl *ctl) { ctl->dump_count = 0; }


// ---------------------------------------------------------------------------
// Persistent executor: one resident grid drains a queue of batches.
//
// The host appends batch descriptors to a ring in pinned host memory and
// advances a host-side tail.  Blocks of the resident grid ingest new
// descriptors into a device ring, and each batch then runs as a sequence of
// data-parallel phases (dedupe fill, dedupe, insert count, resize segments,
// stash drain, re-placement, probe tiles, eviction) split into chunks that
// any block may claim.  One 64-bit word per batch packs the phase, its chunk
// count and the number of chunks claimed, so a claim is one atomic add; the
// block that completes the last chunk of a phase runs the phase's scalar
// epilogue (geometry updates, plans) and publishes the next phase.  Batches
// on one table run in submission order (a per-table sequence number);
// batches on different tables overlap.  Completion is written to host-mapped
// memory.  Every block leaves the loop once the host has set the stop flag
// and every ingested batch is complete.
// ---------------------------------------------------------------------------
enum : uint32_t {
  PH_START = 0, PH_FILL = 1, PH_DEDUPE = 2, PH_COUNT = 3, PH_SEG_A = 4, PH_SEG_B = 5, PH_DRAIN = 6,
  PH_REPLACE = 7, PH_OPS = 8, PH_EVICT = 9, PH_DONE = 10
};
// Chunk sizes.  A claim costs a few dependent device-scope round trips, so
// streaming phases take large chunks; an eviction chunk gives each group
// one item, so a phase's chains run side by side in as many waves as the
// grid holds instead of one after another in fewer waves.
constexpr uint64_t FILL_PER_CHUNK = BLOCK * 64;   // words per fill chunk
constexpr uint64_t COUNT_PER_CHUNK = BLOCK * 16;  // operations per count chunk
constexpr uint64_t DRAIN_TILES = 16;              // stash tiles of BLOCK words per drain chunk
constexpr uint64_t M28 = (1ull << 28) - 1;
constexpr uint32_t DRAIN_WINDOW = 64;             // batches scanned for work

struct TableDesc {
  uint64_t *buckets;
  uint32_t *hint;
  uint64_t *stash;
  uint64_t *pending;
  Ctl *ctl;
  uint64_t *wl;
  uint64_t *dd;
  uint64_t wl_seg_cap, stash_cap, pending_cap, hint_words;
  uint32_t S, max_evictions, K, lf_expand_pct, lf_contract_pct, pre_expand, post_policy, addressing;
};

struct ReqDesc {  // written by the host
  TableDesc t;
  const uint8_t *ops;
  const uint32_t *keys;
  const uint32_t *vals;
  uint32_t *vals_out;
  uint8_t *flags_out;
  uint64_t n;
  uint32_t mode, flags;
  uint64_t seq, table_slot, ticket, dd_size;
};
static_assert(sizeof(ReqDesc) % 8 == 0, "descriptor copied as 64-bit words");

struct ReqState {
  ReqDesc d;
  uint64_t state;  // phase:8 | chunks:28 | claimed:28
  uint64_t done;   // chunks of the current phase completed
  uint64_t aux;    // inserts counted for the pre-batch plan
  uint64_t seg_sp, seg_n, seg_im;
  int64_t seg_dir;
  uint64_t items;  // eviction items of the current eviction phase
  uint32_t resume; // phase that follows the current resize call
  uint32_t pad_;
};

struct DrainQueue {
  ReqState *req;              // device ring
  const ReqDesc *host_ring;   // pinned host ring
  const uint64_t *host_tail;  // pinned: descriptors written by the host
  const uint32_t *host_stop;  // pinned: set when no more work will come
  uint64_t *host_done;        // pinned: per ring slot, ticket + 1 once complete
  uint64_t *host_live;        // pinned: per ring slot, the table's live count after the batch
  uint64_t *table_next;       // per table slot: sequence number allowed to run
  uint64_t cap;
  uint64_t idle_ticks;        // device wall-clock ticks without queue progress before a block gives up
  uint64_t ingested;
  uint64_t head;
  uint64_t completed;
  uint32_t ingest_lock;
  uint32_t error;             // 1: a block hit the idle watchdog
  uint32_t final_seen;        // the host stopped and every submitted batch was ingested
  uint32_t pad_;
};

__device__ __forceinline__ uint64_t make_state(uint32_t ph, uint64_t nch) {
  return ((uint64_t)ph << 56) | ((nch & M28) << 28);
}

__device__ __forceinline__ uint64_t ld_sys(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ ResizeArgs resize_args(const ReqDesc &d) {
  return ResizeArgs{d.t.buckets, d.t.hint, d.t.ctl, d.t.S, d.t.K, d.t.lf_expand_pct, d.t.lf_contract_pct};
}

__device__ __forceinline__ EvictArgs evict_args(const ReqDesc &d) {
  return EvictArgs{d.t.buckets, d.t.hint,       d.t.stash,       d.t.pending,      d.t.ctl,
                   d.t.wl,      d.t.wl_seg_cap, d.t.stash_cap,   d.t.pending_cap,  d.t.max_evictions};
}

__device__ __forceinline__ bool has_inserts(const ReqDesc &d) { return d.mode == OP_INSERT || d.mode == OP_MIXED; }

__device__ __forceinline__ uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// After a resize step: the next segment, the stash drain after splits, or
// the phase the resize call returns to.
__device__ __forceinline__ uint32_t seg_entry(volatile ReqState *r, const ReqDesc &d) {
  volatile Ctl *c = d.t.ctl;
  if (c->seg > 0) {
    r->seg_sp = c->sp;
    r->seg_n = c->seg;
    r->seg_im = c->im;
    r->seg_dir = c->resize_dir;
    return PH_SEG_A;
  }
  if (c->split_happened) return PH_DRAIN;
  return r->resume;
}

// Successor of a finished phase; scalar work between phases happens here.
__device__ __forceinline__ uint32_t successor(volatile ReqState *r, const ReqDesc &d, uint32_t ph) {
  volatile Ctl *c = d.t.ctl;
  const bool linear = d.t.addressing == ADDR_LINEAR;
  switch (ph) {
    case PH_START: return d.n ? PH_FILL : PH_DONE;  // an empty batch changes nothing, as in the plain path
    case PH_FILL: return PH_DEDUPE;
    case PH_DEDUPE: return PH_COUNT;
    case PH_COUNT:
      if (linear && d.t.pre_expand && has_inserts(d)) {
        plan_start(c, resize_args(d), PLAN_PRE, d.mode == OP_MIXED ? r->aux : d.n);
        r->resume = PH_OPS;
        return seg_entry(r, d);
      }
      return PH_OPS;
    case PH_SEG_A: return r->seg_dir < 0 ? PH_SEG_B : seg_entry(r, d);
    case PH_SEG_B: return seg_entry(r, d);
    case PH_DRAIN: return PH_REPLACE;
    case PH_REPLACE: return r->resume;
    case PH_OPS: return PH_EVICT;
    case PH_EVICT:
      if (linear && d.t.post_policy && d.mode != OP_LOOKUP) {
        plan_start(c, resize_args(d), PLAN_POST, 0);
        r->resume = PH_DONE;
        return seg_entry(r, d);
      }
      return PH_DONE;
    default: return PH_DONE;
  }
}

// Chunks of a phase about to start (0: nothing to do).
__device__ __forceinline__ uint64_t enter(volatile ReqState *r, const ReqDesc &d, uint32_t ph) {
  volatile Ctl *c = d.t.ctl;
  const uint64_t gpb = (uint64_t)WAVES * (64 / d.t.S);  // groups per block
  switch (ph) {
    case PH_FILL: return d.dd_size ? ceil_div(d.dd_size, FILL_PER_CHUNK) : 0;
    case PH_DEDUPE: return d.dd_size ? ceil_div(d.n, BLOCK) : 0;
    case PH_COUNT:
      r->aux = 0;
      return (d.t.addressing == ADDR_LINEAR && d.t.pre_expand && d.mode == OP_MIXED) ? ceil_div(d.n, COUNT_PER_CHUNK)
                                                                                     : 0;
    case PH_SEG_A: return ceil_div(r->seg_n, gpb);
    case PH_SEG_B: return ceil_div(c->merge_commit, gpb);
    case PH_DRAIN: {
      const uint64_t total = (min(c->stash_count, d.t.stash_cap) ? stash_slots_for(d.t.stash_cap) : 0) +
                             min(c->pending_count, d.t.pending_cap);
      return total ? max(ceil_div(total, BLOCK * DRAIN_TILES), ceil_div(d.t.hint_words, FILL_PER_CHUNK)) : 0;
    }
    case PH_REPLACE:
    case PH_EVICT:  // r->items: the worklist size, summed when the phase before it finished
      return ceil_div(r->items, (uint64_t)WAVES * evict_groups_per_wave(d.t.S));
    case PH_OPS: return ceil_div(d.n, BLOCK);
    default: return 0;
  }
}

// Scalar work at the end of a phase (also for phases with no chunks).
__device__ __forceinline__ void epilogue(volatile ReqState *r, const ReqDesc &d, uint32_t ph) {
  volatile Ctl *c = d.t.ctl;
  switch (ph) {
    case PH_SEG_A:
      if (r->seg_dir > 0) split_segment_done(c, r->seg_sp, r->seg_n);
      break;
    case PH_SEG_B: merge_segment_done(c, r->seg_sp, r->seg_n, c->merge_commit); break;
    case PH_DRAIN: drain_done(c); break;
    default: break;
  }
}

// Shard work at the end of a phase with chunks (wave 0 of the block that
// completed it): after the probe phase the key-count changes are folded and
// the worklist is sized; after a stash drain the worklist is sized; after an
// eviction phase its statistics are folded and the worklist emptied.
// own: this block ran every chunk of the phase, so no other block's writes
// need acquiring.
__device__ __forceinline__ void phase_fold(ReqState *rs, const ReqDesc &d, uint32_t ph, bool own) {
  if (!own) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  volatile ReqState *r = rs;
  Ctl *c = d.t.ctl;
  uint64_t items = 0;
  switch (ph) {
    case PH_OPS: items = fold_shards_wave(c, false); break;
    case PH_DRAIN: items = wave_sum64(ld_ctl(&shard_of(c, threadIdx.x & 63)->wl_count)); break;
    case PH_REPLACE:
    case PH_EVICT: (void)fold_shards_wave(c, true); break;
    default: return;
  }
  if ((threadIdx.x & 63) == 0) r->items = items;  // read by the same thread in advance
}

// Finish phase `ph` of r and publish the next one (one thread).  Returns the
// state word published for that phase, or 0 when the batch is done.
// own: this block ran every chunk of `ph`.  Then a next phase of at most
// SOLO_CHUNKS chunks is published already fully claimed, by this block: a
// small batch runs phase after phase in one block, without a window scan
// and without the acquires (L2 invalidations) of a handoff, since no other
// block writes its data meanwhile.  Each such phase starts with an L1
// invalidation instead (invalidate_l1: the block's own atomics of the last
// phase are not in its L1).  The release before publishing stays (later
// phases read buckets with coherent loads, which must see this block's plain
// stores), and so does the full release when the batch is done.
constexpr uint64_t SOLO_CHUNKS = 4;
__device__ uint64_t advance(DrainQueue *q, ReqState *rs, const ReqDesc &d, uint32_t ph, bool own) {
  if (!own) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  volatile ReqState *r = rs;
  uint64_t nch = 0;
  epilogue(r, d, ph);
  for (;;) {
    ph = successor(r, d, ph);
    if (ph == PH_DONE) break;
    nch = enter(r, d, ph);
    if (nch > 0) break;
    epilogue(r, d, ph);
  }
  r->done = 0;
  if (ph == PH_DONE) {
    const uint64_t ticket = d.ticket;
    __hip_atomic_store(&q->host_live[ticket % q->cap], ld_ctl(&d.t.ctl->live), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();  // the batch's outputs before its completion flag
    __hip_atomic_store(&q->table_next[d.table_slot], d.seq + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&rs->state, make_state(PH_DONE, 0), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&q->host_done[ticket % q->cap], ticket + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    add64(&q->completed, 1);
    return 0;
  }
  const uint64_t published = make_state(ph, nch) + (own && nch <= SOLO_CHUNKS ? nch : 0);
  __threadfence();
  __hip_atomic_store(&rs->state, published, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  return published;
}

// The block that published a batch's next phase claims its first grain at
// once, without a window scan (the batch is running, so its table order is
// already satisfied).  The claim is a CAS from exactly the published state:
// if other blocks have claimed chunks meanwhile it fails and the block scans
// as usual, and a ring slot reused by a later batch cannot match, since a
// published phase is never PH_START.
__device__ bool claim_published(ReqState *r, uint64_t published, uint32_t *phase, uint64_t *chunk, uint64_t *count,
                                uint64_t *nch) {
  const uint64_t n = (published >> 28) & M28;
  const uint64_t grain = max(1ull, n / (2ull * gridDim.x));
  uint64_t expect = published;
  if (!__hip_atomic_compare_exchange_strong(&r->state, &expect, published + min(grain, n), __ATOMIC_ACQUIRE,
                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    return false;
  *phase = (uint32_t)(published >> 56);
  *chunk = 0;
  *count = min(grain, n);
  *nch = n;
  return true;
}

// A value the whole wave holds, in a scalar register (the first active
// lane's copy).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
         __builtin_amdgcn_readfirstlane((uint32_t)v);
}

// Copy new host descriptors into the device ring, by the 64 lanes of one
// wave.  Only the block holding the ingest lock reads host memory (the tail,
// the stop flag, descriptors); every other block polls device memory.  The
// descriptors' words are copied lane-parallel (up to 64 descriptors per
// call): host reads cross the bus, and a one-thread copy of 16 descriptors
// word by word had been hundreds of dependent reads, long enough to be the
// executor's intake limit.  Lane j then publishes descriptor j.  The stop
// flag is read before the tail, so once it is seen set, the tail read after
// it is final.
__device__ void ingest(DrainQueue *q) {
  const int lane = threadIdx.x & 63;
  uint32_t got = 0;
  if (lane == 0 && __hip_atomic_load(&q->ingest_lock, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
    uint32_t expect = 0;
    got = __hip_atomic_compare_exchange_strong(&q->ingest_lock, &expect, 1u, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!__builtin_amdgcn_readfirstlane(got)) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const bool stop = __hip_atomic_load(q->host_stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
  const uint64_t tail = uniform64(ld_sys(q->host_tail));
  const uint64_t i0 = uniform64(ld_ctl(&q->ingested));
  const uint64_t n = min(tail - i0, (uint64_t)64);
  constexpr uint64_t W = sizeof(ReqDesc) / 8;
  for (uint64_t k = lane; k < n * W; k += 64) {
    const uint64_t i = (i0 + k / W) % q->cap, w = k % W;
    ((uint64_t *)&q->req[i].d)[w] = ld_sys((const uint64_t *)(q->host_ring + i) + w);
  }
  ReqState *r = q->req + (i0 + lane) % q->cap;
  if ((uint64_t)lane < n) {
    volatile ReqState *vr = r;
    vr->done = 0;
    vr->aux = 0;
    vr->items = 0;
    vr->resume = PH_DONE;
  }
  __threadfence();  // every lane's descriptor words and fields before any state
  // one START chunk: the batch's first real phase is chosen when it runs,
  // i.e. after every earlier batch on its table has finished
  if ((uint64_t)lane < n)
    __hip_atomic_store(&r->state, make_state(PH_START, 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  __threadfence();  // the states before the new ingest count
  if (lane == 0) {
    __hip_atomic_store(&q->ingested, i0 + n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (stop && i0 + n == tail) __hip_atomic_store(&q->final_seen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&q->ingest_lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Claim a run of chunks of runnable work, by the 64 lanes of one wave: lane
// j looks at ring entry head + j of the window (its state, then whether its
// table's previous batch is done), so a scan costs a few parallel round
// trips instead of a chain of them per entry; the oldest runnable entry is
// claimed first.  `*chunk` is the first chunk, `*count` how many (a phase of
// n chunks is claimed in grains of about n / (2 x grid) chunks, so a large
// phase costs few claims: the atomic on the request's state word is the
// same address for every block); the claiming lane writes the outputs.
// Returns, in every lane, 0 (work), 1 (none now) or 2 (exit).
static_assert(DRAIN_WINDOW == 64, "one window entry per lane");
__device__ uint32_t find_work(DrainQueue *q, uint64_t *req, uint32_t *phase, uint64_t *chunk, uint64_t *count,
                              uint64_t *nch) {
  const int lane = threadIdx.x & 63;
  ingest(q);
  const uint64_t ing = uniform64(ld_ctl(&q->ingested));
  uint64_t head = uniform64(ld_ctl(&q->head));
  // retire the completed batches at the head of the ring
  {
    const uint64_t t = head + lane;
    // relaxed: a retired entry is only skipped; an acquire load here would
    // invalidate the XCD's L2 on every poll of every idle block
    const bool done = t < ing && (__hip_atomic_load(&q->req[t % q->cap].state, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT) >> 56) == PH_DONE;
    const uint64_t dm = ballot(done);
    const int lead = (dm == ~0ull) ? 64 : __builtin_ctzll(~dm);
    if (lead > 0) {
      if (lane == 0) {
        uint64_t h = head;
        __hip_atomic_compare_exchange_strong(&q->head, &h, head + lead, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
      }
      head = uniform64(ld_ctl(&q->head));
    }
  }
  if (head == ing) {
    if (__hip_atomic_load(&q->final_seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 &&
        ld_ctl(&q->ingested) == ing)
      return 2;
    return 1;
  }
  const uint64_t t = head + lane;
  ReqState *r = q->req + t % q->cap;
  uint64_t st = 0;
  bool runnable = false;
  if (t < ing) {
    st = __hip_atomic_load(&r->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    runnable = (uint32_t)(st >> 56) != PH_DONE && (st & M28) < ((st >> 28) & M28);
  }
  // the descriptor read below must see what was written before the state
  // was released; the acquire fence (an L2 invalidate) is paid only by a
  // scan that found unclaimed chunks, never by an idle poll
  if (ballot(runnable)) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (runnable) {
      const uint64_t slot = ld_ctl(&r->d.table_slot), seq = ld_ctl(&r->d.seq);
      runnable = ld_ctl(&q->table_next[slot]) == seq;
    }
  }
  for (uint64_t m = ballot(runnable); m; m &= m - 1) {
    const int j = __builtin_ctzll(m);
    bool won = false;
    if (lane == j) {
      const uint64_t grain = max(1ull, ((st >> 28) & M28) / (2ull * gridDim.x));
      const uint64_t old = add64(&r->state, grain);
      const uint64_t n = (old >> 28) & M28, c = old & M28;
      if ((uint32_t)(old >> 56) != PH_DONE && c < n) {
        won = true;
        *req = t;
        *phase = (uint32_t)(old >> 56);
        *chunk = c;
        *count = min(grain, n - c);
        *nch = n;
      }
    }
    if (ballot(won)) return 0;
  }
  return 1;
}

// Descriptor of the batch a block works on, read coherently into LDS.
__device__ __forceinline__ void load_desc(ReqDesc *dst, const ReqDesc *src) {
  const uint64_t *s = (const uint64_t *)src;
  uint64_t *d = (uint64_t *)dst;
  for (uint32_t w = threadIdx.x; w < sizeof(ReqDesc) / 8; w += BLOCK) d[w] = ld_ctl(s + w);
}

// A pointer the compiler knows to be global memory.  Pointers read from
// memory are generic (flat) to it; rebuilt from their address as global
// ones, their loads and stores become global instructions, which do not
// share the LDS wait counter with the tile staging.
template <typename T>
__device__ __forceinline__ T *as_global(T *p) {
  return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

// The LDS descriptor copied into scalar registers (every word goes through
// readfirstlane, so the compiler knows it is uniform), its buffers marked
// global.  Every buffer a descriptor names is device or mapped host memory.
__device__ __forceinline__ ReqDesc uniform_desc(const ReqDesc &src) {
  uint32_t w[sizeof(ReqDesc) / 4];
  __builtin_memcpy(w, &src, sizeof(ReqDesc));
#pragma unroll
  for (uint32_t i = 0; i < sizeof(ReqDesc) / 4; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  ReqDesc d;
  __builtin_memcpy(&d, w, sizeof(ReqDesc));
  d.t.buckets = as_global(d.t.buckets);
  d.t.hint = as_global(d.t.hint);
  d.t.stash = as_global(d.t.stash);
  d.t.pending = as_global(d.t.pending);
  d.t.ctl = as_global(d.t.ctl);
  d.t.wl = as_global(d.t.wl);
  d.t.dd = as_global(d.t.dd);
  d.ops = as_global(d.ops);
  d.keys = as_global(d.keys);
  d.vals = as_global(d.vals);
  d.vals_out = as_global(d.vals_out);
  d.flags_out = as_global(d.flags_out);
  return d;
}


template <int S>
__device__ __forceinline__ void run_chunk(ReqState *r, const ReqDesc &d, uint32_t ph, uint64_t c, OpsShared<S> &sh) {
  using T = Traits<S>;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / S, sl = lane % S;
  const uint64_t gib = (uint64_t)wv * T::G + g;  // group in block
  const uint64_t gpb = (uint64_t)WAVES * T::G;
  switch (ph) {
    case PH_FILL: {
      const uint64_t b = c * FILL_PER_CHUNK, e = min(b + FILL_PER_CHUNK, d.dd_size);
      for (uint64_t t = b + threadIdx.x; t < e; t += BLOCK) d.t.dd[t] = EMPTY;
      break;
    }
    case PH_DEDUPE: {
      dedupe_thread(d.t.dd, d.dd_size - 1, d.mode, d.ops, d.keys, d.n, c * BLOCK + threadIdx.x);
      break;
    }
    case PH_COUNT: {
      __shared__ unsigned long long cnt;
      if (threadIdx.x == 0) cnt = 0;
      __syncthreads();
      unsigned long long mine = 0;
      const uint64_t b = c * COUNT_PER_CHUNK, e = min(b + COUNT_PER_CHUNK, d.n);
      for (uint64_t t = b + threadIdx.x; t < e; t += BLOCK) mine += d.ops[t] == OP_INSERT;
      atomicAdd(&cnt, mine);
      __syncthreads();
      if (threadIdx.x == 0 && cnt) add64(&r->aux, cnt);
      break;
    }
    case PH_SEG_A: {
      const ResizeArgs ra = resize_args(d);
      const uint64_t j = c * gpb + gib, n = ld_ctl(&r->seg_n);
      const uint64_t im = ld_ctl(&r->seg_im), sp = ld_ctl(&r->seg_sp);
      if (j < n) {
        if ((int64_t)ld_ctl((const uint64_t *)&r->seg_dir) > 0)
          split_pair<S>(ra, im, sp, j, g, sl);
        else
          merge_test_pair<S>(ra, d.t.ctl, im, sp, j, g, sl);
      }
      break;
    }
    case PH_SEG_B: {
      const ResizeArgs ra = resize_args(d);
      const uint64_t j = c * gpb + gib, commit = ld_ctl(&d.t.ctl->merge_commit);
      if (j < commit) merge_move_pair<S>(ra, ld_ctl(&r->seg_im), ld_ctl(&r->seg_sp), j, g, sl);
      break;
    }
    case PH_DRAIN: {
      const Ctl *cc = d.t.ctl;
      const uint64_t n_stash = min(ld_ctl(&cc->stash_count), d.t.stash_cap) ? stash_slots_for(d.t.stash_cap) : 0;
      const uint64_t total = n_stash + min(ld_ctl(&cc->pending_count), d.t.pending_cap);
      const uint64_t hb = c * FILL_PER_CHUNK, he = min(hb + FILL_PER_CHUNK, d.t.hint_words);
      for (uint64_t t = hb + threadIdx.x; t < he; t += BLOCK) d.t.hint[t] = 0u;
      for (uint64_t k = 0; k < DRAIN_TILES; ++k)
        drain_collect((c * DRAIN_TILES + k) * BLOCK + threadIdx.x, n_stash, total, d.t.stash, d.t.pending, d.t.wl,
                      d.t.wl_seg_cap, d.t.ctl);
      break;
    }
    case PH_REPLACE:
    case PH_EVICT: {
      using E = EvictShape<S>;
      __shared__ uint64_t pre[NSHARD + 1];
      const EvictArgs ea = evict_args(d);
      wl_prefix(d.t.ctl, pre);
      const Geo geo = read_geo(d.t.ctl);
      const uint64_t items = pre[NSHARD];
      const int eg = lane / E::L, esl = lane % E::L;
      const uint64_t egpb = (uint64_t)WAVES * E::G, egib = (uint64_t)wv * E::G + eg;
      uint64_t n_evict = 0, n_full = 0, n_side = 0, n_fresh = 0;
      const uint64_t t = c * egpb + egib;
      const bool unreserved = ld_ctl(&d.t.ctl->stash_count) + items <= d.t.stash_cap;
      evict_round<S>(ea, geo, unreserved, t < items, t < items ? wl_slot(pre, t, d.t.wl_seg_cap) : 0, eg, esl, n_evict,
                     n_full, n_side, n_fresh);
      evict_counters(ea, unreserved, c * WAVES + wv, n_evict, n_full, n_side, n_fresh, esl);
      break;
    }
    case PH_OPS: {
      OpsArgs a{};
      a.buckets = d.t.buckets;
      a.hint = d.t.hint;
      a.stash = d.t.stash;
      a.pending = d.t.pending;
      a.ctl = d.t.ctl;
      a.wl = d.t.wl;
      a.wl_seg_cap = d.t.wl_seg_cap;
      a.dd = d.dd_size ? d.t.dd : nullptr;
      a.dd_mask = d.dd_size ? d.dd_size - 1 : 0;
      a.ops = d.ops;
      a.keys = d.keys;
      a.vals = d.vals;
      a.vals_out = d.vals_out;
      a.flags_out = d.flags_out;
      a.n = d.n;
      a.stash_cap = d.t.stash_cap;
      a.pending_cap = d.t.pending_cap;
      const OpsView view = read_view(d.t.ctl, d.t.stash_cap, d.t.pending_cap);
      // one probe variant only (the second candidate after a miss): a
      // second inlined copy would cost the resident grid occupancy
      int64_t live_acc = 0;
      uint64_t bad_acc = 0;
      switch (d.mode) {
        case OP_INSERT: ops_tile<S, OP_INSERT, false>(a, view, c, sh, live_acc, bad_acc); break;
        case OP_DELETE: ops_tile<S, OP_DELETE, false>(a, view, c, sh, live_acc, bad_acc); break;
        case OP_LOOKUP: ops_tile<S, OP_LOOKUP, false>(a, view, c, sh, live_acc, bad_acc); break;
        default: ops_tile<S, OP_MIXED, false>(a, view, c, sh, live_acc, bad_acc); break;
      }
      ops_counts_add(d.t.ctl, c * WAVES + (threadIdx.x >> 6), live_acc, bad_acc);
      break;
    }
    default: break;  // PH_START: no data-parallel work
  }
}

__global__ void drain_reset_kernel(DrainQueue *q) { q->final_seen = 0; }

// One reading of the constant-rate device clock (clock-rate calibration).
__global__ void wall_clock_kernel(uint64_t *out) { *out = wall_clock64(); }

// Invalidate this compute unit's vector L1 cache (the L2 is untouched).
// An agent-scope acquire fence does this and also invalidates the XCD's L2
// lines of non-coherent memory types; a block that runs consecutive phases of
// one batch alone needs only the former: its own device-scope atomics
// (claims, evictions, stash placements) were performed in its XCD's L2, but
// lines its earlier plain loads brought into the L1 still hold the words
// those atomics replaced, and the next phase's plain loads (split, merge,
// stash drain, probe) would read them.
__device__ __forceinline__ void invalidate_l1() { asm volatile("buffer_inv sc0" ::: "memory"); }

// Occupancy target: 3 waves per SIMD (at most 168 VGPRs).  The 16-slot build
// spills three registers of the control loop, none inside a phase; a cap of
// 128 (4 waves) spills inside the phases and runs slower.
template <int S>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3))) void drain_worker_kernel(DrainQueue *q) {
  __shared__ OpsShared<S> sh;
  __shared__ ReqDesc desc;
  __shared__ uint64_t s_req, s_chunk, s_cnt, s_nch;
  __shared__ uint32_t s_phase, s_cmd;
  __shared__ bool s_last, s_cont, s_solo;
  // watchdog (thread 0 decides for the block): time without any progress
  // of the queue as a whole (nothing newly ingested, nothing retired), so
  // blocks that merely find no chunk while others work do not give up
  uint64_t seen_ing = ~0ull, seen_head = ~0ull;
  uint64_t idle_since = wall_clock64();
  const uint64_t idle_ticks = ld_ctl(&q->idle_ticks);
  if (threadIdx.x == 0) {
    s_cont = false;
    s_solo = false;
  }
  __syncthreads();
  for (;;) {
    // s_cont: this block claimed the next phase of its batch when it
    // published it, so it needs no scan
    if (threadIdx.x < 64 && !s_cont) {
      uint32_t cmd = find_work(q, &s_req, &s_phase, &s_chunk, &s_cnt, &s_nch);
      if (threadIdx.x == 0 && cmd == 1) {
        const uint64_t ing = ld_ctl(&q->ingested), head = ld_ctl(&q->head);
        const uint64_t now = wall_clock64();
        if (ing != seen_ing || head != seen_head) {
          seen_ing = ing;
          seen_head = head;
          idle_since = now;
        }
        if (now - idle_since > idle_ticks) {
          atomicOr(&q->error, 1u);
          cmd = 2;
        }
      }
      if (threadIdx.x == 0) s_cmd = cmd;
    }
    __syncthreads();
    const uint32_t cmd = s_cont ? 0u : s_cmd;
    if (cmd == 2) break;
    if (cmd == 1) {
      __builtin_amdgcn_s_sleep(7);  // about 450 clocks
      __syncthreads();
      continue;
    }
    ReqState *r = q->req + s_req % q->cap;
    // s_solo: this block also ran the batch's previous phases alone since it
    // last acquired, and its descriptor is still in LDS
    if (!s_solo) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      load_desc(&desc, &r->d);
      __syncthreads();
    } else {
      invalidate_l1();
    }
    const ReqDesc d = uniform_desc(desc);
    const uint32_t phase = __builtin_amdgcn_readfirstlane(s_phase);
    const uint64_t chunk = uniform64(s_chunk), cnt = uniform64(s_cnt);
    for (uint64_t k = 0; k < cnt; ++k) {
      run_chunk<S>(r, d, phase, chunk + k, sh);
      __syncthreads();
    }
    const bool own = cnt == uniform64(s_nch);  // every chunk of the phase ran here
    if (threadIdx.x == 0) {
      if (s_solo) {
        s_last = true;  // the phase was published claimed by this block
      } else {
        __threadfence();  // these chunks' writes before their completion count
        s_last = add64(&r->done, s_cnt) + s_cnt == s_nch;
      }
      s_cont = false;
      s_solo = false;
    }
    __syncthreads();
    if (s_last) {
      // the block that completed the phase: shard folds by wave 0, then the
      // scalar epilogue and the next phase by thread 0, which claims the
      // start of that phase for this block
      if (threadIdx.x < 64) phase_fold(r, desc, phase, own);
      __syncthreads();
      if (threadIdx.x == 0) {
        const uint64_t published = advance(q, r, desc, phase, own);
        const uint64_t n = (published >> 28) & M28;
        if (published != 0 && (published & M28) == n) {  // published claimed by this block
          s_phase = (uint32_t)(published >> 56);
          s_chunk = 0;
          s_cnt = n;
          s_nch = n;
          s_cont = true;
          s_solo = true;
        } else {
          s_cont = published != 0 && claim_published(r, published, &s_phase, &s_chunk, &s_cnt, &s_nch);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 32-bit entries: a key-only set (Section III-A: with 32-bit entries a
// 32-slot bucket is one 128-byte line).  The entry is the key itself; EMPTY
// is 0xFFFFFFFF and a deleted stash or pending entry is 0 (both reserved
// keys).  The steps are those of the 64-bit table: P1 hashes, probes the
// first candidate (a 32-lane group per bucket, one 4-byte load per lane, two
// buckets per wave-wide load), the second after a miss, then looks up,
// deletes (one agent-scope atomic store of EMPTY) or inserts: a key already
// present is left as it is (there is no value to replace), a new one claims
// the lowest EMPTY slot of the emptier candidate by a 32-bit CAS; P3 runs
// the bounded cuckoo chains one lane per item on fresh copies of whole
// buckets, then the stash or the pending list.  FIXED addressing, BitHash1/2,
// plain launches.
// ---------------------------------------------------------------------------
constexpr uint32_t EMPTY32 = 0xFFFFFFFFu;
constexpr uint32_t TOMB32 = 0u;
constexpr int SET_S = 32;        // slots per bucket
constexpr int SET_CH = 16;       // wave-wide bucket loads in flight

struct SetArgs {
  uint32_t *buckets;
  uint32_t *hint;
  uint32_t *stash;
  uint32_t *pending;
  Ctl *ctl;
  uint64_t *wl;  // eviction worklist (keys widened to 64 bits), NSHARD segments
  uint64_t wl_seg_cap;
  const uint64_t *dd;  // dedupe set, or null
  uint64_t dd_mask;
  const uint8_t *ops;
  const uint32_t *keys;
  uint8_t *flags_out;
  uint64_t n;
  uint64_t stash_cap, pending_cap;
  uint32_t max_evictions;
  const uint8_t *win;  // dedupe winner flag per operation, or null
};

__device__ __forceinline__ uint32_t cas32(uint32_t *p, uint32_t expected, uint32_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;
}

// Search of the stash (open-addressed, linear probing from mix32(key), ends
// at EMPTY) and the pending list.
__device__ __forceinline__ uint32_t *set_overflow_find(const SetArgs &a, uint64_t n_stash, uint64_t n_pend,
                                                       uint32_t k) {
  if (n_stash) {
    const uint64_t mask = stash_slots_for(a.stash_cap) - 1;
    for (uint64_t i = 0, p = mix32(k) & mask; i <= mask; ++i, p = (p + 1) & mask) {
      const uint32_t x = a.stash[p];
      if (x == EMPTY32) break;
      if (x == k) return a.stash + p;
    }
  }
  for (uint64_t p = 0; p < n_pend; ++p)
    if (a.pending[p] == k) return a.pending + p;
  return nullptr;
}

// One probe round: operations t < count have key keys[t] and bucket
// bkts[t] (owner list[t], or t itself); each 32-lane group loads one bucket
// per wave-wide load and publishes the match and EMPTY masks to the owner.
// bkts[] holds 64 entries, padded from `count` on with a bucket loaded
// anyway.
__device__ __forceinline__ void set_probe_round(const uint32_t *__restrict__ buckets, const uint32_t *keys,
                                                const uint32_t *bkts, const uint8_t *list, int count,
                                                uint32_t *m_out, uint32_t *e_out, int g, int sl) {
  for (int base = 0; base < count; base += 2 * SET_CH) {
    uint32_t w[SET_CH];
#pragma unroll
    for (int j = 0; j < SET_CH; ++j) w[j] = buckets[(uint64_t)bkts[base + 2 * j + g] * SET_S + sl];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < SET_CH; ++j) {
      const int t = base + 2 * j + g;
      const bool mine = t < count;
      const uint32_t ko = keys[t];
      const uint64_t mm = ballot(mine && ko != 0u && w[j] == ko);
      const uint64_t ee = ballot(w[j] == EMPTY32);
      if (mine && sl == 0) {
        const int o = list ? list[t] : t;
        m_out[o] = (uint32_t)(mm >> (g * 32));
        e_out[o] = (uint32_t)(ee >> (g * 32));
      }
    }
  }
}

template <uint32_t MODE>
__global__ __launch_bounds__(BLOCK) void set_ops_kernel(SetArgs a) {
  __shared__ uint32_t s_key[WAVES][64], s_b1[WAVES][64], s_k2[WAVES][64], s_b2[WAVES][64];
  __shared__ uint8_t s_list[WAVES][64];
  __shared__ uint32_t s_m[2][WAVES][64], s_e[2][WAVES][64];
  const Geo geo = read_geo(a.ctl);
  const uint64_t n_stash = min(ld_ctl(&a.ctl->stash_count), a.stash_cap);
  const uint64_t n_pend = min(ld_ctl(&a.ctl->pending_count), a.pending_cap);
  const bool overflow_used = (n_stash | n_pend) != 0;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 5, sl = lane & 31;
  const uint64_t ntiles = (a.n + BLOCK - 1) / BLOCK;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t i = tile * BLOCK + threadIdx.x;
    const bool active = i < a.n;
    uint32_t op = OP_NONE, k = 0;
    if (active) {
      op = (MODE == OP_MIXED) ? (uint32_t)__builtin_nontemporal_load(&a.ops[i]) : MODE;
      k = __builtin_nontemporal_load(&a.keys[i]);
    }
    const bool valid = active && op <= OP_LOOKUP && valid_key(k);
    bool work = valid;
    if (work && op != OP_LOOKUP) {
      if (a.win)
        work = __builtin_nontemporal_load(&a.win[i]) != 0;
      else if (a.dd)
        work = dedupe_winner(a.dd, a.dd_mask, k, (uint32_t)i);
    }
    uint32_t c1 = 0, c2 = 0;
    if (work) {
      c1 = fastmod(bithash1(k), geo.magic, (uint32_t)geo.n_buckets);
      c2 = fastmod(bithash2(k), geo.magic, (uint32_t)geo.n_buckets);
    }
    s_key[wv][lane] = work ? k : 0u;
    s_b1[wv][lane] = c1;
    wave_lds_sync();
    set_probe_round(a.buckets, s_key[wv], s_b1[wv], nullptr, 64, s_m[0][wv], s_e[0][wv], g, sl);
    wave_lds_sync();
    const uint32_t m1 = s_m[0][wv][lane], e1 = s_e[0][wv][lane];
    const bool need2 = work && m1 == 0 && c2 != c1;
    const uint64_t need2_mask = ballot(need2);
    const int n2 = __popcll(need2_mask);
    compact_second(need2, need2_mask, n2, k, c2, c1, lane, s_k2[wv], s_b2[wv], s_list[wv]);
    wave_lds_sync();
    if (n2 > 0) set_probe_round(a.buckets, s_k2[wv], s_b2[wv], s_list[wv], n2, s_m[1][wv], s_e[1][wv], g, sl);
    wave_lds_sync();
    const uint32_t m2 = need2 ? s_m[1][wv][lane] : 0u, e2 = need2 ? s_e[1][wv][lane] : 0u;

    uint8_t out_f = 0;
    int dl = 0;
    bool to_wl = false;
    if (work) {
      uint32_t *slot = nullptr;
      bool in_bucket = false;
      if (m1) {
        slot = a.buckets + (uint64_t)c1 * SET_S + __builtin_ctz(m1);
        in_bucket = true;
      } else if (m2) {
        slot = a.buckets + (uint64_t)c2 * SET_S + __builtin_ctz(m2);
        in_bucket = true;
      } else if (overflow_used && hinted(a.hint, c1, c2)) {
        slot = set_overflow_find(a, n_stash, n_pend, k);
      }
      if (op == OP_LOOKUP) {
        out_f = slot != nullptr;
      } else if (op == OP_DELETE) {
        if (slot && in_bucket) {
          // an atomic store: claims of other XCDs change this line in the
          // same launch (see the 64-bit table's delete)
          __hip_atomic_store(slot, EMPTY32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          out_f = 1;
          dl = -1;
        } else if (slot && cas32(slot, k, TOMB32) == k) {
          out_f = 1;
          dl = -1;
        }
      } else if (!slot) {
        // a new key: claim-then-commit in the emptier candidate first
        dl = 1;
        uint32_t f_first = e1, f_second = (c2 != c1) ? e2 : 0u, b_first = c1, b_second = c2;
        if (__builtin_popcount(f_second) > __builtin_popcount(f_first)) {
          const uint32_t tf = f_first;
          f_first = f_second;
          f_second = tf;
          b_first = c2;
          b_second = c1;
        }
        bool placed = false;
        while (!placed && (f_first | f_second)) {
          if (f_first == 0) {
            f_first = f_second;
            f_second = 0;
            b_first = b_second;
          }
          const int s = __builtin_ctz(f_first);
          if (cas32(a.buckets + (uint64_t)b_first * SET_S + s, EMPTY32, k) == EMPTY32)
            placed = true;
          else
            f_first &= f_first - 1;
        }
        to_wl = !placed;
      }
    }
    const uint64_t wl_mask = ballot(to_wl);
    if (wl_mask) {
      const int leader = __builtin_ctzll(wl_mask);
      uint64_t base = 0;
      if (lane == leader) base = wl_append(a.ctl, tile, (uint64_t)__popcll(wl_mask));
      base = read_lane64(base, leader);
      if (to_wl) a.wl[(tile % NSHARD) * a.wl_seg_cap + base + rank_below(wl_mask)] = k;
    }
    const uint64_t up = ballot(dl > 0), down = ballot(dl < 0), bad = ballot(active && !valid);
    if (lane == 0) {
      Shard *sh = shard_of(a.ctl, (tile * WAVES + wv) % NSHARD);
      const int64_t d = (int64_t)__popcll(up) - (int64_t)__popcll(down);
      if (d != 0) add64(&sh->live, (uint64_t)d);
      if (bad) add64(&sh->invalid_keys, (uint64_t)__popcll(bad));
    }
    if (active && MODE != OP_INSERT && a.flags_out) __builtin_nontemporal_store(out_f, &a.flags_out[i]);
  }
}

// A lane's fresh copy of a whole 32-slot bucket (128 bytes).
__device__ __forceinline__ uint32_t load_set_bucket(const uint32_t *bkt, uint32_t *w) {
  uint64_t x[16];
  load_bucket16_fresh((const uint64_t *)bkt, x);
  uint32_t free_mask = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    w[2 * j] = (uint32_t)x[j];
    w[2 * j + 1] = (uint32_t)(x[j] >> 32);
  }
#pragma unroll
  for (int j = 0; j < SET_S; ++j) free_mask |= (uint32_t)(w[j] == EMPTY32) << j;
  return free_mask;
}

__device__ __forceinline__ bool set_claim(uint32_t *bkt, uint32_t free_mask, uint32_t k) {
  for (; free_mask; free_mask &= free_mask - 1)
    if (cas32(bkt + __builtin_ctz(free_mask), EMPTY32, k) == EMPTY32) return true;
  return false;
}

// Step 4: the first EMPTY or TOMB word of the key's stash run (given a
// reserved position c < capacity), else the pending list.  Returns 0 stash
// (EMPTY word), 3 stash (TOMB word), 1 pending, 2 lost.
__device__ __forceinline__ int set_overflow_place(const SetArgs &a, const Geo &geo, uint32_t k, uint64_t c) {
  int where = -1;
  if (c < a.stash_cap) {
    const uint64_t mask = stash_slots_for(a.stash_cap) - 1;
    for (uint64_t i = 0, p = mix32(k) & mask; i <= mask; ++i, p = (p + 1) & mask) {
      const uint32_t cur = cas32(a.stash + p, EMPTY32, k);
      if (cur == EMPTY32) {
        where = 0;
        break;
      }
      if (cur == TOMB32 && cas32(a.stash + p, TOMB32, k) == TOMB32) {
        where = 3;
        break;
      }
    }
  }
  if (where < 0) {
    const uint64_t p = add64(&a.ctl->pending_count, 1);
    if (p < a.pending_cap) {
      __hip_atomic_store(a.pending + p, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      where = 1;
    } else {
      atomicOr(&a.ctl->error, ERR_PENDING_LOST);
      where = 2;
    }
  }
  set_hint(a.hint, fastmod(bithash1(k), geo.magic, (uint32_t)geo.n_buckets));
  set_hint(a.hint, fastmod(bithash2(k), geo.magic, (uint32_t)geo.n_buckets));
  return where;
}

// P3 of the set: one lane per worklist item, as the 64-bit table's 16-slot
// eviction shape (Algorithm 3 with a pseudo-random victim slot).
__global__ __launch_bounds__(BLOCK) void set_evict_kernel(SetArgs a) {
  __shared__ uint64_t pre[NSHARD + 1];
  wl_prefix(a.ctl, pre);
  const uint64_t cnt = pre[NSHARD];
  if (cnt == 0) return;
  const Geo geo = read_geo(a.ctl);
  const bool unreserved = ld_ctl(&a.ctl->stash_count) + cnt <= a.stash_cap;
  const int lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  const uint32_t nb = (uint32_t)geo.n_buckets;
  uint64_t n_evict = 0, n_full = 0, n_side = 0, n_fresh = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * BLOCK + (threadIdx.x & ~63u); base < cnt; base += stride) {
    const uint64_t t = base + lane;
    bool placed = true;
    uint32_t k = 0;
    if (t < cnt) {
      k = (uint32_t)a.wl[wl_slot(pre, t, a.wl_seg_cap)];
      const uint32_t c1 = fastmod(bithash1(k), geo.magic, nb), c2 = fastmod(bithash2(k), geo.magic, nb);
      uint32_t w[SET_S];
      const uint32_t f1 = load_set_bucket(a.buckets + (uint64_t)c1 * SET_S, w);
      const uint32_t f2 = c2 != c1 ? load_set_bucket(a.buckets + (uint64_t)c2 * SET_S, w) : 0u;
      if (__builtin_popcount(f2) > __builtin_popcount(f1))
        placed = set_claim(a.buckets + (uint64_t)c2 * SET_S, f2, k) ||
                 set_claim(a.buckets + (uint64_t)c1 * SET_S, f1, k);
      else
        placed = set_claim(a.buckets + (uint64_t)c1 * SET_S, f1, k) ||
                 set_claim(a.buckets + (uint64_t)c2 * SET_S, f2, k);
      uint32_t b = c1;
      for (uint32_t kick = 1; kick <= a.max_evictions && !placed; ++kick) {
        uint32_t *bkt = a.buckets + (uint64_t)b * SET_S;
        const uint32_t fm = load_set_bucket(bkt, w);
        if (set_claim(bkt, fm, k)) {
          placed = true;
          break;
        }
        const int s0 = (int)(mix32(k ^ (kick * 0x9E3779B9u)) & (SET_S - 1));
        uint32_t ws = 0;
#pragma unroll
        for (int j = 0; j < SET_S; ++j)
          if (j == s0) ws = w[j];
        if (cas32(bkt + s0, ws, k) != ws) continue;  // the slot changed: count the round, keep the key
        if (ws == EMPTY32) {
          placed = true;
          break;
        }
        ++n_evict;
        k = ws;
        const uint32_t v1 = fastmod(bithash1(k), geo.magic, nb), v2 = fastmod(bithash2(k), geo.magic, nb);
        b = (b == v1) ? v2 : v1;
      }
    }
    const bool push = !placed;
    const uint64_t pm = ballot(push);
    if (pm) {
      const int leader = __builtin_ctzll(pm);
      uint64_t room = 0;
      if (!unreserved) {
        if (lane == leader) {
          const uint64_t nn = (uint64_t)__popcll(pm);
          room = load_fresh(&a.ctl->stash_count) < a.stash_cap ? add64(&a.ctl->stash_count, nn) : a.stash_cap;
        }
        room = read_lane64(room, leader);
      }
      if (push) {
        ++n_full;
        const int where = set_overflow_place(a, geo, k, room + rank_below(pm));
        n_side += (where == 0 || where == 3) ? 1 : where == 1 ? (1ull << 32) : 0;
        n_fresh += where == 0;
      }
    }
  }
  const uint64_t e = wave_sum64(n_evict), f = wave_sum64(n_full), sd = wave_sum64(n_side), fr = wave_sum64(n_fresh);
  if (lane == 0 && (e | f | sd)) {
    Shard *sh = shard_of(a.ctl, ((uint64_t)blockIdx.x * WAVES + (threadIdx.x >> 6)) % NSHARD);
    if (e) add64(&sh->evictions, e);
    if (f) add64(&sh->full_chains, f);
    if ((uint32_t)sd) add64(&sh->stash_inserts, (uint32_t)sd);
    if (fr && unreserved) add64(&sh->stash_unreserved, fr);
    if (sd >> 32) add64(&sh->pending_inserts, sd >> 32);
  }
}

// Every live key of the set as a 64-bit word (value half 0) with its place.
__global__ __launch_bounds__(BLOCK) void set_dump_kernel(const uint32_t *buckets, const uint32_t *stash,
                                                         const uint32_t *pending, Ctl *ctl, uint64_t stash_cap,
                                                         uint64_t pending_cap, uint64_t *out, int64_t *where,
                                                         uint64_t cap) {
  const uint64_t nb = ctl->n_buckets;
  const uint64_t n_stash = min(ctl->stash_count, stash_cap) ? stash_slots_for(stash_cap) : 0;
  const uint64_t n_pend = min(ctl->pending_count, pending_cap);
  const uint64_t n_slots = nb * SET_S, total = n_slots + n_stash + n_pend;
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  const uint64_t span = (total + stride - 1) / stride * stride;
  const int lane = threadIdx.x & 63;
  for (uint64_t t = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; t < span; t += stride) {
    uint32_t w = EMPTY32;
    int64_t pl = 0;
    if (t < n_slots) {
      w = buckets[t];
      pl = (int64_t)(t / SET_S);
    } else if (t < n_slots + n_stash) {
      w = stash[t - n_slots];
      pl = -1;
    } else if (t < total) {
      w = pending[t - n_slots - n_stash];
      pl = -2;
    }
    const bool live = t < total && w != EMPTY32 && w != TOMB32;
    const uint64_t m = ballot(live);
    if (m) {
      const int leader = __builtin_ctzll(m);
      uint64_t base = 0;
      if (lane == leader) base = add64(&ctl->dump_count, (uint64_t)__popcll(m));
      base = read_lane64(base, leader);
      const uint64_t pos = base + rank_below(m);
      if (live && pos < cap) {
        out[pos] = w;
        if (where) where[pos] = pl;
      }
    }
  }
}

}  // namespace hive

// ===========================================================================
// Host side: the C ABI
// ===========================================================================
using namespace hive;

struct hive_table {
  hive_config cfg;
  uint32_t S;
  uint32_t entry_bytes = 8;  // 4: a key-only set of 32-bit entries
  uint64_t initial_buckets;
  uint64_t max_buckets;
  uint64_t stash_cap, pending_cap;
  uint64_t *d_buckets = nullptr;
  uint32_t *d_hint = nullptr;
  uint64_t *d_stash = nullptr;
  uint64_t *d_pending = nullptr;
  Ctl *d_ctl = nullptr;
  uint64_t *d_wl = nullptr;
  uint64_t wl_cap = 0;      // operations per batch the worklist is sized for
  uint64_t wl_seg_cap = 0;  // entries per worklist segment (NSHARD segments)
  uint64_t *d_dd = nullptr;
  uint64_t dd_cap = 0;  // power of two
  uint64_t bytes = 0;
  hipStream_t last = nullptr;
  // phase timing (hive_phase_timing): events at phase boundaries, spans
  // [a, b) of one phase group each, waiting to be read
  struct Span {
    int kind;
    hipEvent_t a, b;
  };
  bool timing = false;
  int open_kind = -1;
  hipEvent_t open_ev = nullptr;
  std::vector<Span> spans;
  std::vector<hipEvent_t> free_events;
  std::vector<hipEvent_t> all_events;
};

struct hive_drain {
  uint32_t S = 16;
  uint64_t cap = 0;
  uint32_t max_tables = 0;
  unsigned grid[2] = {0, 0};  // blocks of a launch: [0] draining, [1] resident
  int fit_per_cu = 0;         // worker blocks that fit one CU (occupancy query)
  DrainQueue *d_q = nullptr;
  ReqState *d_req = nullptr;
  uint64_t *d_table_next = nullptr;
  ReqDesc *h_ring = nullptr;
  uint64_t *h_tail = nullptr;
  uint32_t *h_stop = nullptr;
  uint64_t *h_done = nullptr;
  uint64_t *h_live = nullptr;
  uint64_t submitted = 0;
  // per registered table: its slot in table_next and its next sequence number
  hive_table *tables[4096];
  uint64_t next_seq[4096];
  uint32_t n_tables = 0;
  hipStream_t capture = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipStream_t running_on = nullptr;
  bool running = false;
};

#define HIP_OK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      fprintf(stderr, "hive: %s failed: %s (%s:%d)\n", #expr, hipGetErrorString(e_), __FILE__, \
              __LINE__);                                                                    \
      return HIVE_ERR_HIP;                                                                  \
    }                                                                                       \
  } while (0)

static hive_status launch_check() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    fprintf(stderr, "hive: kernel launch failed: %s\n", hipGetErrorString(e));
    return HIVE_ERR_HIP;
  }
  return HIVE_OK;
}

static unsigned grid_for(uint64_t n, uint64_t per_block, unsigned cap) {
  uint64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

static Ctl initial_ctl(const hive_table *h) {
  Ctl c;
  memset(&c, 0, sizeof(c));
  c.n_buckets = h->initial_buckets;
  c.mode = h->cfg.addressing;
  if (h->cfg.addressing == HIVE_FIXED) {
    c.magic = fastmod_magic((uint32_t)h->initial_buckets);
  } else {
    uint64_t p = 1;
    while (p * 2 <= h->initial_buckets) p *= 2;
    c.im = p - 1;
    c.sp = h->initial_buckets - p;
  }
  c.initial_buckets = h->initial_buckets;
  c.max_buckets = h->max_buckets;
  return c;
}

static hive_status fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t st) {
  if (n == 0) return HIVE_OK;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n, BLOCK * 8ull, 65535)), dim3(BLOCK), 0, st, p, n, v);
  return launch_check();
}

static hive_status fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return HIVE_OK;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, BLOCK * 8ull, 65535)), dim3(BLOCK), 0, st, p, n, v);
  return launch_check();
}

static uint64_t hint_words(uint64_t buckets) { return (buckets + 31) / 32; }

static hive_status reset_table(hive_table *h, hipStream_t st) {
  hive_status s;
  if ((s = fill_u64(h->d_buckets, h->max_buckets * h->S * h->entry_bytes / 8, EMPTY, st)) != HIVE_OK) return s;
  if ((s = fill_u32(h->d_hint, hint_words(h->max_buckets), 0u, st)) != HIVE_OK) return s;
  if ((s = fill_u64(h->d_stash, stash_slots_for(h->stash_cap) * h->entry_bytes / 8, EMPTY, st)) != HIVE_OK) return s;
  if ((s = fill_u64((uint64_t *)shard_of(h->d_ctl, 0), NSHARD * SHARD_STRIDE / 8, 0, st)) != HIVE_OK) return s;
  hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(1), 0, st, h->d_ctl, initial_ctl(h));
  return launch_check();
}

static void free_table(hive_table *h) {
  if (!h) return;
  for (hipEvent_t e : h->all_events) (void)hipEventDestroy(e);
  (void)hipFree(h->d_buckets);
  (void)hipFree(h->d_hint);
  (void)hipFree(h->d_stash);
  (void)hipFree(h->d_pending);
  (void)hipFree(h->d_ctl);
  (void)hipFree(h->d_wl);
  (void)hipFree(h->d_dd);
  delete h;
}

static hive_status alloc(void **p, uint64_t bytes, uint64_t *total) {
  const hipError_t e = hipMalloc(p, bytes ? bytes : 8);
  if (e != hipSuccess) {
    fprintf(stderr, "hive: hipMalloc of %llu bytes failed: %s\n", (unsigned long long)bytes, hipGetErrorString(e));
    (void)hipGetLastError();
    *p = nullptr;
    return HIVE_ERR_OOM;
  }
  *total += bytes;
  return HIVE_OK;
}

// Per-batch scratch (worklist and dedupe set) grows on demand; growing
// synchronizes the stream because the old buffers may still be in use.
// Entries per worklist segment for batches of up to n operations (or stash
// drains of up to n entries): tile t of 256 appends to segment t % NSHARD,
// at most 256 entries from each of ceil(tiles / NSHARD) tiles.
static uint64_t wl_seg_cap_for(uint64_t n) {
  const uint64_t tiles = (n + BLOCK - 1) / BLOCK;
  return std::max<uint64_t>(1, (tiles + NSHARD - 1) / NSHARD) * BLOCK;
}

// n_wl: operations (or drained entries) that may reach the eviction worklist;
// n_dd: operations the dedupe set must hold (0: none).  The set is sized
// from the whole batch, not from its inserts: a delete batch sends nothing
// to the worklist but records every operation in the set.
static uint64_t dd_set_words(uint64_t n) {  // the executor's open-addressed dedupe set
  uint64_t want = 16;
  while (want < 2 * n) want <<= 1;
  return want;
}

// The partitioned dedupe's buffers for a batch of n operations with nt types,
// carved from one scratch allocation (each piece 256-byte aligned).
static uint64_t ddp_layout(uint64_t *base, uint64_t n, uint32_t nt, DdpArgs *d) {
  const uint64_t nch = (n + DD_CHUNK - 1) / DD_CHUNK, nseg = (nch + DDP_SEG - 1) / DDP_SEG;
  auto words = [](uint64_t bytes) { return (bytes + 255) / 256 * 32; };
  uint64_t at = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t w = at;
    at += words(bytes);
    return base ? base + w : nullptr;
  };
  uint64_t *stage = take((uint64_t)std::max<uint32_t>(nt, 2) * nch * DD_CHUNK * 8);
  uint64_t *rec = take(n * 8);
  uint64_t *win = take(nch * DD_CHUNK);
  uint64_t *hist = take((uint64_t)nt * nch * DDP_BINS * 2);
  uint64_t *cnt = take((uint64_t)nt * nch * 4);
  uint64_t *seg = take((uint64_t)nt * nseg * DDP_BINS * 4);
  uint64_t *tot = take((uint64_t)nt * DDP_BINS * 4);
  if (d) {
    d->n = n;
    d->nch = nch;
    d->nseg = nseg;
    d->nt = nt;
    d->stage = stage;
    d->rec = rec;
    d->win = (uint8_t *)win;
    d->hist = (uint16_t *)hist;
    d->cnt = (uint32_t *)cnt;
    d->seg = (uint32_t *)seg;
    d->tot = (uint32_t *)tot;
  }
  return at;
}

// Words of the dedupe scratch for n operations: the partitioned dedupe of
// plain launches (mixed batches: two types) or the executor's set.
static uint64_t dd_words_for(uint64_t n) { return std::max(dd_set_words(n), ddp_layout(nullptr, n, 2, nullptr)); }

// Worklist entries a stash drain may append: the whole stash table and the
// pending list.
static uint64_t drain_words(const hive_table *h) { return stash_slots_for(h->stash_cap) + h->pending_cap; }

// Added to a worklist that holds a batch's entries and a drain: the probe
// launch's and the drain's per-segment fills are each bounded by their own
// rounding of whole tiles per segment, which can exceed the rounding of the
// sum by up to 4 x NSHARD tiles in all.
constexpr uint64_t WL_SLACK = 4ull * NSHARD * BLOCK;

static hive_status ensure_scratch(hive_table *h, uint64_t n, uint64_t n_dd, hipStream_t st) {
  if (n > h->wl_cap) {
    HIP_OK(hipStreamSynchronize(st));
    (void)hipFree(h->d_wl);
    h->d_wl = nullptr;
    const uint64_t cap = std::max<uint64_t>(n, 2 * h->wl_cap);
    const uint64_t seg = wl_seg_cap_for(cap);
    h->bytes -= h->wl_seg_cap * NSHARD * 8;
    h->wl_cap = 0;
    h->wl_seg_cap = 0;
    if (alloc((void **)&h->d_wl, seg * NSHARD * 8, &h->bytes) != HIVE_OK) return HIVE_ERR_OOM;
    h->wl_cap = cap;
    h->wl_seg_cap = seg;
  }
  if (n_dd > 0) {
    const uint64_t want = dd_words_for(n_dd);
    if (want > h->dd_cap) {
      HIP_OK(hipStreamSynchronize(st));
      (void)hipFree(h->d_dd);
      h->d_dd = nullptr;
      h->bytes -= h->dd_cap * 8;
      h->dd_cap = 0;
      if (alloc((void **)&h->d_dd, want * 8, &h->bytes) != HIVE_OK) return HIVE_ERR_OOM;
      h->dd_cap = want;
    }
  }
  return HIVE_OK;
}

// Probe-kernel variants a table may select per operation kind
// (hive_config.probe_tuning): occupancy target in waves per SIMD and loads
// in flight per probe chunk.  Variant 0 is the default; the others exist
// for 16-slot BitHash tables probing the second candidate after a miss
// (probe_both = 0).  The insert kernel's fused round holds twice the loads,
// so variants 1 and 2 would spill registers there and are refused for
// inserts (kInsertTunings).
struct ProbeTuning {
  int waves_per_simd, loads_in_flight;
};
static constexpr ProbeTuning kProbeTunings[] = {{OPS_WAVES_PER_EU, 16}, {6, 16}, {8, 8}, {6, 8}, {8, 4}};
static constexpr int kNumProbeTunings = sizeof(kProbeTunings) / sizeof(kProbeTunings[0]);
static constexpr uint32_t kInsertTunings = (1u << 0) | (1u << 3) | (1u << 4);

template <int S, uint32_t MODE, bool BOTH, int PAIR = PAIR_BITHASH, int V = 0>
static void launch_ops(const OpsArgs &a, uint32_t grid_cap, hipStream_t st) {
  constexpr ProbeTuning t = kProbeTunings[V];
  const uint64_t blocks = std::min<uint64_t>((a.n + BLOCK - 1) / BLOCK, grid_cap ? grid_cap : OPS_GRID);
  hipLaunchKernelGGL((ops_kernel<S, MODE, BOTH, PAIR, t.waves_per_simd, t.loads_in_flight>),
                     dim3((unsigned)blocks), dim3(BLOCK), 0, st, a);
}

template <int S, bool BOTH, int PAIR = PAIR_BITHASH, int V = 0>
static void launch_ops_mode_v(uint32_t mode, const OpsArgs &a, uint32_t grid_cap, hipStream_t st) {
  // inserts never take the variants hive_create refuses for them
  constexpr int VI = ((kInsertTunings >> V) & 1u) ? V : 0;
  switch (mode) {
    case OP_INSERT: launch_ops<S, OP_INSERT, BOTH, PAIR, VI>(a, grid_cap, st); break;
    case OP_DELETE: launch_ops<S, OP_DELETE, BOTH, PAIR, V>(a, grid_cap, st); break;
    case OP_LOOKUP: launch_ops<S, OP_LOOKUP, BOTH, PAIR, V>(a, grid_cap, st); break;
    default: launch_ops<S, OP_MIXED, BOTH, PAIR, V>(a, grid_cap, st); break;
  }
}

template <int S, bool BOTH, int PAIR = PAIR_BITHASH>
static void launch_ops_mode(uint32_t mode, const OpsArgs &a, const hive_config &cfg, hipStream_t st) {
  if constexpr (S == 16 && !BOTH && PAIR == PAIR_BITHASH) {
    switch ((cfg.probe_tuning >> (4 * std::min<uint32_t>(mode, OP_MIXED))) & 15u) {
      case 1: launch_ops_mode_v<S, BOTH, PAIR, 1>(mode, a, cfg.probe_grid, st); return;
      case 2: launch_ops_mode_v<S, BOTH, PAIR, 2>(mode, a, cfg.probe_grid, st); return;
      case 3: launch_ops_mode_v<S, BOTH, PAIR, 3>(mode, a, cfg.probe_grid, st); return;
      case 4: launch_ops_mode_v<S, BOTH, PAIR, 4>(mode, a, cfg.probe_grid, st); return;
      default: break;
    }
  }
  launch_ops_mode_v<S, BOTH, PAIR, 0>(mode, a, cfg.probe_grid, st);
}

// The eviction grid: one group per item up to EVICT_GRID blocks (chains are
// latency-bound, so items run side by side rather than one after another in
// a group); `max_items` bounds the worklist (the batch's inserts, or the
// stash and pending capacity for a drain).
static void phase_mark(hive_table *h, int kind, hipStream_t st);

// Grid of evict_lanes_kernel<PAIR>: a block per 256 possible items, at most
// as many blocks as are resident at once (a wave's range is not shared).
template <int PAIR>
static unsigned evict_lanes_grid(uint64_t max_items) {
  static const unsigned resident = [] {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, evict_lanes_kernel<PAIR>, BLOCK, 0) != hipSuccess ||
        cus < 1 || per_cu < 1) {
      (void)hipGetLastError();
      return (unsigned)EVICT_GRID;
    }
    return (unsigned)std::min(cus * per_cu, EVICT_GRID);
  }();
  return (unsigned)std::min<uint64_t>(grid_for(max_items, (uint64_t)BLOCK, EVICT_GRID), resident);
}

// split_steps (phase timing of a 16-slot BitHash table): steps 3 and 4 in
// two launches, the second timed as its own phase.  refill: 16-slot
// two-hash tables run evict_lanes_kernel (lanes refilled from the wave's
// range); the re-placement after a split, a few thousand items that each
// start a chain at once, keeps one item per lane (evict_kernel).
static void launch_evict(hive_table *h, uint64_t max_items, hipStream_t st, bool split_steps = false,
                         bool refill = true) {
  EvictArgs e{h->d_buckets, h->d_hint,       h->d_stash,   h->d_pending,   h->d_ctl,
              h->d_wl,      h->wl_seg_cap,   h->stash_cap, h->pending_cap, h->cfg.max_evictions};
  const dim3 grid(grid_for(max_items, (uint64_t)WAVES * evict_groups_per_wave(h->S), EVICT_GRID));
  if (split_steps && h->S == 16 && h->cfg.hash_pair == PAIR_BITHASH) {
    hipLaunchKernelGGL((evict_kernel<16, PAIR_BITHASH, true>), grid, dim3(BLOCK), 0, st, e);
    phase_mark(h, HIVE_PHASE_STASH, st);
    hipLaunchKernelGGL(stash_kernel<PAIR_BITHASH>, dim3(grid_for(max_items, BLOCK, EVICT_GRID)), dim3(BLOCK), 0, st,
                       e);
    return;
  }
  switch (h->S) {
    case 16:
      if (!refill && h->cfg.hash_pair != PAIR_TRIPLE) {
        if (h->cfg.hash_pair == PAIR_CRC)
          hipLaunchKernelGGL((evict_kernel<16, PAIR_CRC>), grid, dim3(BLOCK), 0, st, e);
        else if (h->cfg.hash_pair == PAIR_MURMUR)
          hipLaunchKernelGGL((evict_kernel<16, PAIR_MURMUR>), grid, dim3(BLOCK), 0, st, e);
        else
          hipLaunchKernelGGL(evict_kernel<16>, grid, dim3(BLOCK), 0, st, e);
      } else if (h->cfg.hash_pair == PAIR_CRC)
        hipLaunchKernelGGL(evict_lanes_kernel<PAIR_CRC>, dim3(evict_lanes_grid<PAIR_CRC>(max_items)), dim3(BLOCK),
                           0, st, e);
      else if (h->cfg.hash_pair == PAIR_MURMUR)
        hipLaunchKernelGGL(evict_lanes_kernel<PAIR_MURMUR>, dim3(evict_lanes_grid<PAIR_MURMUR>(max_items)),
                           dim3(BLOCK), 0, st, e);
      else if (h->cfg.hash_pair == PAIR_TRIPLE)
        hipLaunchKernelGGL((evict_kernel<16, PAIR_TRIPLE>), grid, dim3(BLOCK), 0, st, e);
      else
        hipLaunchKernelGGL(evict_lanes_kernel<PAIR_BITHASH>, dim3(evict_lanes_grid<PAIR_BITHASH>(max_items)),
                           dim3(BLOCK), 0, st, e);
      break;
    case 32: hipLaunchKernelGGL(evict_kernel<32>, grid, dim3(BLOCK), 0, st, e); break;
    default: hipLaunchKernelGGL(evict_kernel<64>, grid, dim3(BLOCK), 0, st, e); break;
  }
}

// Fold the shards into the totals and empty the worklist.
static void launch_finish(hive_table *h, hipStream_t st) {
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, st, h->d_ctl);
}

// Upper bound on the hashing rounds one resize call can cross: from the
// initial bucket count to the arena size, plus the partial rounds at both
// ends.
static int resize_rounds(const hive_table *h) {
  int r = 2;
  for (uint64_t x = h->initial_buckets; x < h->max_buckets; x *= 2) ++r;
  return r;
}

// merges: the call may contract (pass 2 moves merge pairs; a split-only call
// skips its launches, which would find nothing to do)
template <int S>
static void launch_resize_passes(const ResizeArgs &ra, int rounds, bool merges, hipStream_t st) {
  for (int r = 0; r < rounds; ++r) {
    hipLaunchKernelGGL(resize_pass1_kernel<S>, dim3(RESIZE_GRID), dim3(BLOCK), 0, st, ra);
    if (merges) hipLaunchKernelGGL(resize_pass2_kernel<S>, dim3(RESIZE_GRID), dim3(BLOCK), 0, st, ra);
  }
}

// Phase timing: close the open span (if any) at an event recorded now on
// `st` and open one of `kind` there (kind < 0: open none).  Off unless
// hive_phase_timing enabled it; a failure to get an event turns it off.
static void phase_mark(hive_table *h, int kind, hipStream_t st) {
  if (!h->timing) return;
  hipEvent_t e = nullptr;
  if (!h->free_events.empty()) {
    e = h->free_events.back();
    h->free_events.pop_back();
  } else if (hipEventCreate(&e) == hipSuccess) {
    h->all_events.push_back(e);
  } else {
    (void)hipGetLastError();
    h->timing = false;
    return;
  }
  (void)hipEventRecord(e, st);
  if (h->open_kind >= 0) h->spans.push_back({h->open_kind, h->open_ev, e});
  h->open_kind = kind;
  h->open_ev = e;
}

// batch_items > 0: the call follows a batch's probe launch whose eviction
// worklist (at most batch_items entries) is still to be placed; the
// drained stash joins it and one eviction launch places both.
static hive_status resize_sequence(hive_table *h, uint32_t mode, uint64_t amount, const uint8_t *d_ops,
                                   hipStream_t st, uint64_t batch_items = 0) {
  ResizeArgs ra{h->d_buckets, h->d_hint, h->d_ctl, h->S, h->cfg.resize_k, h->cfg.lf_expand_pct,
                h->cfg.lf_contract_pct};
  phase_mark(h, HIVE_PHASE_RESIZE, st);
  if (mode == PLAN_PRE_MIXED && amount <= BLOCK * 16ull) {
    hipLaunchKernelGGL(count_and_plan_kernel, dim3(1), dim3(BLOCK), 0, st, ra, d_ops, amount);
  } else {
    if (mode == PLAN_PRE_MIXED)
      hipLaunchKernelGGL(count_inserts_kernel, dim3(grid_for(amount, BLOCK * 16ull, 1024)), dim3(BLOCK), 0, st,
                         h->d_ctl, d_ops, amount);
    hipLaunchKernelGGL(resize_plan_kernel, dim3(1), dim3(1), 0, st, ra, mode, amount);
  }
  const int rounds = resize_rounds(h);
  // pre-batch growth and explicit splits never merge
  const bool merges = mode == PLAN_POST || mode == PLAN_MERGE;
  switch (h->S) {
    case 16: launch_resize_passes<16>(ra, rounds, merges, st); break;
    case 32: launch_resize_passes<32>(ra, rounds, merges, st); break;
    default: launch_resize_passes<64>(ra, rounds, merges, st); break;
  }
  phase_mark(h, HIVE_PHASE_DRAIN, st);
  hipLaunchKernelGGL(drain_kernel, dim3(DRAIN_GRID), dim3(BLOCK), 0, st, h->d_stash, h->stash_cap, h->d_pending,
                     h->pending_cap, h->d_hint, hint_words(h->max_buckets), h->d_wl, h->wl_seg_cap, h->d_ctl);
  // live entries of a drain (and the batch's worklist)
  launch_evict(h, batch_items + h->stash_cap + h->pending_cap, st, false, batch_items > 0);
  launch_finish(h, st);
  return launch_check();
}


// ---------------------------------------------------------------------------
// Persistent executor (host side)
// ---------------------------------------------------------------------------
static void free_drain(hive_drain *d) {
  if (!d) return;
  for (int m = 0; m < 2; ++m) {
    if (d->exec[m]) (void)hipGraphExecDestroy(d->exec[m]);
    if (d->graph[m]) (void)hipGraphDestroy(d->graph[m]);
  }
  if (d->capture) (void)hipStreamDestroy(d->capture);
  (void)hipFree(d->d_q);
  (void)hipFree(d->d_req);
  (void)hipFree(d->d_table_next);
  (void)hipHostFree(d->h_ring);
  (void)hipHostFree(d->h_tail);
  (void)hipHostFree(d->h_stop);
  (void)hipHostFree(d->h_done);
  (void)hipHostFree(d->h_live);
  delete d;
}

// Ticks per microsecond of the device's constant-rate clock: two readings
// 10 ms apart on the host clock (launch latency is a small error here).
static hive_status wall_clock_rate(double *ticks_per_us) {
  uint64_t *d_t = nullptr;
  uint64_t t[2] = {0, 0};
  HIP_OK(hipMalloc((void **)&d_t, 16));
  hipLaunchKernelGGL(wall_clock_kernel, dim3(1), dim3(1), 0, 0, d_t);
  hipError_t e = hipDeviceSynchronize();
  const auto h0 = std::chrono::steady_clock::now();
  std::this_thread::sleep_for(std::chrono::milliseconds(10));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(wall_clock_kernel, dim3(1), dim3(1), 0, 0, d_t + 1);
    e = hipDeviceSynchronize();
  }
  const auto h1 = std::chrono::steady_clock::now();
  if (e == hipSuccess) e = hipMemcpy(t, d_t, 16, hipMemcpyDeviceToHost);
  (void)hipFree(d_t);
  if (e != hipSuccess || t[1] <= t[0]) {
    fprintf(stderr, "hive: device clock calibration failed: %s\n", hipGetErrorString(e));
    return HIVE_ERR_HIP;
  }
  const double us = std::chrono::duration<double, std::micro>(h1 - h0).count();
  *ticks_per_us = (double)(t[1] - t[0]) / us;
  return HIVE_OK;
}

// Grid sizes.  A draining grid may fill every CU: it exits once its work is
// done.  A resident grid waits for work that the host has not submitted yet,
// and the host may first need other kernels to run (its own copies: HIP runs
// small pageable copies as kernels); with every CU's registers held by the
// polling grid such a kernel cannot start until the grid exits.  So a
// resident grid takes one block per CU fewer than fit (at least one).
template <int S>
static hive_status drain_grid(uint32_t blocks_per_cu, unsigned grid[2], int *fit_per_cu) {
  int dev = 0, cus = 0, per_cu = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, drain_worker_kernel<S>, BLOCK, 0));
  if (per_cu < 1) return HIVE_ERR_HIP;
  *fit_per_cu = per_cu;
  const unsigned want = blocks_per_cu ? blocks_per_cu : (unsigned)per_cu;
  grid[0] = (unsigned)cus * std::min<unsigned>(want, (unsigned)per_cu);
  grid[1] = (unsigned)cus * std::min<unsigned>(want, (unsigned)std::max(1, per_cu - 1));
  return HIVE_OK;
}

template <int S>
static void launch_drain_kernel(hive_drain *d, int mode, hipStream_t st) {
  hipLaunchKernelGGL(drain_worker_kernel<S>, dim3(d->grid[mode]), dim3(BLOCK), 0, st, d->d_q);
}

static void launch_drain_any(hive_drain *d, int mode, hipStream_t st) {
  switch (d->S) {
    case 16: launch_drain_kernel<16>(d, mode, st); break;
    case 32: launch_drain_kernel<32>(d, mode, st); break;
    default: launch_drain_kernel<64>(d, mode, st); break;
  }
}

// The partitioned dedupe of a batch (five launches) into the scratch at dd,
// which holds dd_words_for(n) words; *win gets the winner flags.
static hive_status launch_dedupe(uint64_t *dd, uint32_t mode, const uint8_t *d_ops, const uint32_t *d_keys,
                                 uint64_t n, hipStream_t st, const uint8_t **win) {
  DdpArgs d{};
  const uint32_t nt = mode == OP_MIXED ? 2 : 1;
  ddp_layout(dd, n, nt, &d);
  d.ops = d_ops;
  d.keys = d_keys;
  d.mode = mode;
  hipLaunchKernelGGL(ddp_collect_kernel, dim3((unsigned)d.nch), dim3(BLOCK), 0, st, d);
  *win = d.win;
  // a batch of one chunk: the chunk's winners are the batch's (the serving
  // loop's requests are mostly this small, and each launch costs the host
  // several microseconds)
  if (d.nch == 1) return launch_check();
  hipLaunchKernelGGL(ddp_segsum_kernel, dim3((unsigned)(nt * d.nseg)), dim3(BLOCK), 0, st, d);
  hipLaunchKernelGGL(ddp_scan_kernel, dim3(nt * (DDP_BINS / 64)), dim3(DDP_SCAN_WAVES * 64), 0, st, d);
  hipLaunchKernelGGL(ddp_scatter_kernel, dim3((unsigned)(nt * d.nseg)), dim3(DDP_WIDE), 0, st, d);
  hipLaunchKernelGGL(ddp_resolve_kernel, dim3(nt * DDP_BINS), dim3(DDP_WIDE), 0, st, d);
  return launch_check();
}

// ---------------------------------------------------------------------------
// Scratch for callers that cannot allocate (hive_mixed_batch_noalloc): the
// dedupe set of one batch lives in this array instead of the table's
// grow-on-demand buffer.  Each GPU holds its own copy for the life of the
// process; host code reaches it only through the per-device address that
// hipGetSymbolAddress returns (the array's name is a host-side stand-in).
// ---------------------------------------------------------------------------
constexpr uint64_t NOALLOC_DD_WORDS = 1ull << 24;  // 128 MiB
constexpr uint64_t NOALLOC_MAX_BATCH = 1ull << 22;  // dd_words_for(n) <= NOALLOC_DD_WORDS (checked at first use)
static __device__ __align__(256) uint64_t scratch[NOALLOC_DD_WORDS];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static uint64_t *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The current device's copy of `scratch`, looked up once per device.
static hive_status noalloc_scratch(uint64_t **out) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return HIVE_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = (uint64_t *)p;
  }
  *out = g_scratch_ptr[dev];
  return HIVE_OK;
}

// no_alloc: take the dedupe set from `scratch` and refuse a batch that would
// grow the table's worklist, so that the call allocates nothing; phase
// timing (which creates events) is skipped for such a call.
static hive_status run_batch(hive_t h, uint32_t mode, const uint8_t *d_ops, const uint32_t *d_keys,
                             const uint32_t *d_vals, uint64_t n, uint32_t flags, uint32_t *d_vals_out,
                             uint8_t *d_flags_out, void *stream, bool no_alloc = false) {
  if (!h || (n > 0 && !d_keys)) return HIVE_ERR_ARG;
  if (n >= 0xFFFFFFFFull) return HIVE_ERR_ARG;  // batch indices are 32-bit in the dedupe set
  if (mode == OP_INSERT && n > 0 && !d_vals && h->entry_bytes == 8) return HIVE_ERR_ARG;  // sets read no values
  if (mode == OP_MIXED && n > 0 && !d_ops) return HIVE_ERR_ARG;
  if (flags & ~(uint32_t)HIVE_UNIQUE) return HIVE_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const bool dedupe = !(flags & HIVE_UNIQUE) && mode != OP_LOOKUP;
  const bool linear = h->cfg.addressing == HIVE_LINEAR;
  const bool inserts = mode == OP_INSERT || mode == OP_MIXED;
  // A batch with inserts on a table with the post-batch rule places its
  // eviction worklist after the rule: the splits' stash drain joins the
  // worklist and one eviction launch places both (the re-placement launch
  // goes).  The worklist then holds the batch's entries and a full drain.
  const uint64_t wl_post = n + drain_words(h) + WL_SLACK;
  const bool post_after = linear && h->cfg.post_policy && inserts && h->entry_bytes == 8 && !h->timing &&
                          (!no_alloc || wl_post <= h->wl_cap);
  // only inserts reach the eviction worklist
  const uint64_t wl_need = inserts ? (post_after ? wl_post : n) : 0;
  uint64_t *dd = nullptr;
  if (no_alloc) {
    if (wl_need > h->wl_cap) {
      fprintf(stderr, "hive: a batch of %llu operations needs a larger worklist than the table's (%llu); "
              "create the table with max_batch >= n for allocation-free calls\n",
              (unsigned long long)n, (unsigned long long)h->wl_cap);
      return HIVE_ERR_BUDGET;
    }
    if (dedupe && (n > NOALLOC_MAX_BATCH || dd_words_for(n) > NOALLOC_DD_WORDS)) {
      fprintf(stderr, "hive: allocation-free batches with dedupe hold at most %llu operations (got %llu)\n",
              (unsigned long long)NOALLOC_MAX_BATCH, (unsigned long long)n);
      return HIVE_ERR_BUDGET;
    }
    if (dedupe) {
      hive_status s = noalloc_scratch(&dd);
      if (s != HIVE_OK) return s;
    }
  }
  h->last = st;
  if (n == 0) return HIVE_OK;
  hive_status s = HIVE_OK;
  if (!no_alloc) {
    if ((s = ensure_scratch(h, wl_need, dedupe ? n : 0, st)) != HIVE_OK) return s;
    dd = h->d_dd;
  }
  // phase timing creates events on demand: off for an allocation-free call
  struct TimingOff {
    hive_table *h;
    bool was;
    ~TimingOff() { h->timing = was; }
  } timing_guard{h, h->timing};
  if (no_alloc) h->timing = false;
  OpsArgs a{};
  a.buckets = h->d_buckets;
  a.hint = h->d_hint;
  a.stash = h->d_stash;
  a.pending = h->d_pending;
  a.ctl = h->d_ctl;
  a.wl = h->d_wl;
  a.wl_seg_cap = h->wl_seg_cap;
  a.ops = d_ops;
  a.keys = d_keys;
  a.vals = d_vals;
  a.vals_out = d_vals_out;
  a.flags_out = d_flags_out;
  a.n = n;
  a.stash_cap = h->stash_cap;
  a.pending_cap = h->pending_cap;
  if (dedupe) {
    phase_mark(h, HIVE_PHASE_DEDUPE, st);
    // within the buffer: ensure_scratch sized the table's from n, and the
    // allocation-free path checked n against NOALLOC_MAX_BATCH
    if ((s = launch_dedupe(dd, mode, d_ops, d_keys, n, st, &a.win)) != HIVE_OK) return s;
  }
  if (h->entry_bytes == 4) {
    SetArgs sa{(uint32_t *)h->d_buckets, h->d_hint, (uint32_t *)h->d_stash, (uint32_t *)h->d_pending, h->d_ctl,
               h->d_wl, h->wl_seg_cap, a.dd, a.dd_mask, d_ops, d_keys, d_flags_out, n, h->stash_cap, h->pending_cap,
               h->cfg.max_evictions, a.win};
    phase_mark(h, HIVE_PHASE_PROBE, st);
    const uint64_t cap = h->cfg.probe_grid ? h->cfg.probe_grid : OPS_GRID;
    const dim3 grid((unsigned)std::min<uint64_t>((n + BLOCK - 1) / BLOCK, cap));
    switch (mode) {
      case OP_INSERT: hipLaunchKernelGGL(set_ops_kernel<OP_INSERT>, grid, dim3(BLOCK), 0, st, sa); break;
      case OP_DELETE: hipLaunchKernelGGL(set_ops_kernel<OP_DELETE>, grid, dim3(BLOCK), 0, st, sa); break;
      case OP_LOOKUP: hipLaunchKernelGGL(set_ops_kernel<OP_LOOKUP>, grid, dim3(BLOCK), 0, st, sa); break;
      default: hipLaunchKernelGGL(set_ops_kernel<OP_MIXED>, grid, dim3(BLOCK), 0, st, sa); break;
    }
    if (mode == OP_INSERT || mode == OP_MIXED) {
      phase_mark(h, HIVE_PHASE_EVICT, st);
      hipLaunchKernelGGL(set_evict_kernel, dim3(grid_for(n, BLOCK, EVICT_GRID)), dim3(BLOCK), 0, st, sa);
    }
    if (mode != OP_LOOKUP) {
      phase_mark(h, HIVE_PHASE_FINISH, st);
      launch_finish(h, st);
    }
    phase_mark(h, -1, st);
    return launch_check();
  }
  if (linear && h->cfg.pre_expand && (mode == OP_INSERT || mode == OP_MIXED)) {
    // grow before the batch so that live + (inserts of the batch) fits
    if ((s = resize_sequence(h, mode == OP_MIXED ? PLAN_PRE_MIXED : PLAN_PRE, n, d_ops, st)) != HIVE_OK) return s;
  }
  phase_mark(h, HIVE_PHASE_PROBE, st);
  switch (h->S) {
    case 16:
      if (h->cfg.hash_pair == PAIR_CRC)
        launch_ops_mode<16, false, PAIR_CRC>(mode, a, h->cfg, st);
      else if (h->cfg.hash_pair == PAIR_MURMUR)
        launch_ops_mode<16, false, PAIR_MURMUR>(mode, a, h->cfg, st);
      else if (h->cfg.hash_pair == PAIR_TRIPLE)
        launch_ops_mode<16, false, PAIR_TRIPLE>(mode, a, h->cfg, st);
      else if (h->cfg.probe_both)
        launch_ops_mode<16, true>(mode, a, h->cfg, st);
      else
        launch_ops_mode<16, false>(mode, a, h->cfg, st);
      break;
    case 32: launch_ops_mode<32, false>(mode, a, h->cfg, st); break;
    default: launch_ops_mode<64, false>(mode, a, h->cfg, st); break;
  }
  if ((s = launch_check()) != HIVE_OK) return s;
  if (post_after) {
    hipLaunchKernelGGL(fold_kernel, dim3(1), dim3(64), 0, st, h->d_ctl);
    if ((s = resize_sequence(h, PLAN_POST, 0, nullptr, st, n)) != HIVE_OK) return s;
    phase_mark(h, -1, st);
    return HIVE_OK;
  }
  if (mode == OP_INSERT || mode == OP_MIXED) {
    phase_mark(h, HIVE_PHASE_EVICT, st);
    launch_evict(h, n, st, h->timing);
  }
  if (mode != OP_LOOKUP) {
    phase_mark(h, HIVE_PHASE_FINISH, st);
    launch_finish(h, st);
  }
  if ((s = launch_check()) != HIVE_OK) return s;
  if (linear && h->cfg.post_policy && mode != OP_LOOKUP) {
    if ((s = resize_sequence(h, PLAN_POST, 0, nullptr, st)) != HIVE_OK) return s;
  }
  phase_mark(h, -1, st);
  return HIVE_OK;
}

extern "C" {

hive_status hive_config_default(hive_config *cfg) {
  if (!cfg) return HIVE_ERR_ARG;
  memset(cfg, 0, sizeof(*cfg));
  cfg->slots_per_bucket = 16;
  cfg->max_evictions = 8;
  cfg->addressing = HIVE_FIXED;
  cfg->resize_k = 1024;
  cfg->lf_expand_pct = 90;
  cfg->lf_contract_pct = 25;
  return HIVE_OK;
}

hive_status hive_create(const hive_config *cfg_in, uint64_t initial_buckets, void *stream, hive_t *out) {
  if (!cfg_in || !out) return HIVE_ERR_ARG;
  *out = nullptr;
  hive_config cfg = *cfg_in;
  const uint32_t S = cfg.slots_per_bucket;
  if (S != 16 && S != 32 && S != 64) return HIVE_ERR_ARG;
  if (cfg.addressing != HIVE_FIXED && cfg.addressing != HIVE_LINEAR) return HIVE_ERR_ARG;
  if (cfg.hash_pair > HIVE_PAIR_TRIPLE) return HIVE_ERR_ARG;
  if (cfg.entry_bits != 0 && cfg.entry_bits != 64 && cfg.entry_bits != 32) return HIVE_ERR_ARG;
  const bool set32 = cfg.entry_bits == 32;
  // key-only sets: 32 slots of 4 bytes (one 128-byte line), FIXED, BitHash1/2
  if (set32 && (S != 32 || cfg.addressing != HIVE_FIXED || cfg.hash_pair != HIVE_PAIR_BITHASH || cfg.probe_both))
    return HIVE_ERR_ARG;
  // only 16-slot FIXED tables on plain launches have the other hash pairs
  if (cfg.hash_pair != HIVE_PAIR_BITHASH && (S != 16 || cfg.addressing != HIVE_FIXED || cfg.probe_both))
    return HIVE_ERR_ARG;
  // probe_tuning: one variant per operation kind (insert, delete, lookup,
  // mixed), four bits each
  if ((cfg.probe_tuning >> 16) != 0 || !((kInsertTunings >> (cfg.probe_tuning & 15u)) & 1u) ||
      (cfg.probe_tuning && (S != 16 || cfg.hash_pair != HIVE_PAIR_BITHASH || cfg.probe_both || set32)))
    return HIVE_ERR_ARG;
  for (int kind = 0; kind < 4; ++kind)
    if (((cfg.probe_tuning >> (4 * kind)) & 15u) >= (uint32_t)kNumProbeTunings) return HIVE_ERR_ARG;
  if (cfg.probe_grid > (1u << 20)) return HIVE_ERR_ARG;
  if (initial_buckets < 1) return HIVE_ERR_ARG;
  if (cfg.max_evictions > 1024) return HIVE_ERR_ARG;
  if (cfg.lf_expand_pct == 0 || cfg.lf_expand_pct > 100 || cfg.lf_contract_pct >= cfg.lf_expand_pct)
    return HIVE_ERR_ARG;
  if (cfg.resize_k == 0) cfg.resize_k = 1024;
  uint64_t max_b = initial_buckets;
  if (cfg.addressing == HIVE_LINEAR) {
    max_b = std::max<uint64_t>(cfg.max_buckets, initial_buckets);
    if (max_b > (1ull << 31)) return HIVE_ERR_ARG;  // 32-bit bucket indices
  } else {
    if (initial_buckets > 0xFFFFFFFFull) return HIVE_ERR_ARG;
    if (cfg.max_buckets > initial_buckets) return HIVE_ERR_ARG;  // FIXED tables do not grow
  }
  if (max_b > (1ull << 40) / S) return HIVE_ERR_ARG;
  hive_table *h = new (std::nothrow) hive_table();
  if (!h) return HIVE_ERR_OOM;
  h->S = S;
  h->entry_bytes = set32 ? 4 : 8;
  h->initial_buckets = initial_buckets;
  h->max_buckets = max_b;
  // default: 1% of the slots of the largest table (the arena)
  h->stash_cap = cfg.stash_capacity ? cfg.stash_capacity : std::max<uint64_t>(1024, max_b * S / 100);
  h->pending_cap = cfg.pending_capacity ? cfg.pending_capacity : h->stash_cap;
  cfg.stash_capacity = h->stash_cap;
  cfg.pending_capacity = h->pending_cap;
  cfg.max_buckets = max_b;
  h->cfg = cfg;
  hive_status s = HIVE_OK;
  if ((s = alloc((void **)&h->d_buckets, max_b * S * h->entry_bytes, &h->bytes)) != HIVE_OK ||
      (s = alloc((void **)&h->d_hint, hint_words(max_b) * 4, &h->bytes)) != HIVE_OK ||
      (s = alloc((void **)&h->d_stash, stash_slots_for(h->stash_cap) * h->entry_bytes, &h->bytes)) != HIVE_OK ||
      (s = alloc((void **)&h->d_pending, h->pending_cap * h->entry_bytes, &h->bytes)) != HIVE_OK ||
      (s = alloc((void **)&h->d_ctl, CTL_BYTES, &h->bytes)) != HIVE_OK) {
    free_table(h);
    return s;
  }
  hipStream_t st = (hipStream_t)stream;
  h->last = st;
  // the worklist must hold a full stash + pending drain (after a split);
  // the drain walks the whole stash table
  const uint64_t min_wl = drain_words(h);
  // a table with the post-batch rule places a batch's worklist after the
  // rule, together with the drain (see run_batch)
  const uint64_t batch_wl = cfg.addressing == HIVE_LINEAR && cfg.post_policy && cfg.max_batch
                                ? cfg.max_batch + min_wl + WL_SLACK
                                : cfg.max_batch;
  if ((s = ensure_scratch(h, std::max<uint64_t>(batch_wl, min_wl), cfg.max_batch, st)) != HIVE_OK) {
    free_table(h);
    return s;
  }
  if ((s = reset_table(h, st)) != HIVE_OK || hipStreamSynchronize(st) != hipSuccess) {
    free_table(h);
    return s != HIVE_OK ? s : HIVE_ERR_HIP;
  }
  *out = h;
  return HIVE_OK;
}

hive_status hive_phase_timing(hive_t h, int enable) {
  if (!h) return HIVE_ERR_ARG;
  h->timing = enable != 0;
  return HIVE_OK;
}

hive_status hive_phase_times(hive_t h, double *ms_out) {
  if (!h || !ms_out) return HIVE_ERR_ARG;
  for (int k = 0; k < HIVE_PHASE_KINDS; ++k) ms_out[k] = 0.0;
  hive_status s = HIVE_OK;
  if (!h->spans.empty() && hipEventSynchronize(h->spans.back().b) != hipSuccess) s = HIVE_ERR_HIP;
  std::vector<hipEvent_t> used;
  for (const auto &sp : h->spans) {
    float ms = 0.f;
    if (s == HIVE_OK && hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) ms_out[sp.kind] += ms;
    used.push_back(sp.a);
    used.push_back(sp.b);
  }
  // an event may end one span and start the next: free each once, except
  // the start of a span still open
  std::sort(used.begin(), used.end());
  used.erase(std::unique(used.begin(), used.end()), used.end());
  for (hipEvent_t e : used)
    if (!(h->open_kind >= 0 && e == h->open_ev)) h->free_events.push_back(e);
  h->spans.clear();
  if (s != HIVE_OK) (void)hipGetLastError();
  return s;
}

hive_status hive_destroy(hive_t h) {
  if (!h) return HIVE_ERR_ARG;
  hipError_t e = hipStreamSynchronize(h->last);
  free_table(h);
  return e == hipSuccess ? HIVE_OK : HIVE_ERR_HIP;
}

hive_status hive_insert_batch(hive_t h, const uint32_t *d_keys, const uint32_t *d_vals, uint64_t n, uint32_t flags,
                              void *stream) {
  return run_batch(h, OP_INSERT, nullptr, d_keys, d_vals, n, flags, nullptr, nullptr, stream);
}

hive_status hive_lookup_batch(hive_t h, const uint32_t *d_keys, uint64_t n, uint32_t *d_vals_out,
                              uint8_t *d_found_out, void *stream) {
  return run_batch(h, OP_LOOKUP, nullptr, d_keys, nullptr, n, HIVE_UNIQUE, d_vals_out, d_found_out, stream);
}

hive_status hive_delete_batch(hive_t h, const uint32_t *d_keys, uint64_t n, uint32_t flags, uint8_t *d_deleted_out,
                              void *stream) {
  return run_batch(h, OP_DELETE, nullptr, d_keys, nullptr, n, flags, nullptr, d_deleted_out, stream);
}

hive_status hive_mixed_batch(hive_t h, const uint8_t *d_ops, const uint32_t *d_keys, const uint32_t *d_vals,
                             uint64_t n, uint32_t flags, uint32_t *d_vals_out, uint8_t *d_flags_out, void *stream) {
  if (h && n > 0 && !d_vals && h->entry_bytes == 8) return HIVE_ERR_ARG;  // inserts read their values
  return run_batch(h, OP_MIXED, d_ops, d_keys, d_vals, n, flags, d_vals_out, d_flags_out, stream);
}

hive_status hive_mixed_batch_noalloc(hive_t h, const uint8_t *d_ops, const uint32_t *d_keys, const uint32_t *d_vals,
                                     uint64_t n, uint32_t flags, uint32_t *d_vals_out, uint8_t *d_flags_out,
                                     void *stream) {
  if (h && n > 0 && !d_vals && h->entry_bytes == 8) return HIVE_ERR_ARG;
  return run_batch(h, OP_MIXED, d_ops, d_keys, d_vals, n, flags, d_vals_out, d_flags_out, stream, true);
}

hive_status hive_resize(hive_t h, int64_t delta, void *stream) {
  if (!h) return HIVE_ERR_ARG;
  if (h->cfg.addressing != HIVE_LINEAR) return HIVE_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  h->last = st;
  if (delta > 0) return resize_sequence(h, PLAN_SPLIT, (uint64_t)delta, nullptr, st);
  if (delta < 0) return resize_sequence(h, PLAN_MERGE, (uint64_t)(-(delta + 1)) + 1, nullptr, st);
  return resize_sequence(h, PLAN_POST, 0, nullptr, st);
}

hive_status hive_stats(hive_t h, hive_stats_t *out, void *stream) {
  if (!h || !out) return HIVE_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  Ctl c;
  HIP_OK(hipMemcpyAsync(&c, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  memset(out, 0, sizeof(*out));
  out->live = c.live;
  out->n_buckets = c.n_buckets;
  out->index_mask = c.im;
  out->split_ptr = c.sp;
  out->stash_count = std::min(c.stash_count, h->stash_cap);
  out->pending_count = std::min(c.pending_count, h->pending_cap);
  out->evictions = c.evictions;
  out->stash_inserts = c.stash_inserts;
  out->pending_inserts = c.pending_inserts;
  out->full_chains = c.full_chains;
  out->invalid_keys = c.invalid_keys;
  out->evict_items = c.evict_items;
  out->bytes_reserved = h->bytes;
  out->slots_per_bucket = h->S;
  out->max_buckets = h->max_buckets;
  out->error_bits = c.error;
  if (c.error & ERR_PENDING_LOST) return HIVE_ERR_LOST;
  if (c.error & ERR_ARENA_FULL) return HIVE_ERR_BUDGET;
  if (out->pending_count) return HIVE_WARN_PENDING;
  if (c.invalid_keys) return HIVE_WARN_INVALID_KEYS;
  return HIVE_OK;
}

hive_status hive_dump(hive_t h, uint64_t *d_words, int64_t *d_where, uint64_t capacity, uint64_t *n_out,
                      void *stream) {
  if (!h || !n_out || (capacity > 0 && !d_words)) return HIVE_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  h->last = st;
  hipLaunchKernelGGL(ctl_zero_dump_kernel, dim3(1), dim3(1), 0, st, h->d_ctl);
  hive_status s = launch_check();
  if (s != HIVE_OK) return s;
  if (h->entry_bytes == 4)
    hipLaunchKernelGGL(set_dump_kernel, dim3(2048), dim3(BLOCK), 0, st, (const uint32_t *)h->d_buckets,
                       (const uint32_t *)h->d_stash, (const uint32_t *)h->d_pending, h->d_ctl, h->stash_cap,
                       h->pending_cap, d_words, d_where, capacity);
  else
    hipLaunchKernelGGL(dump_kernel, dim3(2048), dim3(BLOCK), 0, st, h->d_buckets, h->S, h->d_stash, h->d_pending,
                       h->d_ctl, h->stash_cap, h->pending_cap, d_words, d_where, capacity);
  if ((s = launch_check()) != HIVE_OK) return s;
  Ctl c;
  HIP_OK(hipMemcpyAsync(&c, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  *n_out = c.dump_count;
  return HIVE_OK;
}

hive_status hive_placement(hive_t h, uint64_t *out, void *stream) {
  if (!h || !out) return HIVE_ERR_ARG;
  if (h->cfg.hash_pair != HIVE_PAIR_BITHASH) return HIVE_ERR_ARG;  // the census computes BitHash1 candidates
  hipStream_t st = (hipStream_t)stream;
  h->last = st;
  hipLaunchKernelGGL(ctl_zero_placement_kernel, dim3(1), dim3(1), 0, st, h->d_ctl);
  hive_status s = launch_check();
  if (s != HIVE_OK) return s;
  if (h->entry_bytes == 4)
    hipLaunchKernelGGL(placement_kernel<true>, dim3(2048), dim3(BLOCK), 0, st, (const void *)h->d_buckets, h->S,
                       h->d_ctl);
  else
    hipLaunchKernelGGL(placement_kernel<false>, dim3(2048), dim3(BLOCK), 0, st, (const void *)h->d_buckets, h->S,
                       h->d_ctl);
  if ((s = launch_check()) != HIVE_OK) return s;
  Ctl c;
  HIP_OK(hipMemcpyAsync(&c, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  out[0] = c.place_first;
  out[1] = c.place_second;
  out[2] = std::min(c.stash_count, h->stash_cap) + std::min(c.pending_count, h->pending_cap);
  return HIVE_OK;
}

hive_status hive_live_async(hive_t h, uint64_t *host_dst, void *stream) {
  if (!h || !host_dst) return HIVE_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  h->last = st;
  HIP_OK(hipMemcpyAsync(host_dst, &h->d_ctl->live, 8, hipMemcpyDeviceToHost, st));
  return HIVE_OK;
}

hive_status hive_clear(hive_t h, void *stream) {
  if (!h) return HIVE_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  h->last = st;
  return reset_table(h, st);
}

const char *hive_status_string(hive_status s) {
  switch (s) {
    case HIVE_OK: return "ok";
    case HIVE_ERR_ARG: return "invalid argument";
    case HIVE_ERR_OOM: return "device allocation failed";
    case HIVE_ERR_HIP: return "HIP runtime error";
    case HIVE_ERR_BUDGET: return "bucket arena or capacity exhausted";
    case HIVE_ERR_LOST: return "pending list overflowed: entries lost";
    case HIVE_WARN_INVALID_KEYS: return "reserved keys were ignored";
    case HIVE_WARN_PENDING: return "entries wait in the pending list";
  }
  return "unknown status";
}

uint32_t hive_bithash1(uint32_t key) { return bithash1(key); }
uint32_t hive_bithash2(uint32_t key) { return bithash2(key); }

hive_status hive_bucket_of(hive_t h, uint32_t mixed_hash, uint64_t *bucket) {
  if (!h || !bucket) return HIVE_ERR_ARG;
  Ctl c;
  HIP_OK(hipMemcpyAsync(&c, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->last));
  HIP_OK(hipStreamSynchronize(h->last));
  Geo g{c.n_buckets, c.magic, (uint32_t)c.im, (uint32_t)c.sp, c.mode};
  *bucket = address(g, mixed_hash);
  return HIVE_OK;
}


hive_status hive_drain_create(uint32_t slots_per_bucket, uint32_t blocks_per_cu, uint64_t ring_capacity,
                              uint32_t max_tables, uint64_t idle_timeout_us, hive_drain_t *out) {
  if (!out) return HIVE_ERR_ARG;
  *out = nullptr;
  if (slots_per_bucket != 16 && slots_per_bucket != 32 && slots_per_bucket != 64) return HIVE_ERR_ARG;
  if (ring_capacity < 1 || ring_capacity > (1ull << 24)) return HIVE_ERR_ARG;
  if (max_tables < 1 || max_tables > 4096) return HIVE_ERR_ARG;
  hive_drain *d = new (std::nothrow) hive_drain();
  if (!d) return HIVE_ERR_OOM;
  d->S = slots_per_bucket;
  d->cap = ring_capacity;
  d->max_tables = max_tables;
  hive_status s = HIVE_OK;
  switch (d->S) {
    case 16: s = drain_grid<16>(blocks_per_cu, d->grid, &d->fit_per_cu); break;
    case 32: s = drain_grid<32>(blocks_per_cu, d->grid, &d->fit_per_cu); break;
    default: s = drain_grid<64>(blocks_per_cu, d->grid, &d->fit_per_cu); break;
  }
  if (s != HIVE_OK) {
    free_drain(d);
    return s;
  }
  uint64_t bytes = 0;
  if (alloc((void **)&d->d_q, sizeof(DrainQueue), &bytes) != HIVE_OK ||
      alloc((void **)&d->d_req, sizeof(ReqState) * ring_capacity, &bytes) != HIVE_OK ||
      alloc((void **)&d->d_table_next, 8ull * max_tables, &bytes) != HIVE_OK) {
    free_drain(d);
    return HIVE_ERR_OOM;
  }
  const unsigned hflags = hipHostMallocMapped | hipHostMallocCoherent;
  if (hipHostMalloc((void **)&d->h_ring, sizeof(ReqDesc) * ring_capacity, hflags) != hipSuccess ||
      hipHostMalloc((void **)&d->h_tail, 64, hflags) != hipSuccess ||
      hipHostMalloc((void **)&d->h_stop, 64, hflags) != hipSuccess ||
      hipHostMalloc((void **)&d->h_done, 8 * ring_capacity, hflags) != hipSuccess ||
      hipHostMalloc((void **)&d->h_live, 8 * ring_capacity, hflags) != hipSuccess) {
    (void)hipGetLastError();
    free_drain(d);
    return HIVE_ERR_OOM;
  }
  memset(d->h_ring, 0, sizeof(ReqDesc) * ring_capacity);
  memset(d->h_done, 0, 8 * ring_capacity);
  memset(d->h_live, 0, 8 * ring_capacity);
  *d->h_tail = 0;
  *d->h_stop = 1;
  DrainQueue q;
  memset(&q, 0, sizeof(q));
  q.req = d->d_req;
  q.cap = ring_capacity;
  q.table_next = d->d_table_next;
  {
    // the watchdog runs on the constant-rate device clock; its rate is
    // measured here against the host clock rather than taken on trust
    double ticks_per_us = 0;
    if (wall_clock_rate(&ticks_per_us) != HIVE_OK) {
      free_drain(d);
      return HIVE_ERR_HIP;
    }
    const double us = idle_timeout_us ? (double)idle_timeout_us : 30e6;
    const double ticks = us * ticks_per_us;
    q.idle_ticks = ticks >= 1.8e19 ? ~0ull : (uint64_t)ticks;
  }
  void *dp = nullptr;
  if (hipHostGetDevicePointer(&dp, d->h_ring, 0) != hipSuccess) goto fail;
  q.host_ring = (const ReqDesc *)dp;
  if (hipHostGetDevicePointer(&dp, d->h_tail, 0) != hipSuccess) goto fail;
  q.host_tail = (const uint64_t *)dp;
  if (hipHostGetDevicePointer(&dp, d->h_stop, 0) != hipSuccess) goto fail;
  q.host_stop = (const uint32_t *)dp;
  if (hipHostGetDevicePointer(&dp, d->h_done, 0) != hipSuccess) goto fail;
  q.host_done = (uint64_t *)dp;
  if (hipHostGetDevicePointer(&dp, d->h_live, 0) != hipSuccess) goto fail;
  q.host_live = (uint64_t *)dp;
  if (hipMemcpy(d->d_q, &q, sizeof(q), hipMemcpyHostToDevice) != hipSuccess) goto fail;
  if (hipMemset(d->d_req, 0, sizeof(ReqState) * ring_capacity) != hipSuccess) goto fail;
  if (hipMemset(d->d_table_next, 0, 8ull * max_tables) != hipSuccess) goto fail;
  if (hipStreamCreateWithFlags(&d->capture, hipStreamNonBlocking) != hipSuccess) goto fail;
  if (hipDeviceSynchronize() != hipSuccess) goto fail;
  *out = d;
  return HIVE_OK;
fail:
  (void)hipGetLastError();
  free_drain(d);
  return HIVE_ERR_HIP;
}

hive_status hive_drain_submit(hive_drain_t d, hive_t h, const hive_batch_desc *b, uint64_t *ticket) {
  if (!d || !h || !b || !ticket) return HIVE_ERR_ARG;
  if (h->S != d->S) return HIVE_ERR_ARG;
  // the executor runs BitHash1/2 tables of 64-bit entries only
  if (h->cfg.hash_pair != HIVE_PAIR_BITHASH || h->entry_bytes != 8) return HIVE_ERR_ARG;
  if (b->op_mode > HIVE_OP_MIXED) return HIVE_ERR_ARG;
  if (b->n > 0 && !b->d_keys) return HIVE_ERR_ARG;
  if ((b->op_mode == HIVE_OP_INSERT || b->op_mode == HIVE_OP_MIXED) && b->n > 0 && !b->d_vals) return HIVE_ERR_ARG;
  if (b->op_mode == HIVE_OP_MIXED && b->n > 0 && !b->d_ops) return HIVE_ERR_ARG;
  if (b->n >= 0xFFFFFFFFull || (b->flags & ~(uint32_t)HIVE_UNIQUE)) return HIVE_ERR_ARG;
  const uint64_t t = d->submitted;
  // the ring slot must be free: the batch `cap` tickets earlier is complete
  if (t >= d->cap && __atomic_load_n(&d->h_done[t % d->cap], __ATOMIC_ACQUIRE) != t - d->cap + 1)
    return HIVE_ERR_BUDGET;
  // table slot (tables registered on first use)
  uint32_t slot = 0;
  while (slot < d->n_tables && d->tables[slot] != h) ++slot;
  if (slot == d->n_tables) {
    if (d->n_tables >= d->max_tables) return HIVE_ERR_BUDGET;
    d->tables[slot] = h;
    d->next_seq[slot] = 0;
    d->n_tables++;
  }
  const bool dedupe = !(b->flags & HIVE_UNIQUE) && b->op_mode != HIVE_OP_LOOKUP;
  const uint64_t dd_size = (dedupe && b->n > 0) ? dd_set_words(b->n) : 0;
  // scratch is never reallocated under a running executor; only inserts
  // reach the eviction worklist, while the dedupe set holds every operation
  const uint64_t wl_need = (b->op_mode == HIVE_OP_INSERT || b->op_mode == HIVE_OP_MIXED) ? b->n : 0;
  if (wl_need > h->wl_cap || dd_size > h->dd_cap) {
    if (d->running) return HIVE_ERR_ARG;
    hive_status s = ensure_scratch(h, wl_need, dd_size ? b->n : 0, h->last);
    if (s != HIVE_OK) return s;
  }
  if (wl_need > h->wl_cap || dd_size > h->dd_cap) return HIVE_ERR_OOM;  // cannot happen after a good grow
  ReqDesc r;
  memset(&r, 0, sizeof(r));
  r.t = TableDesc{h->d_buckets,    h->d_hint,  h->d_stash,   h->d_pending, h->d_ctl, h->d_wl, h->d_dd,
                  h->wl_seg_cap,  h->stash_cap,
                  h->pending_cap, hint_words(h->max_buckets), h->S, h->cfg.max_evictions, h->cfg.resize_k,
                  h->cfg.lf_expand_pct, h->cfg.lf_contract_pct, h->cfg.pre_expand, h->cfg.post_policy,
                  h->cfg.addressing};
  r.ops = b->d_ops;
  r.keys = b->d_keys;
  r.vals = b->d_vals;
  r.vals_out = b->d_vals_out;
  r.flags_out = b->d_flags_out;
  r.n = b->n;
  r.mode = b->op_mode;
  r.flags = b->flags;
  r.seq = d->next_seq[slot]++;
  r.table_slot = slot;
  r.ticket = t;
  r.dd_size = dd_size;
  memcpy(&d->h_ring[t % d->cap], &r, sizeof(r));
  __atomic_thread_fence(__ATOMIC_RELEASE);
  __atomic_store_n(d->h_tail, t + 1, __ATOMIC_RELEASE);
  d->submitted = t + 1;
  *ticket = t;
  return HIVE_OK;
}

hive_status hive_drain_launch(hive_drain_t d, int resident, void *stream) {
  if (!d || d->running) return HIVE_ERR_ARG;
  const int mode = resident ? 1 : 0;
  // a resident grid that fills every CU leaves no room for the process's
  // other kernels (HIP's own copy kernels included), which the host may wait
  // on before its next submission: the grid then idles until its watchdog
  // (the resident grid takes at most fit_per_cu - 1 blocks per CU)
  if (resident && d->fit_per_cu < 2) {
    fprintf(stderr, "hive: a resident executor grid needs room for a second block per compute unit "
                    "(the worker fits %d per CU)\n", d->fit_per_cu);
    return HIVE_ERR_BUDGET;
  }
  hipStream_t user = (hipStream_t)stream;
  // a resident grid runs on the executor's own non-blocking stream, after the
  // work already enqueued on `stream`, so it holds up no other stream
  hipStream_t st = resident ? d->capture : user;
  if (resident) {
    hipEvent_t ev;
    HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_OK(hipEventRecord(ev, user));
    HIP_OK(hipStreamWaitEvent(st, ev, 0));
    HIP_OK(hipEventDestroy(ev));
  }
  __atomic_store_n(d->h_stop, resident ? 0u : 1u, __ATOMIC_RELEASE);
  // the grid of the previous launch has exited; clear its exit flag
  hipLaunchKernelGGL(drain_reset_kernel, dim3(1), dim3(1), 0, st, d->d_q);
  HIP_OK(hipGetLastError());
  if (!d->exec[mode]) {
    // each launch form is captured once; replays read everything dynamic
    // from the queue in memory
    HIP_OK(hipStreamBeginCapture(d->capture, hipStreamCaptureModeRelaxed));
    launch_drain_any(d, mode, d->capture);
    hipError_t e = hipGetLastError();
    hipError_t e2 = hipStreamEndCapture(d->capture, &d->graph[mode]);
    if (e != hipSuccess || e2 != hipSuccess) {
      fprintf(stderr, "hive: drain graph capture failed: %s / %s\n", hipGetErrorString(e), hipGetErrorString(e2));
      return HIVE_ERR_HIP;
    }
    HIP_OK(hipGraphInstantiate(&d->exec[mode], d->graph[mode], nullptr, nullptr, 0));
  }
  HIP_OK(hipGraphLaunch(d->exec[mode], st));
  d->running = resident != 0;
  d->running_on = st;
  return HIVE_OK;
}

hive_status hive_drain_poll(hive_drain_t d, uint64_t ticket, int *done) {
  if (!d || !done || ticket >= d->submitted) return HIVE_ERR_ARG;
  if (d->submitted - ticket > d->cap) {
    *done = 1;  // its slot has been reused, so it completed long ago
    return HIVE_OK;
  }
  *done = __atomic_load_n(&d->h_done[ticket % d->cap], __ATOMIC_ACQUIRE) == ticket + 1;
  return HIVE_OK;
}

hive_status hive_drain_result(hive_drain_t d, uint64_t ticket, int *done, uint64_t *live_after) {
  if (!d || !done || !live_after || ticket >= d->submitted || d->submitted - ticket > d->cap) return HIVE_ERR_ARG;
  *done = __atomic_load_n(&d->h_done[ticket % d->cap], __ATOMIC_ACQUIRE) == ticket + 1;
  *live_after = *done ? __atomic_load_n(&d->h_live[ticket % d->cap], __ATOMIC_RELAXED) : 0;
  return HIVE_OK;
}

hive_status hive_drain_results(hive_drain_t d, const uint64_t *tickets, uint64_t n, uint8_t *done,
                               uint64_t *live_after) {
  if (!d || (n && (!tickets || !done || !live_after))) return HIVE_ERR_ARG;
  for (uint64_t i = 0; i < n; ++i)
    if (tickets[i] >= d->submitted || d->submitted - tickets[i] > d->cap) return HIVE_ERR_ARG;
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t t = tickets[i];
    done[i] = __atomic_load_n(&d->h_done[t % d->cap], __ATOMIC_ACQUIRE) == t + 1;
    live_after[i] = done[i] ? __atomic_load_n(&d->h_live[t % d->cap], __ATOMIC_RELAXED) : 0;
  }
  return HIVE_OK;
}

hive_status hive_drain_stop(hive_drain_t d, void *stream) {
  if (!d) return HIVE_ERR_ARG;
  (void)stream;
  __atomic_store_n(d->h_stop, 1u, __ATOMIC_RELEASE);
  d->running = false;
  HIP_OK(hipStreamSynchronize(d->running_on));
  uint32_t err = 0;
  HIP_OK(hipMemcpy(&err, (char *)d->d_q + offsetof(DrainQueue, error), 4, hipMemcpyDeviceToHost));
  return err ? HIVE_ERR_HIP : HIVE_OK;
}

hive_status hive_drain_destroy(hive_drain_t d) {
  if (!d) return HIVE_ERR_ARG;
  if (d->running) {
    __atomic_store_n(d->h_stop, 1u, __ATOMIC_RELEASE);
    (void)hipStreamSynchronize(d->running_on);
  }
  (void)hipDeviceSynchronize();
  free_drain(d);
  return HIVE_OK;
}

uint64_t hive_fastmod_magic(uint32_t d) { return fastmod_magic(d); }
uint32_t hive_fastmod(uint32_t a, uint64_t magic, uint32_t d) { return fastmod(a, magic, d); }

}  // extern "C"
