// Device-side building blocks of the Hive table for gfx950 (64-lane waves).
//
// Layout in HBM (one table):
//   buckets  max_buckets * S packed words, 128-byte aligned; bucket b occupies
//            words [b*S, b*S + S): one 128-byte line for S = 16
//   hint     one bit per bucket: set when a key with this bucket as a
//            candidate was sent to the stash or pending list
//   stash    open-addressed table of packed words (Section IV-A step 4),
//            twice its capacity in slots; deleted entries become TOMB
//   pending  entries that found the stash full
//   ctl      the control block below
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hive {

// An unoccupied bucket slot: key half 0xFFFFFFFF (a reserved key), so no
// live entry ever equals it and a 0xFF byte fill empties a bucket.
constexpr uint64_t EMPTY = ~0ull;
// A deleted stash or pending entry: key half 0 (the other reserved key).
constexpr uint64_t TOMB = 0ull;
constexpr uint32_t NO_VALUE = 0xFFFFFFFFu;

enum : uint32_t { ADDR_FIXED = 0, ADDR_LINEAR = 1 };
enum : uint32_t { OP_INSERT = 0, OP_DELETE = 1, OP_LOOKUP = 2, OP_MIXED = 3, OP_NONE = 7 };

// Latched device conditions (ctl.error).
enum : uint32_t {
  ERR_PENDING_LOST = 1u,   // the pending list overflowed
  ERR_CAS_RETRY = 2u,      // a replace/delete found its word changed (contract breach)
  ERR_ARENA_FULL = 4u,     // a split found no arena room
};

// Control block, one per table, in device memory.  Geometry is read by every
// kernel at its start, so it may change between launches without host sync.
// It is four 128-byte lines, each written by a
// different kind of code, so that the line every probe block reads is never
// the target of atomics; then NSHARD shard lines for counters that many
// waves update (see Shard).
struct alignas(128) Ctl {
  // line 0: geometry (Section III-B global metadata, Section IV-C control
  // fields) and overflow sizes, read by every block of every launch;
  // written only between phases and by rare stash/pending appends
  uint64_t n_buckets;
  uint64_t magic;          // FIXED: fastmod multiplier for n_buckets
  uint64_t im;             // LINEAR: index mask 2^m - 1
  uint64_t sp;             // LINEAR: split pointer
  uint32_t mode;           // ADDR_FIXED / ADDR_LINEAR
  uint32_t pad_mode_;
  uint64_t stash_count;    // stash slots used (including TOMB)
  uint64_t pending_count;  // pending slots used (including TOMB; may pass capacity on loss)
  uint64_t pad0_[9];
  // line 1: totals, folded from the shards after each batch, and error bits
  uint64_t live;
  uint64_t evictions;
  uint64_t stash_inserts;
  uint64_t pending_inserts;
  uint64_t full_chains;
  uint64_t invalid_keys;
  uint64_t evict_items;
  uint32_t error;          // latched ERR_* bits
  uint32_t pad_err_;
  uint64_t pad1_[8];
  // line 2: resize bookkeeping (device-side policy, Section IV-C)
  int64_t resize_dir;      // +1 split, -1 merge, 0 idle
  uint64_t resize_todo;    // pairs the current resize call still has to do
  uint64_t seg;            // pairs of the current round segment
  uint64_t merge_commit;   // merge segment: pairs from the top that fit
  uint64_t ticket;         // last-block ticket, second level
  uint64_t split_happened; // a split ran since the last stash drain
  uint64_t initial_buckets;
  uint64_t max_buckets;
  uint64_t plan_inserts;   // insert operations of a mixed batch, counted for its pre-batch plan
  uint64_t pad2_[7];
  // line 3: maintenance kernels (dump, placement census)
  uint64_t dump_count;
  uint64_t place_first;
  uint64_t place_second;
  uint64_t pad3_[13];
};
static_assert(sizeof(Ctl) == 512, "four lines");

// Counters that every wave (or every group) updates live in NSHARD shards
// instead of one word: a device-scope atomic on one address serialises at
// the memory side, tens of nanoseconds each.  A writer picks its shard from
// its tile index; the totals in Ctl line 1 are folded from the shards once
// per batch.  Shards are SHARD_STRIDE bytes apart so that they fall in
// different memory channels.  wl_count is the fill of the shard's segment of
// the eviction worklist; ticket is the first level of the last-block ticket.
constexpr int NSHARD = 64;
constexpr uint64_t SHARD_STRIDE = 17 * 256;
struct Shard {
  uint64_t live;         // signed change of the key count (two's complement)
  uint64_t wl_count;
  uint64_t evictions;
  uint64_t full_chains;
  uint64_t invalid_keys;
  uint64_t ticket;
  uint64_t stash_inserts;
  uint64_t pending_inserts;
  uint64_t stash_unreserved;  // stash placements of launches that needed no reservation
};
constexpr uint64_t CTL_BYTES = sizeof(Ctl) + NSHARD * SHARD_STRIDE;

__device__ __host__ __forceinline__ Shard *shard_of(const Ctl *c, uint64_t s) {
  return (Shard *)((char *)(c + 1) + s * SHARD_STRIDE);
}

// ---- Section III-C hashes -------------------------------------------------
// BitHash1 and BitHash2 written as compositions of invertible maps of
// Z/2^32 (the final "% nBuckets" of the listing belongs to the addressing):
//   BitHash1: x -> 32767x - 1, then x ^= x>>12, x -> 5x, x ^= x>>4,
//             x -> 2057x, x ^= x>>16;
//   BitHash2: x -> 4097x + 0x7ed55d16, x -> x ^ 0xc761c23c ^ (x>>19),
//             x -> 33x + 0x165667b1, x -> (x + 0xd3a2646c) ^ (x<<9),
//             x -> 9x + 0xfd7046c5, x -> x ^ 0xb55a4f09 ^ (x>>16).
__host__ __device__ __forceinline__ uint32_t bithash1(uint32_t x) {
  x = x * 32767u - 1u;
  x ^= x >> 12;
  x *= 5u;
  x ^= x >> 4;
  x *= 2057u;
  return x ^ (x >> 16);
}

__host__ __device__ __forceinline__ uint32_t bithash2(uint32_t x) {
  x = x * 4097u + 0x7ed55d16u;
  x = x ^ 0xc761c23cu ^ (x >> 19);
  x = x * 33u + 0x165667b1u;
  x = (x + 0xd3a2646cu) ^ (x << 9);
  x = x * 9u + 0xfd7046c5u;
  return x ^ 0xb55a4f09u ^ (x >> 16);
}

// a % d without a divide (gfx950 has no integer divide): Lemire, Kaser and
// Kurz, "Faster remainder by direct computation" (2019).  magic = 2^64/d
// rounded up (wrapping to 0 for d = 1, which still yields 0).
__host__ __device__ __forceinline__ uint64_t fastmod_magic(uint32_t d) { return ~0ull / d + 1ull; }

__host__ __device__ __forceinline__ uint32_t fastmod(uint32_t a, uint64_t magic, uint32_t d) {
  uint64_t low = magic * a;
#if defined(__HIP_DEVICE_COMPILE__)
  return (uint32_t)__umul64hi(low, (uint64_t)d);
#else
  return (uint32_t)(((unsigned __int128)low * d) >> 64);
#endif
}

struct Geo {
  uint64_t n_buckets;
  uint64_t magic;
  uint32_t im, sp;
  uint32_t mode;
};

__host__ __device__ __forceinline__ uint32_t address(const Geo &g, uint32_t h) {
  if (g.mode == ADDR_FIXED) return fastmod(h, g.magic, (uint32_t)g.n_buckets);
  uint32_t a = h & g.im;
  if (a < g.sp) a = h & (2u * g.im + 1u);
  return a;
}

// Control-block fields are read with coherent vector loads: a plain uniform
// load may be served by the scalar cache, which an acquire fence does not
// invalidate, and the control block changes between the phases of the
// persistent executor.
__device__ __forceinline__ uint64_t ld_ctl(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_ctl32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ Geo read_geo(const Ctl *c) {
  Geo g;
  g.n_buckets = ld_ctl(&c->n_buckets);
  g.magic = ld_ctl(&c->magic);
  g.im = (uint32_t)ld_ctl(&c->im);
  g.sp = (uint32_t)ld_ctl(&c->sp);
  g.mode = ld_ctl32(&c->mode);
  return g;
}

__host__ __device__ __forceinline__ uint64_t pack(uint32_t key, uint32_t value) { return ((uint64_t)value << 32) | key; }
__host__ __device__ __forceinline__ uint32_t key_of(uint64_t w) { return (uint32_t)w; }
__host__ __device__ __forceinline__ uint32_t value_of(uint64_t w) { return (uint32_t)(w >> 32); }
__host__ __device__ __forceinline__ bool valid_key(uint32_t k) { return k != 0u && k != 0xFFFFFFFFu; }

// ---- wave helpers ---------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// LDS written by one lane of a wave and read by another lane of the same
// wave: LDS instructions of a wave complete in order, so a compiler-level
// fence is all that is needed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Device-scope (agent) relaxed atomics on 64-bit words.
__device__ __forceinline__ uint64_t cas64(uint64_t *p, uint64_t expected, uint64_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the word found (== expected on success)
}

__device__ __forceinline__ uint64_t load_fresh(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t add64(uint64_t *p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t or32(uint32_t *p, uint32_t v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The stash as an open-addressed table of words: at least twice its entry
// capacity, so that (the count of used slots, tombstones included, never
// exceeds the capacity) linear-probe runs stay short and an EMPTY word
// always ends a search.
__host__ __device__ __forceinline__ uint64_t stash_slots_for(uint64_t cap) {
  uint64_t s = 16;
  while (s < 2 * cap) s <<= 1;
  return s;
}

// Mix for the per-batch dedupe set and the eviction victim choice: the
// "lowbias32" integer hash published by C. Wellons (hash-prospector, 2018).
// It is not one of the bucket hashes, so it is independent of placement.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  return x ^ (x >> 16);
}

}  // namespace hive
