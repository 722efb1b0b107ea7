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
//           hand goes to the stash ring, or the pending list when the ring is
//           full (Section IV-A step 4).
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
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>

#include "hive.h"
#include "hive_device.hpp"

namespace hive {

constexpr int WAVES = 4;  // waves per block
constexpr int BLOCK = 64 * WAVES;
constexpr int EVICT_GRID = 1024;  // blocks of the eviction phase (grid-stride)
constexpr int RESIZE_GRID = 2048; // blocks of a resize pass (grid-stride over pairs)
constexpr int DRAIN_GRID = 256;

template <int S>
struct Traits {
  static_assert(S == 16 || S == 32 || S == 64, "slots per bucket must be 16, 32 or 64");
  static constexpr int G = 64 / S;  // buckets probed by one wave-wide load
  static constexpr int CH = 16;     // loads in flight per chunk of a probe round
  static constexpr int OPS_PER_CHUNK = CH * G;
  using Mask = typename std::conditional<(S <= 32), uint32_t, uint64_t>::type;
  static constexpr uint64_t FULL = (S == 64) ? ~0ull : ((1ull << S) - 1ull);
};

__device__ inline int ctz_mask(uint32_t m) { return __builtin_ctz(m); }
__device__ inline int ctz_mask(uint64_t m) { return __builtin_ctzll(m); }
__device__ inline int popc_mask(uint32_t m) { return __builtin_popcount(m); }
__device__ inline int popc_mask(uint64_t m) { return __builtin_popcountll(m); }

__device__ inline uint64_t read_lane64(uint64_t x, int lane) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

struct OpsArgs {
  uint64_t *buckets;
  uint32_t *hint;
  uint64_t *stash;
  uint64_t *pending;
  Ctl *ctl;
  uint64_t *wl;
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

__global__ __launch_bounds__(BLOCK) void dedupe_build_kernel(uint64_t *dd, uint64_t mask, uint32_t mode,
                                                             const uint8_t *ops, const uint32_t *keys, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  const uint32_t op = (mode == OP_MIXED) ? ops[i] : mode;
  const uint32_t k = keys[i];
  if (op > OP_DELETE || !valid_key(k)) return;
  const uint64_t e = ((uint64_t)k << 32) | (uint32_t)i;
  uint64_t s = mix32(k) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    uint64_t cur = dd[s];
    if (cur == EMPTY) {
      cur = cas64(&dd[s], EMPTY, e);
      if (cur == EMPTY) return;
    }
    if ((uint32_t)(cur >> 32) == k) {
      if (op == OP_INSERT)
        __hip_atomic_fetch_max(&dd[s], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else
        __hip_atomic_fetch_min(&dd[s], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    s = (s + 1) & mask;
  }
}

__device__ inline bool dedupe_winner(const uint64_t *dd, uint64_t mask, uint32_t k, uint32_t i) {
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

// One probe round of match-and-elect: for each of `count` operations (ops
// list[t], or t when list is null) the 16-lane group loads bucket bkt[o] and
// publishes, through LDS, the match mask, the empty-slot mask and the word of
// the lowest matching slot.
template <int S>
__device__ inline void probe_round(const uint64_t *__restrict__ buckets, const uint32_t *key, const uint32_t *bkt,
                                   const uint8_t *list, int count, typename Traits<S>::Mask *m_out,
                                   typename Traits<S>::Mask *e_out, uint64_t *w_out, int g, int sl) {
  using T = Traits<S>;
  using Mask = typename T::Mask;
  for (int base = 0; base < count; base += T::OPS_PER_CHUNK) {
    uint64_t w[T::CH];
#pragma unroll
    for (int j = 0; j < T::CH; ++j) {
      w[j] = EMPTY;
      const int t = base + j * T::G + g;
      if (base + j * T::G < count && t < count) {
        const int o = list ? list[t] : t;
        if (key[o] != 0u) w[j] = buckets[(uint64_t)bkt[o] * S + sl];
      }
    }
#pragma unroll
    for (int j = 0; j < T::CH; ++j) {
      if (base + j * T::G < count) {
        const int t = base + j * T::G + g;
        const bool mine = t < count;
        const int o = mine ? (list ? list[t] : t) : 0;
        const uint32_t ko = mine ? key[o] : 0u;
        const uint64_t mm = ballot(ko != 0u && key_of(w[j]) == ko);
        const uint64_t ee = ballot(w[j] == EMPTY);
        const Mask gm = (Mask)((mm >> (g * S)) & T::FULL);
        const Mask ge = (Mask)((ee >> (g * S)) & T::FULL);
        if (mine) {
          if (sl == 0) {
            m_out[o] = gm;
            e_out[o] = ge;
          }
          if (gm != 0 && sl == ctz_mask(gm)) w_out[o] = w[j];
        }
      }
    }
  }
}

__device__ inline bool hinted(const uint32_t *hint, uint32_t c1, uint32_t c2) {
  return ((hint[c1 >> 5] >> (c1 & 31)) & 1u) | ((hint[c2 >> 5] >> (c2 & 31)) & 1u);
}

// Lane-wise search of the stash ring and the pending list.
__device__ inline uint64_t *overflow_find(uint64_t *stash, uint64_t n_stash, uint64_t *pending, uint64_t n_pend,
                                          uint32_t k, uint64_t *word, bool fresh) {
  for (uint64_t p = 0; p < n_stash; ++p) {
    const uint64_t x = fresh ? load_fresh(stash + p) : stash[p];
    if (key_of(x) == k) {
      *word = x;
      return stash + p;
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

// Lane-wise search of the two candidate buckets with fresh (L2) loads.
template <int S>
__device__ inline uint64_t *bucket_find_fresh(uint64_t *buckets, uint32_t c1, uint32_t c2, uint32_t k,
                                              uint64_t *word) {
  for (int j = 0; j < 2; ++j) {
    const uint32_t b = j ? c2 : c1;
    if (j && c2 == c1) break;
    for (int s = 0; s < S; ++s) {
      const uint64_t x = load_fresh(buckets + (uint64_t)b * S + s);
      if (key_of(x) == k) {
        *word = x;
        return buckets + (uint64_t)b * S + s;
      }
    }
  }
  return nullptr;
}

// ---------------------------------------------------------------------------
// P1: hash, probe, and replace / lookup / delete / claim.
// ---------------------------------------------------------------------------
template <int S, uint32_t MODE>
__global__ __launch_bounds__(BLOCK) void ops_kernel(OpsArgs a) {
  using T = Traits<S>;
  using Mask = typename T::Mask;
  __shared__ uint32_t s_key[WAVES][64];
  __shared__ uint32_t s_b1[WAVES][64];
  __shared__ uint32_t s_b2[WAVES][64];
  __shared__ uint8_t s_list[WAVES][64];
  __shared__ Mask s_m[2][WAVES][64];
  __shared__ Mask s_e[2][WAVES][64];
  __shared__ uint64_t s_w[2][WAVES][64];

  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / S, sl = lane % S;
  const uint64_t i = ((uint64_t)blockIdx.x * WAVES + wv) * 64 + lane;
  const bool active = i < a.n;
  const Geo geo = read_geo(a.ctl);
  const uint64_t n_stash = min(a.ctl->stash_count, a.stash_cap);
  const uint64_t n_pend = min(a.ctl->pending_count, a.pending_cap);
  const bool overflow_used = (n_stash | n_pend) != 0;

  uint32_t op = OP_NONE, k = 0, v = 0;
  if (active) {
    op = (MODE == OP_MIXED) ? (uint32_t)a.ops[i] : MODE;
    k = a.keys[i];
    if (op == OP_INSERT) v = a.vals[i];
  }
  const bool valid = active && op <= OP_LOOKUP && valid_key(k);
  bool work = valid;
  if (work && a.dd && op != OP_LOOKUP) work = dedupe_winner(a.dd, a.dd_mask, k, (uint32_t)i);
  uint32_t c1 = 0, c2 = 0;
  if (work) {
    c1 = address(geo, bithash1(k));
    c2 = address(geo, bithash2(k));
  }
  s_key[wv][lane] = work ? k : 0u;
  s_b1[wv][lane] = c1;
  s_b2[wv][lane] = c2;
  wave_lds_sync();

  // round 1: first candidate of every operation
  probe_round<S>(a.buckets, s_key[wv], s_b1[wv], nullptr, 64, s_m[0][wv], s_e[0][wv], s_w[0][wv], g, sl);
  wave_lds_sync();
  const Mask m1 = s_m[0][wv][lane], e1 = s_e[0][wv][lane];
  const bool need2 = work && m1 == 0 && c2 != c1;
  const uint64_t need2_mask = ballot(need2);
  const int n2 = __popcll(need2_mask);
  if (need2) s_list[wv][rank_below(need2_mask)] = (uint8_t)lane;
  wave_lds_sync();
  // round 2: second candidate of the operations that missed in the first
  if (n2 > 0)
    probe_round<S>(a.buckets, s_key[wv], s_b2[wv], s_list[wv], n2, s_m[1][wv], s_e[1][wv], s_w[1][wv], g, sl);
  wave_lds_sync();
  const Mask m2 = need2 ? s_m[1][wv][lane] : (Mask)0;
  const Mask e2 = need2 ? s_e[1][wv][lane] : (Mask)0;

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
    } else if (overflow_used && hinted(a.hint, c1, c2)) {
      slot = overflow_find(a.stash, n_stash, a.pending, n_pend, k, &word, false);
    }
    if (op == OP_LOOKUP) {
      if (slot) {
        out_v = value_of(word);
        out_f = 1;
      }
    } else if (slot) {
      // replace (Algorithm 1) or delete (Algorithm 4): one CAS from the word
      // seen.  Only operations on this key may change its word, and the
      // batch contract gives each key one such operation, so the CAS fails
      // only when that contract is broken; then search again with fresh
      // loads.
      bool done = false;
      for (int attempt = 0; attempt < 4 && slot; ++attempt) {
        // a deleted bucket slot becomes EMPTY, a deleted stash/pending entry TOMB
        const uint64_t desired = (op == OP_INSERT) ? kv : (in_bucket ? EMPTY : TOMB);
        if (cas64(slot, word, desired) == word) {
          done = true;
          break;
        }
        atomicOr(&a.ctl->error, ERR_CAS_RETRY);
        slot = bucket_find_fresh<S>(a.buckets, c1, c2, k, &word);
        in_bucket = slot != nullptr;
        if (!slot) slot = overflow_find(a.stash, n_stash, a.pending, n_pend, k, &word, true);
      }
      if (op == OP_DELETE && done) {
        out_f = 1;
        dl = -1;
      }
    } else if (op == OP_INSERT) {
      // claim-then-commit (Algorithm 2) in the candidate with more empty
      // slots first, ties to the first hash: bucketed two-choice placement
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
      bool placed = false;
      while (!placed && (f_first | f_second)) {
        if (f_first == 0) {
          f_first = f_second;
          f_second = 0;
          b_first = b_second;
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

  // eviction worklist: one atomic per wave
  const uint64_t wl_mask = ballot(to_wl);
  if (wl_mask) {
    const int leader = __builtin_ctzll(wl_mask);
    uint64_t base = 0;
    if (lane == leader) base = add64(&a.ctl->wl_count, (uint64_t)__popcll(wl_mask));
    base = read_lane64(base, leader);
    if (to_wl) a.wl[base + rank_below(wl_mask)] = kv;
  }
  const uint64_t up = ballot(dl > 0), down = ballot(dl < 0), bad = ballot(active && !valid);
  if (lane == 0) {
    const int64_t d = (int64_t)__popcll(up) - (int64_t)__popcll(down);
    if (d != 0) add64(&a.ctl->live, (uint64_t)d);
    if (bad) add64(&a.ctl->invalid_keys, (uint64_t)__popcll(bad));
  }
  if (active) {
    if (MODE == OP_LOOKUP || MODE == OP_MIXED) {
      if (a.vals_out) a.vals_out[i] = out_v;
      if (a.flags_out) a.flags_out[i] = out_f;
    } else if (MODE == OP_DELETE) {
      if (a.flags_out) a.flags_out[i] = out_f;
    }
  }
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
  const uint64_t *wl;
  uint64_t stash_cap;
  uint64_t pending_cap;
  uint32_t max_evictions;
};

// Claim any empty slot of a bucket with one CAS (lowest slot first).
template <int S>
__device__ inline bool claim_lane(uint64_t *bkt, uint64_t kv) {
  for (int s = 0; s < S; ++s) {
    const uint64_t w = load_fresh(bkt + s);
    if (w == EMPTY && cas64(bkt + s, EMPTY, kv) == EMPTY) return true;
  }
  return false;
}

template <int S>
__device__ inline int count_empty_lane(const uint64_t *bkt) {
  int n = 0;
  for (int s = 0; s < S; ++s) n += load_fresh(bkt + s) == EMPTY;
  return n;
}

// Step 2 for one item (lane-wise): the candidate with more empty slots
// first, ties to the first hash, then the other candidate.
template <int S>
__device__ inline bool two_choice_claim_lane(uint64_t *buckets, uint32_t c1, uint32_t c2, uint64_t kv) {
  uint32_t first = c1, second = c2;
  if (c2 != c1 && count_empty_lane<S>(buckets + (uint64_t)c2 * S) > count_empty_lane<S>(buckets + (uint64_t)c1 * S)) {
    first = c2;
    second = c1;
  }
  if (claim_lane<S>(buckets + (uint64_t)first * S, kv)) return true;
  return second != first && claim_lane<S>(buckets + (uint64_t)second * S, kv);
}

// Put kv into slot s0 (or the next slots) by CAS, displacing the occupant.
// Returns 1 with *victim set, 2 when the slot turned out empty (claimed), 0
// when every CAS lost a race.
template <int S>
__device__ inline int displace_lane(uint64_t *bkt, uint64_t kv, int s0, uint64_t *victim) {
  for (int t = 0; t < S; ++t) {
    const int s = (s0 + t) & (S - 1);
    uint64_t cur = load_fresh(bkt + s);
    for (int attempt = 0; attempt < 4; ++attempt) {
      const uint64_t found = cas64(bkt + s, cur, kv);
      if (found == cur) {
        if (cur == EMPTY) return 2;
        *victim = cur;
        return 1;
      }
      cur = found;
    }
  }
  return 0;
}

__device__ inline void set_hint(uint32_t *hint, uint32_t b) { or32(&hint[b >> 5], 1u << (b & 31)); }

__device__ inline void overflow_push(const EvictArgs &a, const Geo &geo, uint64_t kv) {
  bool stashed = false;
  uint64_t c = load_fresh(&a.ctl->stash_count);
  while (c < a.stash_cap) {
    const uint64_t found = cas64(&a.ctl->stash_count, c, c + 1);
    if (found == c) {
      __hip_atomic_store(a.stash + c, kv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      stashed = true;
      break;
    }
    c = found;
  }
  if (stashed) {
    add64(&a.ctl->stash_inserts, 1);
  } else {
    const uint64_t p = add64(&a.ctl->pending_count, 1);
    if (p < a.pending_cap) {
      __hip_atomic_store(a.pending + p, kv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      add64(&a.ctl->pending_inserts, 1);
    } else {
      atomicOr(&a.ctl->error, ERR_PENDING_LOST);
    }
  }
  const uint32_t k = key_of(kv);
  set_hint(a.hint, address(geo, bithash1(k)));
  set_hint(a.hint, address(geo, bithash2(k)));
}

template <int S>
__global__ __launch_bounds__(BLOCK) void evict_kernel(EvictArgs a) {
  const Geo geo = read_geo(a.ctl);
  const uint64_t cnt = a.ctl->wl_count;
  uint64_t n_evict = 0, n_full = 0;
  for (uint64_t t = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; t < cnt; t += (uint64_t)gridDim.x * BLOCK) {
    uint64_t kv = a.wl[t];
    const uint32_t k1 = address(geo, bithash1(key_of(kv))), k2 = address(geo, bithash2(key_of(kv)));
    // step 2 once more with fresh loads (items from P1 saw both buckets full,
    // possibly through a stale cache line; items drained from the stash after
    // a split have not tried the new geometry), then the chain from the first
    // candidate
    bool placed = two_choice_claim_lane<S>(a.buckets, k1, k2, kv);
    uint32_t b = k1;
    for (uint32_t kick = 1; kick <= a.max_evictions && !placed; ++kick) {
      uint64_t *bkt = a.buckets + (uint64_t)b * S;
      if (claim_lane<S>(bkt, kv)) {
        placed = true;
        break;
      }
      // victim: a pseudo-random slot (the paper's "first occupied" slot is
      // always slot 0 of a full bucket, which lets two chains swap the same
      // pair of entries back and forth)
      uint64_t victim = 0;
      const int s0 = (int)(mix32(key_of(kv) ^ (kick * 0x9E3779B9u)) & (S - 1));
      const int r = displace_lane<S>(bkt, kv, s0, &victim);
      if (r == 2) {
        placed = true;
        break;
      }
      if (r == 0) continue;  // every CAS raced: count the round, keep the item
      ++n_evict;
      kv = victim;
      const uint32_t v1 = address(geo, bithash1(key_of(kv)));
      const uint32_t v2 = address(geo, bithash2(key_of(kv)));
      b = (b == v1) ? v2 : v1;  // AltBucket: the victim's other candidate
    }
    if (!placed) {
      ++n_full;
      overflow_push(a, geo, kv);
    }
  }
  if (n_evict) add64(&a.ctl->evictions, n_evict);
  if (n_full) add64(&a.ctl->full_chains, n_full);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (blockIdx.x == 0 && cnt) add64(&a.ctl->evict_items, cnt);
    // the last block to finish has seen every block read wl_count: reset it
    const uint64_t done = add64(&a.ctl->p3_done, 1);
    if (done == gridDim.x - 1) {
      __hip_atomic_store(&a.ctl->wl_count, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.ctl->p3_done, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
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
__device__ inline void plan_next(Ctl *c) {
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
__device__ inline void plan_policy(Ctl *c, const ResizeArgs &a, uint64_t extra, bool allow_contract) {
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

__global__ __launch_bounds__(BLOCK) void resize_plan_kernel(ResizeArgs a, uint32_t mode, uint64_t amount,
                                                            const uint8_t *ops) {
  __shared__ unsigned long long n_ins;
  if (threadIdx.x == 0) n_ins = 0;
  __syncthreads();
  if (mode == PLAN_PRE_MIXED) {
    unsigned long long mine = 0;
    for (uint64_t i = threadIdx.x; i < amount; i += BLOCK) mine += ops[i] == OP_INSERT;
    atomicAdd(&n_ins, mine);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  Ctl *c = a.ctl;
  c->resize_dir = 0;
  c->resize_todo = 0;
  c->ticket = 0;
  if (c->mode != ADDR_LINEAR) {
    c->seg = 0;
    return;
  }
  switch (mode) {
    case PLAN_PRE: plan_policy(c, a, amount, false); break;
    case PLAN_PRE_MIXED: plan_policy(c, a, n_ins, false); break;
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

// Ticket for "the last block of this launch": every block has finished its
// reads of the control block and its writes to the table.
__device__ inline bool last_block(uint64_t *ticket) {
  __shared__ bool last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = add64(ticket, 1) == gridDim.x - 1;
  }
  __syncthreads();
  return last;
}

__device__ inline uint32_t nth_set_bit(uint64_t m, uint32_t r) {
  for (uint32_t i = 0; i < r; ++i) m &= m - 1;
  return (uint32_t)__builtin_ctzll(m);
}

// Pass 1: split the segment's pairs (Section IV-C-1), or test merge pairs.
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
    if (dir > 0) {
      // pair (src, src + 2^m): an entry stays when one of its candidate
      // hashes still addresses src under the next round's mask, otherwise
      // it moves; movers are compacted into the partner's first slots
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
    } else {
      // merge pair (lo, lo + 2^m), walked from the top: it fits when hi's
      // entries fit lo's empty slots (Section IV-C-2)
      const uint64_t lo = sp - 1 - j, hi = lo + im + 1;
      const uint64_t wl = a.buckets[lo * S + sl], wh = a.buckets[hi * S + sl];
      const uint64_t fl = (ballot(wl == EMPTY) >> (g * S)) & T::FULL;
      const uint64_t lh = (ballot(wh != EMPTY) >> (g * S)) & T::FULL;
      if (sl == 0 && __builtin_popcountll(lh) > __builtin_popcountll(fl))
        __hip_atomic_fetch_min(&c->merge_commit, j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (dir > 0 && last_block(&c->ticket)) {
    c->ticket = 0;
    c->sp = sp + seg;
    c->n_buckets += seg;
    c->resize_todo -= seg;
    c->split_happened = 1;
    plan_next(c);
  }
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
  for (uint64_t j = ((uint64_t)blockIdx.x * WAVES + wv) * T::G + g; j < commit; j += groups) {
    const uint64_t lo = sp - 1 - j, hi = lo + im + 1;
    const uint64_t wl = a.buckets[lo * S + sl], wh = a.buckets[hi * S + sl];
    const uint64_t fl = (ballot(wl == EMPTY) >> (g * S)) & T::FULL;
    const uint64_t lh = (ballot(wh != EMPTY) >> (g * S)) & T::FULL;
    if (wh != EMPTY) {
      // the r-th live entry of hi goes to the r-th empty slot of lo
      const uint32_t r = __builtin_popcountll(lh & ((1ull << sl) - 1ull));
      a.buckets[lo * S + nth_set_bit(fl, r)] = wh;
      a.buckets[hi * S + sl] = EMPTY;
    }
    // stash entries with a candidate in hi now address lo
    if (sl == 0 && ((a.hint[hi >> 5] >> (hi & 31)) & 1u)) set_hint(a.hint, (uint32_t)lo);
  }
  if (last_block(&c->ticket)) {
    c->ticket = 0;
    c->sp = sp - commit;
    c->n_buckets -= commit;
    c->resize_todo -= commit;
    if (commit < seg) c->resize_todo = 0;  // a pair did not fit: the call stops here
    plan_next(c);
  }
}

// After splits: move every stash and pending entry to the eviction worklist
// (they are re-placed by the eviction phase under the new geometry) and
// clear the hint bits (Section III-B "Overflow Stash").
__global__ __launch_bounds__(BLOCK) void drain_kernel(uint64_t *stash, uint64_t stash_cap, uint64_t *pending,
                                                      uint64_t pending_cap, uint32_t *hint, uint64_t hint_n,
                                                      uint64_t *wl, Ctl *c) {
  if (!c->split_happened) return;
  const uint64_t n_stash = min(c->stash_count, stash_cap);
  const uint64_t n_pend = min(c->pending_count, pending_cap);
  const uint64_t total = n_stash + n_pend;
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  const uint64_t tid = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (total) {
    for (uint64_t t = tid; t < hint_n; t += stride) hint[t] = 0u;
  }
  const uint64_t span = (total + stride - 1) / stride * stride;
  const int lane = threadIdx.x & 63;
  for (uint64_t t = tid; t < span; t += stride) {
    uint64_t w = TOMB;
    if (t < n_stash)
      w = stash[t];
    else if (t < total)
      w = pending[t - n_stash];
    const bool live = w != TOMB;
    const uint64_t m = ballot(live);
    if (m) {
      const int leader = __builtin_ctzll(m);
      uint64_t base = 0;
      if (lane == leader) base = add64(&c->wl_count, (uint64_t)__popcll(m));
      base = read_lane64(base, leader);
      if (live) wl[base + rank_below(m)] = w;
    }
  }
  if (last_block(&c->drain_ticket)) {
    c->drain_ticket = 0;
    c->stash_count = 0;
    c->pending_count = 0;
    c->split_happened = 0;
  }
}

// ---------------------------------------------------------------------------
// Dump: every live word with its place (bucket, -1 stash, -2 pending).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void dump_kernel(const uint64_t *buckets, uint32_t S, const uint64_t *stash,
                                                     const uint64_t *pending, Ctl *ctl, uint64_t stash_cap,
                                                     uint64_t pending_cap, uint64_t *out, int64_t *where,
                                                     uint64_t cap) {
  const uint64_t nb = ctl->n_buckets;
  const uint64_t n_stash = min(ctl->stash_count, stash_cap);
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
__global__ __launch_bounds__(BLOCK) void placement_kernel(const uint64_t *buckets, uint32_t S, Ctl *ctl) {
  const Geo geo = read_geo(ctl);
  const uint64_t n_slots = geo.n_buckets * S;
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  const uint64_t span = (n_slots + stride - 1) / stride * stride;
  for (uint64_t t = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; t < span; t += stride) {
    const uint64_t w = t < n_slots ? buckets[t] : EMPTY;
    const bool live = w != EMPTY;
    const bool first = live && address(geo, bithash1(key_of(w))) == (uint32_t)(t / S);
    const uint64_t mf = ballot(first), ms = ballot(live && !first);
    if ((threadIdx.x & 63) == 0) {
      if (mf) add64(&ctl->place_first, (uint64_t)__popcll(mf));
      if (ms) add64(&ctl->place_second, (uint64_t)__popcll(ms));
    }
  }
}

__global__ void ctl_zero_placement_kernel(Ctl *ctl) {
  ctl->place_first = 0;
  ctl->place_second = 0;
}

__global__ void ctl_reset_kernel(Ctl *ctl, Ctl init) { *ctl = init; }
__global__ void ctl_zero_dump_kernel(Ctl *ctl) { ctl->dump_count = 0; }

}  // namespace hive

// ===========================================================================
// Host side: the C ABI
// ===========================================================================
using namespace hive;

struct hive_table {
  hive_config cfg;
  uint32_t S;
  uint64_t initial_buckets;
  uint64_t max_buckets;
  uint64_t stash_cap, pending_cap;
  uint64_t *d_buckets = nullptr;
  uint32_t *d_hint = nullptr;
  uint64_t *d_stash = nullptr;
  uint64_t *d_pending = nullptr;
  Ctl *d_ctl = nullptr;
  uint64_t *d_wl = nullptr;
  uint64_t wl_cap = 0;
  uint64_t *d_dd = nullptr;
  uint64_t dd_cap = 0;  // power of two
  uint64_t bytes = 0;
  hipStream_t last = nullptr;
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
  if ((s = fill_u64(h->d_buckets, h->max_buckets * h->S, EMPTY, st)) != HIVE_OK) return s;
  if ((s = fill_u32(h->d_hint, hint_words(h->max_buckets), 0u, st)) != HIVE_OK) return s;
  hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(1), 0, st, h->d_ctl, initial_ctl(h));
  return launch_check();
}

static void free_table(hive_table *h) {
  if (!h) return;
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
  if (hipMalloc(p, bytes ? bytes : 8) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return HIVE_ERR_OOM;
  }
  *total += bytes;
  return HIVE_OK;
}

// Per-batch scratch (worklist and dedupe set) grows on demand; growing
// synchronizes the stream because the old buffers may still be in use.
static hive_status ensure_scratch(hive_table *h, uint64_t n, bool need_dd, hipStream_t st) {
  if (n > h->wl_cap) {
    HIP_OK(hipStreamSynchronize(st));
    (void)hipFree(h->d_wl);
    h->d_wl = nullptr;
    uint64_t cap = std::max<uint64_t>(n, 2 * h->wl_cap);
    h->bytes -= h->wl_cap * 8;
    h->wl_cap = 0;
    if (alloc((void **)&h->d_wl, cap * 8, &h->bytes) != HIVE_OK) return HIVE_ERR_OOM;
    h->wl_cap = cap;
  }
  if (need_dd) {
    uint64_t want = 16;
    while (want < 2 * n) want <<= 1;
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

template <int S, uint32_t MODE>
static void launch_ops(const OpsArgs &a, hipStream_t st) {
  const uint64_t blocks = (a.n + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL((ops_kernel<S, MODE>), dim3((unsigned)blocks), dim3(BLOCK), 0, st, a);
}

template <int S>
static void launch_ops_mode(uint32_t mode, const OpsArgs &a, hipStream_t st) {
  switch (mode) {
    case OP_INSERT: launch_ops<S, OP_INSERT>(a, st); break;
    case OP_DELETE: launch_ops<S, OP_DELETE>(a, st); break;
    case OP_LOOKUP: launch_ops<S, OP_LOOKUP>(a, st); break;
    default: launch_ops<S, OP_MIXED>(a, st); break;
  }
}

static void launch_evict(hive_table *h, hipStream_t st) {
  EvictArgs e{h->d_buckets, h->d_hint, h->d_stash, h->d_pending, h->d_ctl, h->d_wl,
              h->stash_cap, h->pending_cap, h->cfg.max_evictions};
  switch (h->S) {
    case 16: hipLaunchKernelGGL(evict_kernel<16>, dim3(EVICT_GRID), dim3(BLOCK), 0, st, e); break;
    case 32: hipLaunchKernelGGL(evict_kernel<32>, dim3(EVICT_GRID), dim3(BLOCK), 0, st, e); break;
    default: hipLaunchKernelGGL(evict_kernel<64>, dim3(EVICT_GRID), dim3(BLOCK), 0, st, e); break;
  }
}

// Upper bound on the hashing rounds one resize call can cross: from the
// initial bucket count to the arena size, plus the partial rounds at both
// ends.
static int resize_rounds(const hive_table *h) {
  int r = 2;
  for (uint64_t x = h->initial_buckets; x < h->max_buckets; x *= 2) ++r;
  return r;
}

template <int S>
static void launch_resize_passes(const ResizeArgs &ra, int rounds, hipStream_t st) {
  for (int r = 0; r < rounds; ++r) {
    hipLaunchKernelGGL(resize_pass1_kernel<S>, dim3(RESIZE_GRID), dim3(BLOCK), 0, st, ra);
    hipLaunchKernelGGL(resize_pass2_kernel<S>, dim3(RESIZE_GRID), dim3(BLOCK), 0, st, ra);
  }
}

static hive_status resize_sequence(hive_table *h, uint32_t mode, uint64_t amount, const uint8_t *d_ops,
                                   hipStream_t st) {
  ResizeArgs ra{h->d_buckets, h->d_hint, h->d_ctl, h->S, h->cfg.resize_k, h->cfg.lf_expand_pct,
                h->cfg.lf_contract_pct};
  hipLaunchKernelGGL(resize_plan_kernel, dim3(1), dim3(BLOCK), 0, st, ra, mode, amount, d_ops);
  const int rounds = resize_rounds(h);
  switch (h->S) {
    case 16: launch_resize_passes<16>(ra, rounds, st); break;
    case 32: launch_resize_passes<32>(ra, rounds, st); break;
    default: launch_resize_passes<64>(ra, rounds, st); break;
  }
  hipLaunchKernelGGL(drain_kernel, dim3(DRAIN_GRID), dim3(BLOCK), 0, st, h->d_stash, h->stash_cap, h->d_pending,
                     h->pending_cap, h->d_hint, hint_words(h->max_buckets), h->d_wl, h->d_ctl);
  launch_evict(h, st);
  return launch_check();
}

static hive_status run_batch(hive_t h, uint32_t mode, const uint8_t *d_ops, const uint32_t *d_keys,
                             const uint32_t *d_vals, uint64_t n, uint32_t flags, uint32_t *d_vals_out,
                             uint8_t *d_flags_out, void *stream) {
  if (!h || (n > 0 && !d_keys)) return HIVE_ERR_ARG;
  if (n >= 0xFFFFFFFFull) return HIVE_ERR_ARG;  // batch indices are 32-bit in the dedupe set
  if (mode == OP_INSERT && n > 0 && !d_vals) return HIVE_ERR_ARG;
  if (mode == OP_MIXED && n > 0 && !d_ops) return HIVE_ERR_ARG;
  if (flags & ~(uint32_t)HIVE_UNIQUE) return HIVE_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  h->last = st;
  if (n == 0) return HIVE_OK;
  const bool dedupe = !(flags & HIVE_UNIQUE) && mode != OP_LOOKUP;
  hive_status s = ensure_scratch(h, n, dedupe, st);
  if (s != HIVE_OK) return s;
  OpsArgs a{};
  a.buckets = h->d_buckets;
  a.hint = h->d_hint;
  a.stash = h->d_stash;
  a.pending = h->d_pending;
  a.ctl = h->d_ctl;
  a.wl = h->d_wl;
  a.ops = d_ops;
  a.keys = d_keys;
  a.vals = d_vals;
  a.vals_out = d_vals_out;
  a.flags_out = d_flags_out;
  a.n = n;
  a.stash_cap = h->stash_cap;
  a.pending_cap = h->pending_cap;
  if (dedupe) {
    uint64_t cap = 16;
    while (cap < 2 * n) cap <<= 1;
    if ((s = fill_u64(h->d_dd, cap, EMPTY, st)) != HIVE_OK) return s;
    hipLaunchKernelGGL(dedupe_build_kernel, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, h->d_dd,
                       cap - 1, mode, d_ops, d_keys, n);
    if ((s = launch_check()) != HIVE_OK) return s;
    a.dd = h->d_dd;
    a.dd_mask = cap - 1;
  }
  const bool linear = h->cfg.addressing == HIVE_LINEAR;
  if (linear && h->cfg.pre_expand && (mode == OP_INSERT || mode == OP_MIXED)) {
    // grow before the batch so that live + (inserts of the batch) fits
    if ((s = resize_sequence(h, mode == OP_MIXED ? PLAN_PRE_MIXED : PLAN_PRE, n, d_ops, st)) != HIVE_OK) return s;
  }
  switch (h->S) {
    case 16: launch_ops_mode<16>(mode, a, st); break;
    case 32: launch_ops_mode<32>(mode, a, st); break;
    default: launch_ops_mode<64>(mode, a, st); break;
  }
  if ((s = launch_check()) != HIVE_OK) return s;
  if (mode == OP_INSERT || mode == OP_MIXED) {
    launch_evict(h, st);
    if ((s = launch_check()) != HIVE_OK) return s;
  }
  if (linear && h->cfg.post_policy && mode != OP_LOOKUP) {
    if ((s = resize_sequence(h, PLAN_POST, 0, nullptr, st)) != HIVE_OK) return s;
  }
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
  h->initial_buckets = initial_buckets;
  h->max_buckets = max_b;
  h->stash_cap = cfg.stash_capacity ? cfg.stash_capacity : std::max<uint64_t>(1024, initial_buckets * S / 100);
  h->pending_cap = cfg.pending_capacity ? cfg.pending_capacity : h->stash_cap;
  cfg.stash_capacity = h->stash_cap;
  cfg.pending_capacity = h->pending_cap;
  cfg.max_buckets = max_b;
  h->cfg = cfg;
  hive_status s = HIVE_OK;
  if ((s = alloc((void **)&h->d_buckets, max_b * S * 8, &h->bytes)) != HIVE_OK ||
      (s = alloc((void **)&h->d_hint, hint_words(max_b) * 4, &h->bytes)) != HIVE_OK ||
      (s = alloc((void **)&h->d_stash, h->stash_cap * 8, &h->bytes)) != HIVE_OK ||
      (s = alloc((void **)&h->d_pending, h->pending_cap * 8, &h->bytes)) != HIVE_OK ||
      (s = alloc((void **)&h->d_ctl, sizeof(Ctl), &h->bytes)) != HIVE_OK) {
    free_table(h);
    return s;
  }
  hipStream_t st = (hipStream_t)stream;
  h->last = st;
  // the worklist must hold a full stash + pending drain (after a split)
  const uint64_t min_wl = h->stash_cap + h->pending_cap;
  if ((s = ensure_scratch(h, std::max<uint64_t>(cfg.max_batch, min_wl), cfg.max_batch > 0, st)) != HIVE_OK) {
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
  if (h && n > 0 && !d_vals) return HIVE_ERR_ARG;  // inserts read their values
  return run_batch(h, OP_MIXED, d_ops, d_keys, d_vals, n, flags, d_vals_out, d_flags_out, stream);
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
  hipStream_t st = (hipStream_t)stream;
  h->last = st;
  hipLaunchKernelGGL(ctl_zero_placement_kernel, dim3(1), dim3(1), 0, st, h->d_ctl);
  hive_status s = launch_check();
  if (s != HIVE_OK) return s;
  hipLaunchKernelGGL(placement_kernel, dim3(2048), dim3(BLOCK), 0, st, h->d_buckets, h->S, h->d_ctl);
  if ((s = launch_check()) != HIVE_OK) return s;
  Ctl c;
  HIP_OK(hipMemcpyAsync(&c, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  out[0] = c.place_first;
  out[1] = c.place_second;
  out[2] = std::min(c.stash_count, h->stash_cap) + std::min(c.pending_count, h->pending_cap);
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

uint64_t hive_fastmod_magic(uint32_t d) { return fastmod_magic(d); }
uint32_t hive_fastmod(uint32_t a, uint64_t magic, uint32_t d) { return fastmod(a, magic, d); }

}  // extern "C"
