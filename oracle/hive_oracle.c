/* CPU oracle for the Hive hash table (Polak, Troendle, Jang, arXiv 2510.15095).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library under paper_2510_15095_amd/
 * may include, link or call this file; only the tests, the package's smoke
 * check and the benchmark's CPU-baseline leg load it.  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * Two models, both plain single-threaded C:
 *
 *   O1  the dictionary definition of the operations (Section III-D): a map M
 *       from valid 32-bit keys to 32-bit values; insert sets M[k] = v
 *       (insert-or-replace), delete reports whether k was present and erases
 *       it, lookup returns M[k] or "absent".  A batch is applied in index
 *       order.  This is the result the GPU must reproduce bit-exactly.
 *
 *   O2  a sequential model of the Hive table itself, taking the paper's steps
 *       in its order: packed 64-bit words (Section III-A), S-slot buckets with
 *       a per-bucket free mask (Section III-B), BitHash1/BitHash2
 *       (Section III-C), the four-step insert -- replace, claim-then-commit,
 *       bounded cuckoo eviction, overflow stash (Section IV-A, Algorithms 1-3)
 *       -- lookup and delete by match-and-elect (Section IV-B, Algorithm 4),
 *       and linear-hashing split and merge in K-bucket batches with the load
 *       factor policy (Section IV-C).  O2 gives the geometry (bucket count,
 *       index mask, split pointer) a resize sequence must reach and checks the
 *       structural invariants; its logical results are tested equal to O1's.
 *
 * Readings of passages the paper leaves open (each is also listed in the
 * design notes):
 *   - EMPTY is the all-ones word; keys 0 and 0xFFFFFFFF are reserved, so no
 *     live entry equals EMPTY or the stash tombstone (the zero word).
 *   - Slots and lanes are numbered from 0; "first set" is the lowest index.
 *   - Claim-then-commit (Algorithm 2) takes the lowest free slot; the "restore
 *     on failure" step never runs in a sequential model.
 *   - Step 2 tries the candidate bucket with more free slots first (ties go
 *     to the first hash), then the other: bucketed two-choice placement
 *     (Section V opening paragraph).
 *   - Cuckoo eviction starts at the first candidate; with no free slot it
 *     evicts the lowest occupied slot (Algorithm 3, "first occupied"), which
 *     with a full bucket is slot 0; the victim moves to its alternate bucket,
 *     the other candidate, or the same bucket when both candidates coincide.
 *   - After max_evictions rounds the item still in hand enters the stash
 *     ring; when the ring is full it joins the pending list.  Both are part
 *     of the table: lookup, replace and delete search them after the two
 *     candidate buckets.
 *   - FIXED addressing reduces the mixed hash modulo the bucket count, as the
 *     listing does; LINEAR addressing uses the index mask and split pointer
 *     (Section IV-C): a = H & im, and a = H & (2 im + 1) when a < sp.
 *   - A split keeps an entry in the source bucket when any of its candidate
 *     hashes still addresses the source under the next-round mask; otherwise
 *     it moves to the partner bucket.  After a split batch every stash and
 *     pending entry is re-inserted through steps 2-4.
 *   - A merge batch walks pairs from the top (split pointer - 1) downward,
 *     regressing the round first when the split pointer is 0, and stops at
 *     the first pair whose movers exceed the low bucket's free slots.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define O_EMPTY 0xFFFFFFFFFFFFFFFFull /* unoccupied bucket slot            */
#define O_TOMB 0x0ull                 /* deleted stash entry (key 0 word) */

static uint64_t pack(uint32_t key, uint32_t value) { return ((uint64_t)value << 32) | key; }
static uint32_t key_of(uint64_t w) { return (uint32_t)(w & 0xFFFFFFFFull); }
static uint32_t value_of(uint64_t w) { return (uint32_t)(w >> 32); }
static int valid_key(uint32_t k) { return k != 0u && k != 0xFFFFFFFFu; }

/* ======================================================================
 * O1: dictionary (Section III-D).  Separate chaining over a node pool.
 * ====================================================================== */
typedef struct {
  uint32_t key, value;
  int64_t next; /* index into pool, -1 terminates */
} o1_node;

typedef struct {
  int64_t *heads;
  uint64_t nheads;
  o1_node *pool;
  uint64_t pool_len, pool_cap;
  int64_t free_list;
  uint64_t size;
} o1_dict;

o1_dict *o1_create(uint64_t expected) {
  o1_dict *d = (o1_dict *)calloc(1, sizeof(o1_dict));
  if (!d) return NULL;
  d->nheads = expected < 64 ? 64 : expected;
  d->heads = (int64_t *)malloc(d->nheads * sizeof(int64_t));
  d->pool_cap = 64;
  d->pool = (o1_node *)malloc(d->pool_cap * sizeof(o1_node));
  if (!d->heads || !d->pool) return NULL;
  for (uint64_t i = 0; i < d->nheads; ++i) d->heads[i] = -1;
  d->free_list = -1;
  return d;
}

void o1_destroy(o1_dict *d) {
  if (!d) return;
  free(d->heads);
  free(d->pool);
  free(d);
}

static int64_t *o1_find(o1_dict *d, uint32_t key) {
  int64_t *link = &d->heads[key % d->nheads];
  while (*link >= 0 && d->pool[*link].key != key) link = &d->pool[*link].next;
  return link; /* points at the node's index, or at a -1 terminator */
}

static int o1_put(o1_dict *d, uint32_t key, uint32_t value) {
  int64_t *link = o1_find(d, key);
  if (*link >= 0) {
    d->pool[*link].value = value;
    return 0;
  }
  int64_t idx;
  if (d->free_list >= 0) {
    idx = d->free_list;
    d->free_list = d->pool[idx].next;
  } else {
    if (d->pool_len == d->pool_cap) {
      uint64_t cap = d->pool_cap * 2;
      o1_node *p = (o1_node *)realloc(d->pool, cap * sizeof(o1_node));
      if (!p) return -1;
      d->pool = p;
      d->pool_cap = cap;
      link = o1_find(d, key); /* pool moved; heads did not, but be plain */
    }
    idx = (int64_t)d->pool_len++;
  }
  d->pool[idx].key = key;
  d->pool[idx].value = value;
  d->pool[idx].next = -1;
  *link = idx;
  d->size++;
  return 0;
}

/* ops: 0 insert, 1 delete, 2 lookup.  Outputs (nullable):
 *   lookup: vals_out = value or 0xFFFFFFFF, flags_out = found
 *   delete: flags_out = was present; vals_out untouched
 *   insert: nothing
 * Reserved keys are no-ops (lookup: absent, delete: 0). Returns 0, or -1 on
 * allocation failure. */
int o1_apply(o1_dict *d, const uint8_t *ops, const uint32_t *keys, const uint32_t *vals, uint64_t n,
             uint32_t *vals_out, uint8_t *flags_out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t k = keys[i];
    int ok = valid_key(k);
    switch (ops[i]) {
      case 0:
        if (ok && o1_put(d, k, vals[i]) != 0) return -1;
        break;
      case 1: {
        uint8_t was = 0;
        if (ok) {
          int64_t *link = o1_find(d, k);
          if (*link >= 0) {
            int64_t idx = *link;
            *link = d->pool[idx].next;
            d->pool[idx].next = d->free_list;
            d->free_list = idx;
            d->size--;
            was = 1;
          }
        }
        if (flags_out) flags_out[i] = was;
        break;
      }
      case 2: {
        int64_t idx = ok ? *o1_find(d, k) : -1;
        if (vals_out) vals_out[i] = idx >= 0 ? d->pool[idx].value : 0xFFFFFFFFu;
        if (flags_out) flags_out[i] = idx >= 0;
        break;
      }
      default:
        return -2;
    }
  }
  return 0;
}

uint64_t o1_size(const o1_dict *d) { return d->size; }

/* all entries as packed words, in no particular order; returns the count */
uint64_t o1_dump(const o1_dict *d, uint64_t *words, uint64_t cap) {
  uint64_t n = 0;
  for (uint64_t h = 0; h < d->nheads; ++h)
    for (int64_t i = d->heads[h]; i >= 0; i = d->pool[i].next) {
      if (n < cap) words[n] = pack(d->pool[i].key, d->pool[i].value);
      ++n;
    }
  return n;
}

/* ======================================================================
 * O2: sequential Hive model.
 * ====================================================================== */

/* --- Section III-C: BitHash1 and BitHash2 -----------------------------
 * Each hash is a fixed chain of invertible 32-bit maps.  The chains below
 * restate the listing's steps as maps on Z/2^32:
 *   affine(a, b):      x -> a*x + b
 *   xorshr(s, c):      x -> x ^ (x >> s) ^ c
 *   addxorshl(c, s):   x -> (x + c) ^ (x << s)
 * BitHash1: x -> -x - 1 + 2^15 x (affine 2^15 - 1, -1); x ^= x >> 12;
 *           x -> 5x; x ^= x >> 4; x -> 2057x; x ^= x >> 16.
 * BitHash2: x -> 4097x + 0x7ed55d16; x -> x ^ (x >> 19) ^ 0xc761c23c;
 *           x -> 33x + 0x165667b1; x -> (x + 0xd3a2646c) ^ (x << 9);
 *           x -> 9x + 0xfd7046c5; x -> x ^ (x >> 16) ^ 0xb55a4f09.
 * The listing then reduces modulo the bucket count; that reduction is part
 * of the addressing below, so these return the full 32-bit mix. */
typedef enum { ST_AFFINE, ST_XORSHR, ST_ADDXORSHL } step_kind;
typedef struct {
  step_kind kind;
  uint32_t a; /* multiplier (affine) or shift */
  uint32_t c; /* additive or xor constant     */
} hash_step;

static const hash_step BITHASH1[] = {
    {ST_AFFINE, 32767u, 0xFFFFFFFFu}, /* (2^15 - 1) x - 1 */
    {ST_XORSHR, 12u, 0u},
    {ST_AFFINE, 5u, 0u},
    {ST_XORSHR, 4u, 0u},
    {ST_AFFINE, 2057u, 0u},
    {ST_XORSHR, 16u, 0u},
};
static const hash_step BITHASH2[] = {
    {ST_AFFINE, 4097u, 0x7ed55d16u}, /* x + c + (x << 12) */
    {ST_XORSHR, 19u, 0xc761c23cu},
    {ST_AFFINE, 33u, 0x165667b1u}, /* x + c + (x << 5) */
    {ST_ADDXORSHL, 9u, 0xd3a2646cu},
    {ST_AFFINE, 9u, 0xfd7046c5u}, /* x + c + (x << 3) */
    {ST_XORSHR, 16u, 0xb55a4f09u},
};

static uint32_t run_chain(const hash_step *st, int n, uint32_t x) {
  for (int i = 0; i < n; ++i) {
    switch (st[i].kind) {
      case ST_AFFINE: x = st[i].a * x + st[i].c; break;
      case ST_XORSHR: x = x ^ (x >> st[i].a) ^ st[i].c; break;
      case ST_ADDXORSHL: x = (x + st[i].c) ^ (x << st[i].a); break;
    }
  }
  return x;
}

uint32_t o2_bithash1(uint32_t key) { return run_chain(BITHASH1, 6, key); }
uint32_t o2_bithash2(uint32_t key) { return run_chain(BITHASH2, 6, key); }

enum { ADDR_FIXED = 0, ADDR_LINEAR = 1 };

typedef struct {
  /* configuration */
  uint32_t S;             /* slots per bucket, 1..64 */
  uint32_t E;             /* max_evictions */
  uint64_t stash_cap;     /* stash ring capacity (entries) */
  int addressing;         /* ADDR_FIXED or ADDR_LINEAR */
  uint64_t max_buckets;   /* bucket arena */
  uint64_t min_buckets;   /* merges never go below this */
  uint64_t K;             /* pairs per resize step */
  uint32_t lf_expand_pct, lf_contract_pct;
  /* geometry (Section III-B global metadata; Section IV-C control fields) */
  uint64_t n_buckets;
  uint64_t im, sp;
  /* storage */
  uint64_t *slots;     /* max_buckets * S packed words */
  uint64_t *free_mask; /* bit i set <=> slot i free (Section III-B) */
  uint64_t *stash;     /* ring of packed words (Section IV-A step 4) */
  uint64_t stash_head, stash_tail;
  uint64_t *pending;
  uint64_t pending_len, pending_cap;
  uint64_t live;
  /* counters */
  uint64_t evictions;       /* victim displacements */
  uint64_t stash_inserts;   /* items that entered the ring */
  uint64_t pending_inserts; /* items that went to pending */
  uint64_t full_chains;     /* inserts whose chain ran all E rounds */
  uint64_t invalid_keys;
  uint64_t kick_hist[65];   /* evictions per insert (capped at 64) */
} o2_table;

static uint64_t full_mask(uint32_t S) { return S >= 64 ? ~0ull : ((1ull << S) - 1); }

static uint64_t lowest_bit_index(uint64_t m) { return (uint64_t)__builtin_ctzll(m); }

static uint64_t o2_address(const o2_table *t, uint32_t h) {
  if (t->addressing == ADDR_FIXED) return h % t->n_buckets;
  uint64_t a = h & t->im;
  if (a < t->sp) a = h & (2 * t->im + 1);
  return a;
}

static void o2_candidates(const o2_table *t, uint32_t key, uint64_t *c1, uint64_t *c2) {
  *c1 = o2_address(t, o2_bithash1(key));
  *c2 = o2_address(t, o2_bithash2(key));
}

uint64_t o2_bucket_of(const o2_table *t, uint32_t mixed_hash) { return o2_address(t, mixed_hash); }

static uint64_t *slot_at(o2_table *t, uint64_t b, uint32_t s) { return &t->slots[b * t->S + s]; }

static void reset_geometry(o2_table *t, uint64_t n_buckets) {
  t->n_buckets = n_buckets;
  if (t->addressing == ADDR_LINEAR) {
    uint64_t p = 1;
    while (p * 2 <= n_buckets) p *= 2;
    t->im = p - 1;
    t->sp = n_buckets - p;
  } else {
    t->im = 0;
    t->sp = 0;
  }
}

o2_table *o2_create(uint32_t S, uint32_t E, uint64_t stash_cap, int addressing, uint64_t n_buckets,
                    uint64_t max_buckets, uint64_t K, uint32_t lf_expand_pct, uint32_t lf_contract_pct) {
  if (S < 1 || S > 64 || n_buckets < 1 || max_buckets < n_buckets) return NULL;
  if (addressing != ADDR_FIXED && addressing != ADDR_LINEAR) return NULL;
  if (addressing == ADDR_FIXED && n_buckets > 0xFFFFFFFFull) return NULL;
  o2_table *t = (o2_table *)calloc(1, sizeof(o2_table));
  if (!t) return NULL;
  t->S = S;
  t->E = E;
  t->stash_cap = stash_cap;
  t->addressing = addressing;
  t->max_buckets = addressing == ADDR_LINEAR ? max_buckets : n_buckets;
  t->min_buckets = n_buckets;
  t->K = K ? K : 1;
  t->lf_expand_pct = lf_expand_pct;
  t->lf_contract_pct = lf_contract_pct;
  reset_geometry(t, n_buckets);
  t->slots = (uint64_t *)malloc(t->max_buckets * S * sizeof(uint64_t));
  t->free_mask = (uint64_t *)malloc(t->max_buckets * sizeof(uint64_t));
  t->stash = (uint64_t *)malloc((stash_cap ? stash_cap : 1) * sizeof(uint64_t));
  t->pending_cap = 16;
  t->pending = (uint64_t *)malloc(t->pending_cap * sizeof(uint64_t));
  if (!t->slots || !t->free_mask || !t->stash || !t->pending) return NULL;
  for (uint64_t i = 0; i < t->max_buckets * S; ++i) t->slots[i] = O_EMPTY;
  for (uint64_t b = 0; b < t->max_buckets; ++b) t->free_mask[b] = full_mask(S);
  return t;
}

void o2_destroy(o2_table *t) {
  if (!t) return;
  free(t->slots);
  free(t->free_mask);
  free(t->stash);
  free(t->pending);
  free(t);
}

/* Location of a key: bucket slot, stash ring position, or pending index. */
typedef enum { LOC_NONE, LOC_BUCKET, LOC_STASH, LOC_PENDING } loc_kind;
typedef struct {
  loc_kind kind;
  uint64_t bucket; /* LOC_BUCKET */
  uint64_t index;  /* slot, ring position (absolute), or pending index */
} o2_loc;

/* Match-and-elect over one bucket (Section III-F; Algorithms 1 and 4): every
 * slot is compared with the key and the lowest matching slot is elected. */
static int64_t match_and_elect(o2_table *t, uint64_t b, uint32_t key) {
  uint64_t matches = 0;
  for (uint32_t s = 0; s < t->S; ++s)
    if (*slot_at(t, b, s) != O_EMPTY && key_of(*slot_at(t, b, s)) == key) matches |= 1ull << s;
  return matches ? (int64_t)lowest_bit_index(matches) : -1;
}

static o2_loc o2_locate(o2_table *t, uint32_t key) {
  o2_loc loc = {LOC_NONE, 0, 0};
  uint64_t c1, c2;
  o2_candidates(t, key, &c1, &c2);
  uint64_t cand[2] = {c1, c2};
  for (int j = 0; j < 2; ++j) {
    if (j == 1 && c2 == c1) break;
    int64_t s = match_and_elect(t, cand[j], key);
    if (s >= 0) {
      loc.kind = LOC_BUCKET;
      loc.bucket = cand[j];
      loc.index = (uint64_t)s;
      return loc;
    }
  }
  for (uint64_t p = t->stash_head; p < t->stash_tail; ++p) {
    uint64_t w = t->stash[p % t->stash_cap];
    if (w != O_TOMB && key_of(w) == key) {
      loc.kind = LOC_STASH;
      loc.index = p;
      return loc;
    }
  }
  for (uint64_t i = 0; i < t->pending_len; ++i)
    if (key_of(t->pending[i]) == key) {
      loc.kind = LOC_PENDING;
      loc.index = i;
      return loc;
    }
  return loc;
}

/* Algorithm 2, ClaimThenCommit: the lowest free slot of bucket b is claimed
 * (its free bit cleared) and the word published.  Returns the slot or -1. */
static int64_t claim_then_commit(o2_table *t, uint64_t b, uint64_t kv) {
  uint64_t mask = t->free_mask[b] & full_mask(t->S);
  if (mask == 0) return -1;
  uint64_t s = lowest_bit_index(mask);
  t->free_mask[b] &= ~(1ull << s);
  *slot_at(t, b, (uint32_t)s) = kv;
  return (int64_t)s;
}

static uint64_t popcount64(uint64_t x) { return (uint64_t)__builtin_popcountll(x); }

/* Section IV-A step 2: two-choice claim -- the candidate with more free
 * slots first (ties: first hash), then the other. */
static int step2_claim(o2_table *t, uint32_t key, uint64_t kv) {
  uint64_t c1, c2;
  o2_candidates(t, key, &c1, &c2);
  uint64_t f1 = popcount64(t->free_mask[c1] & full_mask(t->S));
  uint64_t f2 = popcount64(t->free_mask[c2] & full_mask(t->S));
  uint64_t first = (f2 > f1) ? c2 : c1, second = (f2 > f1) ? c1 : c2;
  if (claim_then_commit(t, first, kv) >= 0) return 1;
  if (second != first && claim_then_commit(t, second, kv) >= 0) return 1;
  return 0;
}

static uint64_t alt_bucket(o2_table *t, uint32_t key, uint64_t b) {
  uint64_t c1, c2;
  o2_candidates(t, key, &c1, &c2);
  return (b == c1) ? c2 : c1;
}

/* Algorithm 3, CuckooEvictAndInsert.  Returns 1 when everything is placed;
 * otherwise 0 with *in_hand set to the item still displaced. */
static int cuckoo_evict_and_insert(o2_table *t, uint64_t b0, uint64_t kv0, uint64_t *in_hand, uint32_t *kicks) {
  uint64_t kv = kv0, b = b0;
  *kicks = 0;
  for (uint32_t kick = 1; kick <= t->E; ++kick) {
    if (claim_then_commit(t, b, kv) >= 0) return 1;
    uint64_t fm = t->free_mask[b] & full_mask(t->S);
    if (fm != 0) { /* placed without eviction */
      uint64_t s = lowest_bit_index(fm);
      t->free_mask[b] = fm & ~(1ull << s);
      *slot_at(t, b, (uint32_t)s) = kv;
      return 1;
    }
    uint64_t occ = ~fm & full_mask(t->S);
    uint64_t s = lowest_bit_index(occ);
    uint64_t victim = *slot_at(t, b, (uint32_t)s);
    *slot_at(t, b, (uint32_t)s) = kv;
    t->evictions++;
    (*kicks)++;
    kv = victim;
    b = alt_bucket(t, key_of(kv), b);
  }
  *in_hand = kv;
  return 0;
}

static int pending_push(o2_table *t, uint64_t kv) {
  if (t->pending_len == t->pending_cap) {
    uint64_t cap = t->pending_cap * 2;
    uint64_t *p = (uint64_t *)realloc(t->pending, cap * sizeof(uint64_t));
    if (!p) return -1;
    t->pending = p;
    t->pending_cap = cap;
  }
  t->pending[t->pending_len++] = kv;
  t->pending_inserts++;
  return 0;
}

/* Section IV-A step 4: ring buffer with head and tail; when full, the item
 * is held as pending until the next resize. */
static int stash_or_pending(o2_table *t, uint64_t kv) {
  if (t->stash_tail - t->stash_head < t->stash_cap) {
    t->stash[t->stash_tail % t->stash_cap] = kv;
    t->stash_tail++;
    t->stash_inserts++;
    return 0;
  }
  return pending_push(t, kv);
}

/* Steps 2-4 for a word whose key is known to be absent. */
static int place_new(o2_table *t, uint64_t kv) {
  if (step2_claim(t, key_of(kv), kv)) {
    t->kick_hist[0]++;
    return 0;
  }
  uint64_t c1, c2, in_hand = 0;
  uint32_t kicks = 0;
  o2_candidates(t, key_of(kv), &c1, &c2);
  int placed = cuckoo_evict_and_insert(t, c1, kv, &in_hand, &kicks);
  t->kick_hist[kicks > 64 ? 64 : kicks]++;
  if (placed) return 0;
  t->full_chains++;
  return stash_or_pending(t, in_hand);
}

/* Section IV-A: the four-step insert. */
static int o2_insert(o2_table *t, uint32_t key, uint32_t value) {
  uint64_t kv = pack(key, value);
  o2_loc loc = o2_locate(t, key); /* step 1: replace */
  switch (loc.kind) {
    case LOC_BUCKET: *slot_at(t, loc.bucket, (uint32_t)loc.index) = kv; return 0;
    case LOC_STASH: t->stash[loc.index % t->stash_cap] = kv; return 0;
    case LOC_PENDING: t->pending[loc.index] = kv; return 0;
    case LOC_NONE: break;
  }
  t->live++;
  return place_new(t, kv); /* steps 2-4 */
}

/* Section IV-B, Algorithm 4 (and the stash/pending extension). */
static int o2_delete(o2_table *t, uint32_t key) {
  o2_loc loc = o2_locate(t, key);
  switch (loc.kind) {
    case LOC_BUCKET:
      *slot_at(t, loc.bucket, (uint32_t)loc.index) = O_EMPTY;
      t->free_mask[loc.bucket] |= 1ull << loc.index;
      break;
    case LOC_STASH: t->stash[loc.index % t->stash_cap] = O_TOMB; break;
    case LOC_PENDING: t->pending[loc.index] = t->pending[--t->pending_len]; break;
    case LOC_NONE: return 0;
  }
  t->live--;
  return 1;
}

static int o2_lookup(o2_table *t, uint32_t key, uint32_t *value) {
  o2_loc loc = o2_locate(t, key);
  uint64_t w;
  switch (loc.kind) {
    case LOC_BUCKET: w = *slot_at(t, loc.bucket, (uint32_t)loc.index); break;
    case LOC_STASH: w = t->stash[loc.index % t->stash_cap]; break;
    case LOC_PENDING: w = t->pending[loc.index]; break;
    default: *value = 0xFFFFFFFFu; return 0;
  }
  *value = value_of(w);
  return 1;
}

/* Same contract as o1_apply. */
int o2_apply(o2_table *t, const uint8_t *ops, const uint32_t *keys, const uint32_t *vals, uint64_t n,
             uint32_t *vals_out, uint8_t *flags_out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t k = keys[i];
    int ok = valid_key(k);
    if (!ok) t->invalid_keys++;
    switch (ops[i]) {
      case 0:
        if (ok && o2_insert(t, k, vals[i]) != 0) return -1;
        break;
      case 1: {
        int was = ok ? o2_delete(t, k) : 0;
        if (flags_out) flags_out[i] = (uint8_t)was;
        break;
      }
      case 2: {
        uint32_t v = 0xFFFFFFFFu;
        int found = ok ? o2_lookup(t, k, &v) : 0;
        if (vals_out) vals_out[i] = v;
        if (flags_out) flags_out[i] = (uint8_t)found;
        break;
      }
      default:
        return -2;
    }
  }
  return 0;
}

/* Re-insert every stash and pending entry through steps 2-4 (after a split
 * batch; Section III-B "Overflow Stash" and Section IV-A step 4). */
static int drain_overflow(o2_table *t) {
  uint64_t n = 0, cap = (t->stash_tail - t->stash_head) + t->pending_len;
  uint64_t *items = (uint64_t *)malloc((cap ? cap : 1) * sizeof(uint64_t));
  if (!items) return -1;
  for (uint64_t p = t->stash_head; p < t->stash_tail; ++p) {
    uint64_t w = t->stash[p % t->stash_cap];
    if (w != O_TOMB) items[n++] = w;
  }
  for (uint64_t i = 0; i < t->pending_len; ++i) items[n++] = t->pending[i];
  t->stash_head = t->stash_tail = 0;
  t->pending_len = 0;
  int rc = 0;
  for (uint64_t i = 0; i < n && rc == 0; ++i) rc = place_new(t, items[i]);
  free(items);
  return rc;
}

/* Section IV-C-1: split up to K pairs (sp, sp + 2^m); returns pairs split or
 * -1 on error.  Entries of the source bucket stay when a candidate hash of
 * theirs still addresses the source under the next-round mask; the rest are
 * compacted into slots 0..n-1 of the partner. */
int64_t o2_split(o2_table *t, uint64_t K) {
  if (t->addressing != ADDR_LINEAR) return -1;
  int64_t done = 0;
  for (uint64_t i = 0; i < K; ++i) {
    if (t->sp == t->im + 1) { /* every bucket of this round is split (a merge */
      t->im = 2 * t->im + 1;  /* regress leaves this form): start the next    */
      t->sp = 0;              /* round; addresses are the same in both forms  */
    }
    uint64_t src = t->sp, dst = t->sp + t->im + 1;
    if (dst >= t->max_buckets) break;
    uint64_t next_mask = 2 * t->im + 1;
    uint32_t n_move = 0;
    uint64_t move_mask = 0;
    for (uint32_t s = 0; s < t->S; ++s) {
      uint64_t w = *slot_at(t, src, s);
      if (w == O_EMPTY) continue;
      uint32_t h[2] = {o2_bithash1(key_of(w)), o2_bithash2(key_of(w))};
      int stay = 0;
      for (int j = 0; j < 2; ++j)
        if ((h[j] & t->im) == src && (h[j] & next_mask) == src) stay = 1;
      if (!stay) {
        *slot_at(t, dst, n_move) = w; /* compacted placement */
        *slot_at(t, src, s) = O_EMPTY;
        move_mask |= 1ull << s;
        n_move++;
      }
    }
    t->free_mask[src] |= move_mask;
    t->free_mask[dst] &= ~((n_move >= 64) ? ~0ull : ((1ull << n_move) - 1));
    t->sp++;
    t->n_buckets++;
    if (t->sp == t->im + 1) { /* round complete: double the address range */
      t->im = 2 * t->im + 1;
      t->sp = 0;
    }
    done++;
  }
  if (done > 0 && drain_overflow(t) != 0) return -1;
  return done;
}

static uint64_t nth_set_bit(uint64_t m, uint64_t r) {
  for (uint64_t i = 0; i < r; ++i) m &= m - 1;
  return lowest_bit_index(m);
}

/* Section IV-C-2: merge up to K pairs, top down; returns pairs merged. */
int64_t o2_merge(o2_table *t, uint64_t K) {
  if (t->addressing != ADDR_LINEAR) return -1;
  int64_t done = 0;
  for (uint64_t i = 0; i < K; ++i) {
    if (t->n_buckets <= t->min_buckets) break;
    if (t->sp == 0) { /* round regress; addresses are unchanged by it */
      if (t->im == 0) break;
      t->im >>= 1;
      t->sp = t->im + 1;
    }
    uint64_t lo = t->sp - 1, hi = lo + t->im + 1;
    uint64_t lo_free = t->free_mask[lo] & full_mask(t->S);
    uint64_t live_hi = 0;
    for (uint32_t s = 0; s < t->S; ++s)
      if (*slot_at(t, hi, s) != O_EMPTY) live_hi |= 1ull << s;
    if (popcount64(live_hi) > popcount64(lo_free)) break; /* abort */
    uint64_t used = 0, rank = 0;
    for (uint32_t s = 0; s < t->S; ++s) {
      if (!(live_hi >> s & 1)) continue;
      uint64_t pos = nth_set_bit(lo_free, rank++);
      *slot_at(t, lo, (uint32_t)pos) = *slot_at(t, hi, s);
      *slot_at(t, hi, s) = O_EMPTY;
      used |= 1ull << pos;
    }
    t->free_mask[hi] = full_mask(t->S);
    t->free_mask[lo] &= ~used;
    t->sp--;
    t->n_buckets--;
    done++;
  }
  return done;
}

/* Load-factor policy (Section IV-C): integer comparisons of live against
 * pct% of the slot capacity. */
static int over_expand(const o2_table *t, uint64_t extra) {
  return (t->live + extra) * 100 > (uint64_t)t->lf_expand_pct * t->n_buckets * t->S;
}

int64_t o2_policy_pre(o2_table *t, uint64_t n_ins) {
  if (t->addressing != ADDR_LINEAR) return 0;
  int64_t total = 0;
  while (over_expand(t, n_ins)) {
    int64_t s = o2_split(t, t->K);
    if (s <= 0) break;
    total += s;
  }
  return total;
}

int64_t o2_policy_post(o2_table *t) {
  if (t->addressing != ADDR_LINEAR) return 0;
  int64_t total = 0;
  while (over_expand(t, 0)) {
    int64_t s = o2_split(t, t->K);
    if (s <= 0) break;
    total += s;
  }
  while (t->live * 100 < (uint64_t)t->lf_contract_pct * t->n_buckets * t->S && t->n_buckets > t->min_buckets) {
    int64_t m = o2_merge(t, t->K);
    if (m <= 0) break;
    total -= m;
  }
  return total;
}

/* Counters and geometry: live, n_buckets, im, sp, stash entries (ring
 * occupancy including tombstones), pending, evictions, stash_inserts,
 * pending_inserts, full_chains, invalid_keys. */
void o2_stats(const o2_table *t, uint64_t *out) {
  out[0] = t->live;
  out[1] = t->n_buckets;
  out[2] = t->im;
  out[3] = t->sp;
  out[4] = t->stash_tail - t->stash_head;
  out[5] = t->pending_len;
  out[6] = t->evictions;
  out[7] = t->stash_inserts;
  out[8] = t->pending_inserts;
  out[9] = t->full_chains;
  out[10] = t->invalid_keys;
}

void o2_kick_hist(const o2_table *t, uint64_t *out65) { memcpy(out65, t->kick_hist, sizeof(t->kick_hist)); }

/* Every live word with its place: bucket index, -1 for the stash, -2 for
 * pending.  Returns the number of live words (writes at most cap). */
uint64_t o2_dump(const o2_table *t, uint64_t *words, int64_t *where, uint64_t cap) {
  uint64_t n = 0;
  for (uint64_t b = 0; b < t->n_buckets; ++b)
    for (uint32_t s = 0; s < t->S; ++s) {
      uint64_t w = t->slots[b * t->S + s];
      if (w == O_EMPTY) continue;
      if (n < cap) {
        words[n] = w;
        if (where) where[n] = (int64_t)b;
      }
      ++n;
    }
  for (uint64_t p = t->stash_head; p < t->stash_tail; ++p) {
    uint64_t w = t->stash[p % t->stash_cap];
    if (w == O_TOMB) continue;
    if (n < cap) {
      words[n] = w;
      if (where) where[n] = -1;
    }
    ++n;
  }
  for (uint64_t i = 0; i < t->pending_len; ++i) {
    if (n < cap) {
      words[n] = t->pending[i];
      if (where) where[n] = -2;
    }
    ++n;
  }
  return n;
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return (x > y) - (x < y);
}

/* Structural invariants; returns 0 when all hold, else writes a message.
 *   I1 every key once across buckets, stash and pending
 *   I3 every bucket entry sits in one of its two candidate buckets
 *   I4 free bit set exactly when the slot is EMPTY; buckets outside the
 *      table are all EMPTY
 *   I5 stash within capacity; pending only when the ring is full; items
 *      enter the ring only from chains that ran all E rounds
 *   I6 LINEAR: n_buckets == im + 1 + sp and 0 <= sp <= im + 1
 *   live equals the number of live words */
int o2_check(const o2_table *t, char *msg, int msglen) {
  o2_table *tt = (o2_table *)t;
  uint64_t total = 0;
  for (uint64_t b = 0; b < t->max_buckets; ++b) {
    uint64_t fm = t->free_mask[b];
    if (fm & ~full_mask(t->S)) {
      snprintf(msg, msglen, "I4: bucket %llu has free bits beyond S", (unsigned long long)b);
      return 4;
    }
    for (uint32_t s = 0; s < t->S; ++s) {
      uint64_t w = t->slots[b * t->S + s];
      int empty = (w == O_EMPTY);
      if (empty != (int)((fm >> s) & 1)) {
        snprintf(msg, msglen, "I4: bucket %llu slot %u free bit disagrees", (unsigned long long)b, s);
        return 4;
      }
      if (empty) continue;
      if (b >= t->n_buckets) {
        snprintf(msg, msglen, "I4: live entry beyond the table in bucket %llu", (unsigned long long)b);
        return 4;
      }
      uint64_t c1, c2;
      o2_candidates(t, key_of(w), &c1, &c2);
      if (b != c1 && b != c2) {
        snprintf(msg, msglen, "I3: key %u in bucket %llu, candidates %llu/%llu", key_of(w), (unsigned long long)b,
                 (unsigned long long)c1, (unsigned long long)c2);
        return 3;
      }
      if (!valid_key(key_of(w))) {
        snprintf(msg, msglen, "I1: reserved key stored");
        return 1;
      }
      total++;
    }
  }
  uint64_t ring = t->stash_tail - t->stash_head;
  if (ring > t->stash_cap) {
    snprintf(msg, msglen, "I5: stash over capacity");
    return 5;
  }
  if (t->pending_len > 0 && ring < t->stash_cap) {
    snprintf(msg, msglen, "I5: pending non-empty while the ring has room");
    return 5;
  }
  if (t->stash_inserts + t->pending_inserts > t->full_chains) {
    snprintf(msg, msglen, "I5: overflow entries exceed exhausted chains");
    return 5;
  }
  uint64_t n_dump = o2_dump(t, NULL, NULL, 0);
  uint32_t *keys = (uint32_t *)malloc((n_dump ? n_dump : 1) * sizeof(uint32_t));
  uint64_t *words = (uint64_t *)malloc((n_dump ? n_dump : 1) * sizeof(uint64_t));
  if (!keys || !words) {
    free(keys);
    free(words);
    snprintf(msg, msglen, "allocation failed");
    return 99;
  }
  o2_dump(t, words, NULL, n_dump);
  for (uint64_t i = 0; i < n_dump; ++i) keys[i] = key_of(words[i]);
  qsort(keys, n_dump, sizeof(uint32_t), cmp_u32);
  int rc = 0;
  for (uint64_t i = 1; i < n_dump && rc == 0; ++i)
    if (keys[i] == keys[i - 1]) {
      snprintf(msg, msglen, "I1: key %u appears twice", keys[i]);
      rc = 1;
    }
  free(keys);
  free(words);
  if (rc) return rc;
  if (n_dump != t->live) {
    snprintf(msg, msglen, "live %llu != %llu stored", (unsigned long long)t->live, (unsigned long long)n_dump);
    return 2;
  }
  (void)total;
  (void)tt;
  if (t->addressing == ADDR_LINEAR) {
    if (t->n_buckets != t->im + 1 + t->sp || t->sp > t->im + 1) {
      snprintf(msg, msglen, "I6: geometry n=%llu im=%llu sp=%llu", (unsigned long long)t->n_buckets,
               (unsigned long long)t->im, (unsigned long long)t->sp);
      return 6;
    }
  }
  return 0;
}
