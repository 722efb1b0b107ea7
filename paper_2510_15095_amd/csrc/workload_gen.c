/* Seeded synthetic workload generator: the fast path of workload.py.
 *
 * Holds none of the hash table's arithmetic.  It maps generator indices to
 * keys through a 4-round Feistel permutation of the 32-bit integers (skipping
 * the two indices whose image is a reserved key), derives values with
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), and resolves per-type key
 * disjointness for mixed batches.  Built with gcc, loaded through ctypes. */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint32_t feistel_f(uint32_t half, uint32_t rk) {
  uint32_t x = half * 0x9E3779B1u + rk;
  x ^= x >> 15;
  x *= 0x2C1B3C6Du;
  x ^= x >> 12;
  return x & 0xFFFFu;
}

static inline uint32_t perm(const uint32_t *rk, uint32_t x) {
  uint32_t l = x >> 16, r = x & 0xFFFFu;
  for (int i = 0; i < 4; ++i) {
    uint32_t t = l ^ feistel_f(r, rk[i]);
    l = r;
    r = t;
  }
  return (l << 16) | r;
}

static inline uint32_t perm_inv(const uint32_t *rk, uint32_t y) {
  uint32_t l = y >> 16, r = y & 0xFFFFu;
  for (int i = 3; i >= 0; --i) {
    uint32_t t = r ^ feistel_f(l, rk[i]);
    r = l;
    l = t;
  }
  return (l << 16) | r;
}

static inline uint32_t key_of(const uint32_t *rk, int64_t a, int64_t b, int64_t i) {
  int64_t j = i + (i >= a) + (i >= b - 1);
  return perm(rk, (uint32_t)j);
}

void wl_keys(const uint32_t *rk, int64_t a, int64_t b, const int64_t *idx, int64_t n, uint32_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < n; ++t) out[t] = key_of(rk, a, b, idx[t]);
}

void wl_keys_range(const uint32_t *rk, int64_t a, int64_t b, int64_t start, int64_t n, uint32_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < n; ++t) out[t] = key_of(rk, a, b, start + t);
}

/* index of each key; -1 for a reserved key */
void wl_index_of(const uint32_t *rk, int64_t a, int64_t b, const uint32_t *keys, int64_t n, int64_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < n; ++t) {
    int64_t j = (int64_t)perm_inv(rk, keys[t]);
    out[t] = (j == a || j == b) ? -1 : j - (j > a) - (j > b);
  }
}

static inline uint64_t splitmix64_first(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void wl_values(const uint32_t *keys, int64_t n, uint32_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < n; ++t) out[t] = (uint32_t)splitmix64_first(keys[t]);
}

/* Per-type key disjointness for one mixed batch.
 *
 * Ops are visited in index order.  Op i takes ranks[i]; while that rank is
 * owned by another op type, or is a delete rank already used in this batch,
 * op i takes the next rank from `pool` instead.  The first op to take a rank
 * owns it for its type.  Returns the number of pool entries consumed, or -1
 * when the pool ran dry (the caller retries with a larger pool). */
typedef struct {
  int64_t rank;
  int8_t owner; /* -1 = empty */
} slot_t;

int64_t wl_resolve_mixed(const uint8_t *ops, int64_t n, int64_t *ranks, const int64_t *pool, int64_t pool_n) {
  uint64_t cap = 16;
  while (cap < (uint64_t)n * 2) cap <<= 1;
  slot_t *set = (slot_t *)malloc(cap * sizeof(slot_t));
  if (!set) return -2;
  for (uint64_t s = 0; s < cap; ++s) set[s].owner = -1;
  int64_t used = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t r = ranks[i];
    for (;;) {
      uint64_t s = splitmix64_first((uint64_t)r) & (cap - 1);
      while (set[s].owner >= 0 && set[s].rank != r) s = (s + 1) & (cap - 1);
      if (set[s].owner < 0) {
        set[s].rank = r;
        set[s].owner = (int8_t)ops[i];
        break;
      }
      if (set[s].owner == (int8_t)ops[i] && ops[i] != 1 /* delete */) break;
      if (used >= pool_n) {
        free(set);
        return -1;
      }
      r = pool[used++];
    }
    ranks[i] = r;
  }
  free(set);
  return used;
}

/* Seeded permutation of [0, n) for sampling without replacement and for
 * shuffles: a 4-round balanced Feistel network on the smallest even bit width
 * 2h with 2^(2h) >= n, restricted to [0, n) by cycle walking (apply the
 * permutation again until the value falls inside the domain).  Cycle walking
 * of a permutation is a permutation of the sub-domain. */
static inline uint64_t dom_f(uint64_t half, uint32_t rk, uint64_t mask) {
  uint64_t x = (half * 0x9E3779B97F4A7C15ull) ^ rk;
  x ^= x >> 29;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 32;
  return x & mask;
}

static inline uint64_t dom_perm(const uint32_t *rk, uint64_t x, int hb) {
  uint64_t mask = (hb == 64) ? ~0ull : ((1ull << hb) - 1);
  uint64_t l = x >> hb, r = x & mask;
  for (int i = 0; i < 4; ++i) {
    uint64_t t = l ^ dom_f(r, rk[i], mask);
    l = r;
    r = t;
  }
  return (l << hb) | r;
}

int wl_domain_perm(const uint32_t *rk, int64_t n, const int64_t *pos, int64_t m, int64_t *out) {
  if (n <= 0 || n > (1ll << 40)) return -1;
  int hb = 1;
  while ((1ll << (2 * hb)) < n) ++hb;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t t = 0; t < m; ++t) {
    uint64_t x = (uint64_t)pos[t];
    if (pos[t] < 0 || pos[t] >= n) {
      bad |= 1;
      continue;
    }
    do x = dom_perm(rk, x, hb);
    while (x >= (uint64_t)n);
    out[t] = (int64_t)x;
  }
  return bad ? -1 : 0;
}
