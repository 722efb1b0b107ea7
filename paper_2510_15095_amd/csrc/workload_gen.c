/* Seeded synthetic workload generator: the fast path of workload.py.
 *
 * Holds none of the hash table's arithmetic.  It maps generator indices to
 * keys through a 4-round Feistel permutation of the 32-bit integers (skipping
 * the two indices whose image is a reserved key), derives values with
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), and generates whole mixed
 * batches (op codes, Zipf or uniform keys with per-type key disjointness).
 * Built with gcc, loaded through ctypes. */
#include <math.h>
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

/* Entry of the per-batch set of ranks taken by each op type (mixed batches
 * below). */
typedef struct {
  int64_t rank;
  int8_t owner; /* -1 = empty */
} slot_t;

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

/* ---------------------------------------------------------------------------
 * Mixed batches, generated whole in C (many at once, one thread per batch).
 *
 * A batch's random numbers come from one SplitMix64 stream seeded with its
 * batch seed (state += golden ratio, output = the SplitMix64 mix of the
 * state).  In stream order:
 *   1. op codes: n_ins inserts, n_del deletes, the rest lookups, then a
 *      Fisher-Yates shuffle (i = n-1 down to 1 swaps i with a draw below
 *      i+1; a draw below m is the high 64 bits of output x m);
 *   2. one rank per op: Zipf(s) over 1..N by rejection-inversion (Hoermann
 *      and Derflinger 1996) from uniforms (output >> 11) x 2^-53, or, for
 *      s <= 0, 1 + a draw below N;
 *   3. per-type disjointness, ops in index order: an op keeps its rank unless
 *      the rank is owned by another op type or is a delete rank already used,
 *      and then takes further ranks from the stream until one fits (the first
 *      op to take a rank owns it for its type);
 *   4. key = the key stream's key of index rank - 1; value =
 *      lo32(splitmix64(key)) xor salt.
 * ------------------------------------------------------------------------ */

static const uint64_t SM_GOLDEN = 0x9E3779B97F4A7C15ull;

typedef struct {
  uint64_t s;
} sm64_t;

static inline uint64_t sm_next(sm64_t *g) {
  g->s += SM_GOLDEN;
  uint64_t z = g->s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline double sm_u01(sm64_t *g) { return (double)(sm_next(g) >> 11) * 0x1.0p-53; }

static inline uint64_t sm_below(sm64_t *g, uint64_t m) {
  return (uint64_t)(((unsigned __int128)sm_next(g) * m) >> 64);
}

typedef struct {
  int64_t n;
  double s, q, lo, hi;
} zipf_t;

static inline double zipf_H(const zipf_t *z, double x) { return expm1(z->q * log(x)) / z->q; }
static inline double zipf_Hinv(const zipf_t *z, double y) { return exp(log1p(z->q * y) / z->q); }

static void zipf_init(zipf_t *z, int64_t n, double s) {
  z->n = n;
  z->s = s;
  z->q = 1.0 - s;
  z->lo = zipf_H(z, 1.5) - 1.0;
  z->hi = zipf_H(z, (double)n + 0.5);
}

static inline int64_t draw_rank(const zipf_t *z, int64_t universe, sm64_t *g) {
  if (!z) return 1 + (int64_t)sm_below(g, (uint64_t)universe);
  for (;;) {
    const double u = z->lo + sm_u01(g) * (z->hi - z->lo);
    double k = floor(zipf_Hinv(z, u) + 0.5);
    if (k < 1.0) k = 1.0;
    if (k > (double)z->n) k = (double)z->n;
    if (u >= zipf_H(z, k + 0.5) - pow(k, -z->s)) return (int64_t)k;
  }
}

/* One batch; returns 0, -1 when the universe cannot supply disjoint ranks,
 * -2 when out of memory. */
static int mixed_one(uint64_t seed, int64_t n, int64_t n_ins, int64_t n_del, int64_t universe, double zipf_s,
                     const uint32_t *rk, int64_t a, int64_t b, uint32_t salt, uint8_t *ops, uint32_t *keys,
                     uint32_t *vals, int64_t *ranks) {
  sm64_t g = {seed};
  zipf_t zz;
  const zipf_t *z = NULL;
  if (zipf_s > 0.0) {
    zipf_init(&zz, universe, zipf_s);
    z = &zz;
  }
  for (int64_t i = 0; i < n; ++i) ops[i] = i < n_ins ? 0 : (i < n_ins + n_del ? 1 : 2);
  for (int64_t i = n - 1; i >= 1; --i) {
    const int64_t j = (int64_t)sm_below(&g, (uint64_t)i + 1);
    const uint8_t t = ops[i];
    ops[i] = ops[j];
    ops[j] = t;
  }
  for (int64_t i = 0; i < n; ++i) ranks[i] = draw_rank(z, universe, &g);
  uint64_t cap = 16;
  while (cap < (uint64_t)n * 2) cap <<= 1;
  slot_t *set = (slot_t *)malloc(cap * sizeof(slot_t));
  if (!set) return -2;
  for (uint64_t s = 0; s < cap; ++s) set[s].owner = -1;
  int64_t redraws = 0;
  const int64_t max_redraws = 64 * (n > 1024 ? n : 1024);
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
      if (set[s].owner == (int8_t)ops[i] && ops[i] != 1) break;
      if (++redraws > max_redraws) {
        free(set);
        return -1;
      }
      r = draw_rank(z, universe, &g);
    }
    ranks[i] = r;
  }
  free(set);
  for (int64_t i = 0; i < n; ++i) {
    keys[i] = key_of(rk, a, b, ranks[i] - 1);
    vals[i] = (uint32_t)splitmix64_first(keys[i]) ^ salt;
  }
  return 0;
}

/* `count` batches; batch c writes n[c] entries at offset off[c] of the
 * output arrays.  rk: 4 round keys per batch; ab: the key stream's two
 * skipped indices per batch.  Returns 0, or the first failing status. */
int wl_mixed_many(int64_t count, const uint64_t *seed, const int64_t *n, const int64_t *off, const int64_t *n_ins,
                  const int64_t *n_del, const int64_t *universe, const double *zipf_s, const uint32_t *rk,
                  const int64_t *ab, const uint32_t *salt, uint8_t *ops, uint32_t *keys, uint32_t *vals,
                  int64_t *ranks) {
  int status = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < count; ++c) {
    const int r = mixed_one(seed[c], n[c], n_ins[c], n_del[c], universe[c], zipf_s[c], rk + 4 * c, ab[2 * c],
                            ab[2 * c + 1], salt[c], ops + off[c], keys + off[c], vals + off[c], ranks + off[c]);
    if (r != 0) {
#pragma omp critical
      if (status == 0) status = r;
    }
  }
  return status;
}
