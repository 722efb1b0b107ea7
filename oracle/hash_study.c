/* CPU oracle for the hash-function study -- TEST INFRASTRUCTURE.
 *
 * Only the tests and the benchmark may call this; the library never does.
 *
 * Section III-C compares the bucket spread of BitHash1/2 with widely used
 * non-cryptographic hashes (CRC-32, CRC-64, MurmurHash, CityHash) through the
 * collision count Y = sum over buckets of (load - 1)+ against its expectation
 * under uniform hashing (the theorem there).  This file holds plain, slow
 * transcriptions of those hashes from their public definitions, applied to a
 * key's four little-endian bytes; a key's bucket is its hash modulo m.
 *
 *   CRC-32    reflected, polynomial 0xEDB88320, initial value and final xor
 *             all ones (the IEEE 802.3 / zlib CRC), bit by bit, no table.
 *   CRC-64    reflected, polynomial 0xC96C5795D7870F42, initial value and
 *             final xor all ones (the CRC-64 of xz, ECMA-182 polynomial),
 *             bit by bit; the bucket takes the whole 64-bit value modulo m.
 *   Murmur3   MurmurHash3, 32-bit x86 variant (Appleby, public domain),
 *             seed 0 (the paper gives none).
 *   City32    CityHash32 (Pike and Alakuijala), its path for inputs of at
 *             most four bytes: bytes folded in as signed chars, then two
 *             Murmur-style mixing rounds and the 32-bit finalizer.
 *             Parity unpinned: no published outputs are at hand, so only the
 *             device transcription is compared with this one.
 *
 * Keys of the study are 32-bit integers, so the block loops below only ever
 * see whole 4-byte blocks; the byte-string entry points exist for the
 * published check values. */
#include <stddef.h>
#include <stdint.h>

enum { HS_BITHASH1 = 0, HS_BITHASH2 = 1, HS_CRC32 = 2, HS_CRC64 = 3, HS_MURMUR3 = 4, HS_CITY32 = 5 };

uint32_t o2_bithash1(uint32_t key);
uint32_t o2_bithash2(uint32_t key);

uint32_t hs_crc32(const uint8_t *p, size_t len) {
  uint32_t crc = 0xFFFFFFFFu;
  for (size_t i = 0; i < len; ++i) {
    crc ^= p[i];
    for (int b = 0; b < 8; ++b) crc = (crc & 1u) ? (crc >> 1) ^ 0xEDB88320u : crc >> 1;
  }
  return crc ^ 0xFFFFFFFFu;
}

uint64_t hs_crc64(const uint8_t *p, size_t len) {
  uint64_t crc = ~0ull;
  for (size_t i = 0; i < len; ++i) {
    crc ^= p[i];
    for (int b = 0; b < 8; ++b) crc = (crc & 1u) ? (crc >> 1) ^ 0xC96C5795D7870F42ull : crc >> 1;
  }
  return ~crc;
}

static uint32_t rotl(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }
static uint32_t rotr(uint32_t x, int r) { return (x >> r) | (x << (32 - r)); }

/* the 32-bit finalizer shared by MurmurHash3 and CityHash32 */
static uint32_t final_mix(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

uint32_t hs_murmur3(const uint8_t *p, size_t len, uint32_t seed) {
  const uint32_t m1 = 0xCC9E2D51u, m2 = 0x1B873593u;
  uint32_t h = seed;
  size_t i = 0;
  for (; i + 4 <= len; i += 4) {
    uint32_t k = (uint32_t)p[i] | (uint32_t)p[i + 1] << 8 | (uint32_t)p[i + 2] << 16 | (uint32_t)p[i + 3] << 24;
    k = rotl(k * m1, 15) * m2;
    h = rotl(h ^ k, 13) * 5u + 0xE6546B64u;
  }
  uint32_t k = 0;
  for (size_t t = len - i; t > 0; --t) k ^= (uint32_t)p[i + t - 1] << (8 * (t - 1));
  if (len - i) h ^= rotl(k * m1, 15) * m2;
  return final_mix(h ^ (uint32_t)len);
}

/* one Murmur-style round of CityHash32: mix a into h */
static uint32_t city_round(uint32_t a, uint32_t h) {
  a = rotr(a * 0xCC9E2D51u, 17) * 0x1B873593u;
  return rotr(h ^ a, 19) * 5u + 0xE6546B64u;
}

uint32_t hs_city32_short(const uint8_t *p, size_t len) {
  uint32_t b = 0, c = 9;
  for (size_t i = 0; i < len && i < 4; ++i) {
    b = b * 0xCC9E2D51u + (uint32_t)(int32_t)(int8_t)p[i];
    c ^= b;
  }
  return final_mix(city_round(b, city_round((uint32_t)len, c)));
}

static uint64_t hash_of(int kind, uint32_t key) {
  const uint8_t bytes[4] = {(uint8_t)key, (uint8_t)(key >> 8), (uint8_t)(key >> 16), (uint8_t)(key >> 24)};
  switch (kind) {
    case HS_BITHASH1: return o2_bithash1(key);
    case HS_BITHASH2: return o2_bithash2(key);
    case HS_CRC32: return hs_crc32(bytes, 4);
    case HS_CRC64: return hs_crc64(bytes, 4);
    case HS_MURMUR3: return hs_murmur3(bytes, 4, 0);
    default: return hs_city32_short(bytes, 4);
  }
}

/* out[i] = hash(kind, keys[i]) mod m.  Returns -1 for an unknown kind or m = 0. */
int hs_buckets(int kind, const uint32_t *keys, uint64_t n, uint64_t m, uint32_t *out) {
  if (kind < HS_BITHASH1 || kind > HS_CITY32 || m == 0) return -1;
  for (uint64_t i = 0; i < n; ++i) out[i] = (uint32_t)(hash_of(kind, keys[i]) % m);
  return 0;
}
