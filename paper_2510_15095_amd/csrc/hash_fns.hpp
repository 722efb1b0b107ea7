// Hash functions for bucket addressing beyond BitHash1/2 (Section III-C
// compares them).  Every function reads a key as its four little-endian
// bytes:
//   CRC-32   reflected 0xEDB88320, all-ones initial value and final xor;
//   CRC-64   reflected 0xC96C5795D7870F42 (ECMA-182, as in xz), all-ones
//            initial value and final xor;
//   Murmur3  MurmurHash3, x86 32-bit variant, seed 0;
//   City32   CityHash32, its path for inputs of at most four bytes (bytes
//            folded in as signed chars, two mixing rounds, the finalizer).
// The CRCs here read their 256-entry tables from constant memory, the
// "lookup-based" form the paper evaluates; the tables are computed at
// compile time.
//
// A hash pair names the two candidate-bucket hashes of a table:
//   PAIR_BITHASH  BitHash1 and BitHash2 (the paper's choice, the default);
//   PAIR_CRC      CRC-32 and the low 32 bits of CRC-64;
//   PAIR_MURMUR   MurmurHash3 and CityHash32;
//   PAIR_TRIPLE   three candidates: BitHash1, BitHash2 and CityHash32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hive_device.hpp"

namespace hive {

enum : int { PAIR_BITHASH = 0, PAIR_CRC = 1, PAIR_MURMUR = 2, PAIR_TRIPLE = 3 };

struct CrcTables {
  uint32_t t32[256];
  uint64_t t64[256];
};

// Entry i: the CRC register after shifting in byte i alone.
constexpr CrcTables make_crc_tables() {
  CrcTables t{};
  for (uint32_t i = 0; i < 256; ++i) {
    uint32_t a = i;
    uint64_t b = i;
    for (int s = 0; s < 8; ++s) {
      a = (a >> 1) ^ ((a & 1u) ? 0xEDB88320u : 0u);
      b = (b >> 1) ^ ((b & 1u) ? 0xC96C5795D7870F42ull : 0ull);
    }
    t.t32[i] = a;
    t.t64[i] = b;
  }
  return t;
}

static __constant__ CrcTables kCrcTables = make_crc_tables();

__device__ __forceinline__ uint32_t crc32_key(uint32_t k) {
  uint32_t c = ~0u;
#pragma unroll
  for (int i = 0; i < 4; ++i) c = kCrcTables.t32[(c ^ (k >> (8 * i))) & 0xFFu] ^ (c >> 8);
  return ~c;
}

__device__ __forceinline__ uint64_t crc64_key(uint32_t k) {
  uint64_t c = ~0ull;
#pragma unroll
  for (int i = 0; i < 4; ++i) c = kCrcTables.t64[(c ^ (k >> (8 * i))) & 0xFFu] ^ (c >> 8);
  return ~c;
}

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }
__device__ __forceinline__ uint32_t rotr32(uint32_t x, int r) { return (x >> r) | (x << (32 - r)); }

// the 32-bit finalizer of MurmurHash3, also used by CityHash32
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  return h ^ (h >> 16);
}

__device__ __forceinline__ uint32_t murmur3_key(uint32_t k) {
  // one whole 4-byte block, no tail, length 4, seed 0
  k *= 0xCC9E2D51u;
  k = rotl32(k, 15) * 0x1B873593u;
  const uint32_t h = rotl32(k, 13) * 5u + 0xE6546B64u;
  return fmix32(h ^ 4u);
}

__device__ __forceinline__ uint32_t city_mur(uint32_t a, uint32_t h) {
  a *= 0xCC9E2D51u;
  a = rotr32(a, 17) * 0x1B873593u;
  h = rotr32(h ^ a, 19);
  return h * 5u + 0xE6546B64u;
}

__device__ __forceinline__ uint32_t city32_key(uint32_t k) {
  uint32_t b = 0, c = 9;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int32_t v = (int8_t)(k >> (8 * i));
    b = b * 0xCC9E2D51u + (uint32_t)v;
    c ^= b;
  }
  return fmix32(city_mur(b, city_mur(4u, c)));
}

template <int PAIR>
struct HashPair;

template <>
struct HashPair<PAIR_BITHASH> {
  __device__ static __forceinline__ uint32_t h1(uint32_t k) { return bithash1(k); }
  __device__ static __forceinline__ uint32_t h2(uint32_t k) { return bithash2(k); }
};

template <>
struct HashPair<PAIR_CRC> {
  __device__ static __forceinline__ uint32_t h1(uint32_t k) { return crc32_key(k); }
  __device__ static __forceinline__ uint32_t h2(uint32_t k) { return (uint32_t)crc64_key(k); }
};

template <>
struct HashPair<PAIR_MURMUR> {
  __device__ static __forceinline__ uint32_t h1(uint32_t k) { return murmur3_key(k); }
  __device__ static __forceinline__ uint32_t h2(uint32_t k) { return city32_key(k); }
};

// Three candidate buckets: BitHash1, BitHash2 and CityHash32 (the paper's
// third-hash configuration in its hash-function comparison, Section V-B).
template <>
struct HashPair<PAIR_TRIPLE> {
  __device__ static __forceinline__ uint32_t h1(uint32_t k) { return bithash1(k); }
  __device__ static __forceinline__ uint32_t h2(uint32_t k) { return bithash2(k); }
  __device__ static __forceinline__ uint32_t h3(uint32_t k) { return city32_key(k); }
};

// Candidate buckets per key under a hash choice.
template <int PAIR>
struct PairArity {
  static constexpr int D = PAIR == PAIR_TRIPLE ? 3 : 2;
};

}  // namespace hive
