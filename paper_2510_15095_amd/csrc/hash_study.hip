// Hash-function study on MI355X (gfx950): bucket spread of BitHash1/2 and of
// widely used hashes (Section III-C), measured as the collision count
// Y = sum over buckets of (load - 1)+ that the uniform-hashing theorem there
// gives an expectation for.
//
// Every hash reads a key as its four little-endian bytes.  The CRCs are
// table-driven, the form the paper evaluates as "lookup-based": each block
// builds the two 256-entry tables in LDS, one entry per thread, and a key
// then costs four table reads per CRC.  The others are pure ALU (shared
// with the table's hash pairs):
//   CRC-32   reflected 0xEDB88320, all-ones initial value and final xor;
//   CRC-64   reflected 0xC96C5795D7870F42 (ECMA-182, as in xz), all-ones
//            initial value and final xor; the bucket reduces all 64 bits;
//   Murmur3  MurmurHash3 x86 32-bit, seed 0;
//   City32   CityHash32 for inputs of at most four bytes (bytes folded in
//            as signed chars, two mixing rounds, the 32-bit finalizer).
// A key's bucket is its hash modulo m (a mask when m is a power of two).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hash_fns.hpp"
#include "hive.h"
#include "hive_device.hpp"

namespace hive_hs {

using hive::city32_key;
using hive::murmur3_key;

constexpr int BLOCK = 256;

struct Tables {
  uint32_t crc32[256];
  uint64_t crc64[256];
};

// Entry t of each table: the CRC register after shifting in byte t alone.
__device__ __forceinline__ void build_tables(Tables &t) {
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    uint32_t a = (uint32_t)i;
    uint64_t b = (uint64_t)i;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      a = (a >> 1) ^ ((a & 1u) ? 0xEDB88320u : 0u);
      b = (b >> 1) ^ ((b & 1u) ? 0xC96C5795D7870F42ull : 0ull);
    }
    t.crc32[i] = a;
    t.crc64[i] = b;
  }
}

__device__ __forceinline__ uint64_t hash_key(uint32_t kind, uint32_t k, const Tables &t) {
  switch (kind) {
    case HIVE_HASH_BITHASH1: return hive::bithash1(k);
    case HIVE_HASH_BITHASH2: return hive::bithash2(k);
    case HIVE_HASH_CRC32: {
      uint32_t c = ~0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) c = t.crc32[(c ^ (k >> (8 * i))) & 0xFFu] ^ (c >> 8);
      return ~c;
    }
    case HIVE_HASH_CRC64: {
      uint64_t c = ~0ull;
#pragma unroll
      for (int i = 0; i < 4; ++i) c = t.crc64[(c ^ (k >> (8 * i))) & 0xFFu] ^ (c >> 8);
      return ~c;
    }
    case HIVE_HASH_MURMUR3: return murmur3_key(k);
    default: return city32_key(k);
  }
}

__device__ __forceinline__ uint32_t bucket_of(uint32_t kind, uint32_t k, const Tables &t, uint64_t m, bool pow2) {
  const uint64_t h = hash_key(kind, k, t);
  return (uint32_t)(pow2 ? (h & (m - 1)) : (h % m));
}

// out (optional): each key's bucket; bitmap (optional): bit b set for every
// bucket b that receives a key.  With 16-byte aligned arrays a lane moves
// four keys and four buckets per access (a 4-byte access per lane leaves
// half of the memory bandwidth unused).
__global__ __launch_bounds__(BLOCK) void bucket_kernel(uint32_t kind, const uint32_t *keys, uint64_t n, uint64_t m,
                                                        uint32_t *out, uint32_t *bitmap) {
  __shared__ Tables t;
  build_tables(t);
  __syncthreads();
  const bool pow2 = (m & (m - 1)) == 0;
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  const uint64_t tid = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool wide = (((uintptr_t)keys | (uintptr_t)out) & 15) == 0;
  const uint64_t n4 = wide ? n / 4 : 0;
  for (uint64_t q = tid; q < n4; q += stride) {
    const uint4 k = ((const uint4 *)keys)[q];
    const uint4 b = make_uint4(bucket_of(kind, k.x, t, m, pow2), bucket_of(kind, k.y, t, m, pow2),
                               bucket_of(kind, k.z, t, m, pow2), bucket_of(kind, k.w, t, m, pow2));
    if (out) ((uint4 *)out)[q] = b;
    if (bitmap) {
      atomicOr(&bitmap[b.x >> 5], 1u << (b.x & 31));
      atomicOr(&bitmap[b.y >> 5], 1u << (b.y & 31));
      atomicOr(&bitmap[b.z >> 5], 1u << (b.z & 31));
      atomicOr(&bitmap[b.w >> 5], 1u << (b.w & 31));
    }
  }
  for (uint64_t i = 4 * n4 + tid; i < n; i += stride) {
    const uint32_t b = bucket_of(kind, keys[i], t, m, pow2);
    if (out) out[i] = b;
    if (bitmap) atomicOr(&bitmap[b >> 5], 1u << (b & 31));
  }
}

// counter[0] += the number of set bits of bitmap[0, words).
__global__ __launch_bounds__(BLOCK) void popcount_kernel(const uint32_t *bitmap, uint64_t words,
                                                          unsigned long long *counter) {
  __shared__ unsigned long long part[BLOCK / 64];
  unsigned long long c = 0;
  for (uint64_t w = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; w < words; w += (uint64_t)gridDim.x * BLOCK)
    c += __popc(bitmap[w]);
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int i = 0; i < BLOCK / 64; ++i) s += part[i];
    if (s) atomicAdd(counter, s);
  }
}

unsigned grid_for(uint64_t items) {
  const uint64_t blocks = (items + BLOCK - 1) / BLOCK;
  return (unsigned)(blocks < 4096 ? (blocks ? blocks : 1) : 4096);
}

}  // namespace hive_hs

using namespace hive_hs;

extern "C" {

hive_status hive_hash_buckets(uint32_t kind, const uint32_t *d_keys, uint64_t n, uint64_t m, uint32_t *d_out,
                              void *stream) {
  if (kind >= HIVE_HASH_KINDS || m == 0 || m > (1ull << 32) || (n && (!d_keys || !d_out))) return HIVE_ERR_ARG;
  if (n == 0) return HIVE_OK;
  hipLaunchKernelGGL(bucket_kernel, dim3(grid_for((n + 3) / 4)), dim3(BLOCK), 0, (hipStream_t)stream, kind, d_keys, n,
                     m, d_out, (uint32_t *)nullptr);
  return hipGetLastError() == hipSuccess ? HIVE_OK : HIVE_ERR_HIP;
}

hive_status hive_hash_collisions(uint32_t kind, const uint32_t *d_keys, uint64_t n, uint64_t m, uint32_t *d_scratch,
                                 uint64_t *y_out, void *stream) {
  if (kind >= HIVE_HASH_KINDS || m == 0 || m > (1ull << 32) || !d_scratch || !y_out || (n && !d_keys))
    return HIVE_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const uint64_t words = (m + 31) / 32;
  unsigned long long *counter = (unsigned long long *)d_scratch;  // words 0 and 1
  uint32_t *bitmap = d_scratch + 2;
  if (hipMemsetAsync(d_scratch, 0, (words + 2) * 4, st) != hipSuccess) return HIVE_ERR_HIP;
  if (n) {
    hipLaunchKernelGGL(bucket_kernel, dim3(grid_for((n + 3) / 4)), dim3(BLOCK), 0, st, kind, d_keys, n, m,
                       (uint32_t *)nullptr, bitmap);
    hipLaunchKernelGGL(popcount_kernel, dim3(grid_for(words)), dim3(BLOCK), 0, st, bitmap, words, counter);
  }
  unsigned long long occupied = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&occupied, counter, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return HIVE_ERR_HIP;
  *y_out = n - occupied;
  return HIVE_OK;
}

}  // extern "C"
