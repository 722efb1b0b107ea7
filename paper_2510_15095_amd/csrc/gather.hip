// Random 128-byte line gathers: the memory ceiling of bucket probing.
//
// A probe reads whole 16-slot buckets, one 128-byte line each, at random
// addresses, so the rate HBM sustains for such reads bounds every probe
// launch more tightly than its streaming bandwidth.  This kernel issues
// exactly that access pattern with the probe kernel's shape (a 16-lane
// group per line, 16 line loads of a wave in flight before any is used)
// and nothing else: out[i] = XOR of the 16 words of line idx[i], so every
// load is consumed.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hive.h"

namespace hive_gather {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;

// x rotated right by N lanes within each row of 16 lanes (a DPP move: a
// vector ALU operation, no LDS traffic).
template <int N>
__device__ __forceinline__ uint32_t row_ror(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x120 + N, 0xF, 0xF, false);
}

// XOR of the 16 words of a 16-lane group, in every lane of the group.
__device__ __forceinline__ uint64_t row_xor(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo ^= row_ror<8>(lo);
  hi ^= row_ror<8>(hi);
  lo ^= row_ror<4>(lo);
  hi ^= row_ror<4>(hi);
  lo ^= row_ror<2>(lo);
  hi ^= row_ror<2>(hi);
  lo ^= row_ror<1>(lo);
  hi ^= row_ror<1>(hi);
  return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(BLOCK) void gather_kernel(const uint64_t *table, uint64_t n_lines, const uint32_t *idx,
                                                        uint64_t n, uint64_t *out) {
  const int lane = threadIdx.x & 63, g = lane >> 4, sl = lane & 15;
  const uint64_t wave = (uint64_t)blockIdx.x * WAVES + (threadIdx.x >> 6);
  const uint64_t waves = (uint64_t)gridDim.x * WAVES;
  for (uint64_t base = wave * 64; base < n; base += waves * 64) {
    // one coalesced index load per lane, handed to the groups by shuffles,
    // so the 16 line loads issue back to back (as the probe's come from LDS)
    const uint64_t me = base + lane;
    const uint32_t mine = me < n ? idx[me] : 0xFFFFFFFFu;
    uint64_t w[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint64_t line = (uint32_t)__shfl((int)mine, 4 * j + g);
      w[j] = line < n_lines ? table[line * 16 + sl] : 0;  // an index past the table reads nothing
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint64_t x = row_xor(w[j]);
      const uint64_t i = base + 4 * j + g;
      if (sl == 0 && i < n) out[i] = x;
    }
  }
}

}  // namespace hive_gather

extern "C" hive_status hive_gather_lines(const uint64_t *d_table, uint64_t n_lines, const uint32_t *d_idx,
                                         uint64_t n, uint64_t *d_out, void *stream) {
  using namespace hive_gather;
  if (n && (!d_table || !d_idx || !d_out || n_lines == 0)) return HIVE_ERR_ARG;
  if (n_lines > (1ull << 32)) return HIVE_ERR_ARG;
  if (n == 0) return HIVE_OK;
  const uint64_t waves = (n + 63) / 64;
  const uint64_t blocks = (waves + WAVES - 1) / WAVES;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)(blocks < 32768 ? blocks : 32768)), dim3(BLOCK), 0,
                     (hipStream_t)stream, d_table, n_lines, d_idx, n, d_out);
  return hipGetLastError() == hipSuccess ? HIVE_OK : HIVE_ERR_HIP;
}
