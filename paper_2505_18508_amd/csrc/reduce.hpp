// Block-wide reductions for 64-wide wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

extern "C" __device__ uint32_t __ockl_wfred_add_u32(uint32_t);
extern "C" __device__ uint64_t __ockl_wfred_add_u64(uint64_t);

namespace ising {

// Sums over the active lanes of a wave (lanes a partial last wave does not
// have count 0), returned to every active lane: the device library's
// cross-lane reduction.  Used before one atomic per wave, since 64 lanes
// adding to one LDS or global address are processed one lane at a time.
__device__ __forceinline__ uint32_t wave_total(uint32_t v) { return __ockl_wfred_add_u32(v); }
__device__ __forceinline__ uint64_t wave_total(uint64_t v) { return __ockl_wfred_add_u64(v); }

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over a block of BLOCK threads (BLOCK a multiple of 64); the result is
// valid in thread 0.  Contains barriers: every thread of the block must call.
template <int BLOCK>
__device__ __forceinline__ int64_t block_sum(int64_t v) {
  __shared__ int64_t part[BLOCK / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) part[wave] = v;
  __syncthreads();
  int64_t total = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) total += part[k];
  }
  return total;
}

}  // namespace ising
