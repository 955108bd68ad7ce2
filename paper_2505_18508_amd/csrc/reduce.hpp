// Block-wide reductions for 64-wide wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

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
