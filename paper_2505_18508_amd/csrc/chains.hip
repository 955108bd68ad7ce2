// The threshold compare chains of the bit-sliced kernels, run on given words
// for cross-checks (paper, Section III: a replica at dE = 4k > 0 flips iff
// its uniform word is below T_k).  One thread per set of 32 words; every
// lane of the launch runs (lanes past the last set repeat it), so the
// screened chains see whole waves as in the sweep kernels.
#include <hip/hip_runtime.h>

#include "bitslice.hpp"
#include "internal.hpp"
#include "word32.hpp"

namespace ising {
namespace {

constexpr int kChainsBlock = 256;

// Per-replica thresholds of the 16-word chains (replica r = word index & 3),
// taken from the three given ones in a fixed pattern.
struct ReplicaThr {
  uint32_t a[4], b[4], c[4];
};

__device__ __forceinline__ ReplicaThr replica_thr(uint32_t T1, uint32_t T2, uint32_t T3) {
  return ReplicaThr{{T1, T2, T3, T1}, {T2, T1, T2, T3}, {T3, T3, T1, T2}};
}

__global__ void __launch_bounds__(kChainsBlock)
    k_compare_chains(int64_t n, const uint32_t* u, const uint32_t* sel2, const uint32_t* sel3, uint32_t T1,
                     uint32_t T2, uint32_t T3, uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * kChainsBlock + threadIdx.x;
  const int64_t w = i < n ? i : n - 1;
  uint32_t x[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) x[j] = u[w * 32 + j];
  const uint32_t s2 = sel2[w], s3 = sel3[w];
  uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < 32; j += 2) mn = min(min(mn, x[j]), x[j + 1]);
  const ReplicaThr p = replica_thr(T1, T2, T3);
  uint32_t r[8];
  r[0] = lt_select32(x, s2, T1, T2);
  r[1] = lt_select32_3(x, s2, s3, T1, T2, T3);
  // the one-level chain of the four-replica kernels: four blocks of four
  // words, word 4 j + q against replica q's threshold
  uint32_t c1 = 0u, d1 = 0u, d2 = 0u;
#pragma unroll
  for (int j = 3; j >= 0; --j) {
    if (j == 3)
      lt_shift_in4<1, true>(c1, d1, d2, x + 4 * j, p.a, p.b, p.c);
    else
      lt_shift_in4<1>(c1, d1, d2, x + 4 * j, p.a, p.b, p.c);
  }
  r[2] = c1;
  r[3] = w32_screened_lt(x, mn, T1);
  r[4] = w32_screened_lt(x, mn, T2);
  r[5] = w32_screened_lt(x, mn, T3);
  r[6] = lt_select16(x, s2 & 0xFFFFu, p.a, p.b);
  r[7] = lt_select16_3(x, s2 & 0xFFFFu, s3 & 0xFFFFu, p.a, p.b, p.c);
  if (i < n) {
#pragma unroll
    for (int k = 0; k < 8; ++k) out[i * 8 + k] = r[k];
  }
}

}  // namespace

hipError_t launch_compare_chains(int64_t n, const uint32_t* u, const uint32_t* sel2, const uint32_t* sel3,
                                 uint32_t T1, uint32_t T2, uint32_t T3, uint32_t* out, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + kChainsBlock - 1) / kChainsBlock;
  hipLaunchKernelGGL(k_compare_chains, dim3((unsigned)blocks), dim3(kChainsBlock), 0, stream, n, u, sel2, sel3, T1,
                     T2, T3, out);
  return hipGetLastError();
}

}  // namespace ising
