// Metropolis decision of a word that holds one site of 32 replicas (bit j:
// replica 32 g + j), shared by the on-chip and the streamed 32-replica
// kernels.  Paper, Section III: a replica whose flip lowers or keeps the
// energy flips; one at dE = 4k > 0 flips iff its uniform word is below the
// threshold T_k = floor(2^32 exp(-4 k beta)) of the sweep.  The eight Philox
// blocks of (site, sweep, replica quad, tag 0) give the 32 words.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bitslice.hpp"
#include "philox.hpp"

namespace ising {

// Sweeps whose smallest nonzero threshold lies below this bound screen their
// compares: a wave of 64 site words draws 2,048 words, so a level's chain is
// then skipped in most waves.
constexpr uint32_t kW32ScreenBelow = 1u << 21;

// A sweep's mode: 2 x (number of nonzero thresholds) + 1 when its compares
// are screened.  A function of the schedule alone, the same in every thread.
// Fewer nonzero levels than deg/2 are always screened: the thresholds of one
// beta are powers of exp(-4 beta), so a vanished level leaves the others
// below 2^16 (one level) or 2^11 (two of three), far under the bound.  The
// modes are thus 0, 3 and, in 2-D, 4, 5 or, in 3-D, 5, 6, 7.
template <int NDIM>
__device__ __forceinline__ int w32_mode(uint32_t T1, uint32_t T2, uint32_t T3) {
  const int lev = sweep_levels<NDIM>(T1, T2, T3);
  const uint32_t low = lev == 1 ? T1 : lev == 2 ? T2 : T3;
  return 2 * lev + (lev > 0 && (lev < NDIM || low < kW32ScreenBelow) ? 1 : 0);
}

// The 32 Philox words of a site word: u[j] for replica j.
__device__ __forceinline__ void w32_draws(uint64_t seed, uint32_t ci, uint32_t t, uint32_t quad0, uint32_t* u) {
#pragma unroll
  for (int q = 7; q >= 0; --q) {
    const u32x4 r = philox_lane_c0(seed, ci, t, quad0 + (uint32_t)q, kTagMetropolis);
#pragma unroll
    for (int j = 0; j < 4; ++j) u[4 * q + j] = r.v[j];
  }
}

// Bits of the 32 words u below T, where mn is this lane's smallest word:
// when no lane of the wave holds a word below T every lane's result is zero,
// and the wave skips the chain.
__device__ __forceinline__ uint32_t w32_screened_lt(const uint32_t* u, uint32_t mn, uint32_t T) {
  uint32_t c = 0u;
  if (__builtin_amdgcn_ballot_w64(mn < T) != 0u) {
#pragma unroll
    for (int q = 7; q >= 0; --q) {
      if (q == 7)
        lt_shift_in4_kept<true>(c, u + 4 * q, T);
      else
        lt_shift_in4_kept(c, u + 4 * q, T);
    }
  }
  return c;
}

// Flip bits of a site word from x[d] = unsatisfied-bond bits of its DEG
// bonds (any order): with u unsatisfied bonds dE = 2 deg - 4u, so u >= deg/2
// flips outright and u < deg/2 is level k = deg/2 - u.  LEV = number of
// nonzero thresholds of the sweep (a prefix, as they decrease with k); a
// level past LEV never flips.  SCREEN runs each level's own chain only in
// waves where some word falls below its threshold; otherwise (all deg/2
// levels nonzero, w32_mode) two or three levels share one chain whose
// threshold each replica's level bits pick.
// STATS: words that drew (n_words) and draws that decide (n_draws) over the
// valid replica lanes.
template <int NDIM, int LEV, bool SCREEN, bool STATS>
__device__ __forceinline__ uint32_t w32_decide(const uint32_t* x, uint64_t seed, uint32_t ci, uint32_t t,
                                               uint32_t quad0, uint32_t T1, uint32_t T2, uint32_t T3,
                                               uint32_t valid_lanes, uint32_t& n_words, uint32_t& n_draws) {
  constexpr int DEG = 2 * NDIM;
  uint32_t u0, u1, u2;
  bond_count3<DEG>(x, u0, u1, u2);
  uint32_t acc, k1, k2, k3 = 0u;
  if (NDIM == 2) {
    acc = u1 | u2;     // u >= 2
    k1 = u0 & ~acc;    // u == 1
    k2 = ~(u0 | acc);  // u == 0
  } else {
    acc = u2 | (u1 & u0);  // u >= 3
    k1 = u1 & ~u0 & ~u2;   // u == 2
    k2 = u0 & ~u1 & ~u2;   // u == 1
    k3 = ~(u0 | u1 | u2);  // u == 0
  }
  if (LEV == 0) return acc;
  const uint32_t need = k1 | (LEV >= 2 ? k2 : 0u) | (LEV >= 3 ? k3 : 0u);
  if (STATS) {
    n_words += 1u;
    n_draws += __popc(need & valid_lanes);
  }
  static_assert(SCREEN || LEV == 0 || LEV == NDIM, "unscreened sweeps with draws have every level nonzero");
  if (!SCREEN) {
    uint32_t u[32];
    w32_draws(seed, ci, t, quad0, u);
    const uint32_t c = LEV == 2 ? lt_select32(u, k2, T1, T2) : lt_select32_3(u, k2, k3, T1, T2, T3);
    return acc | (need & c);
  }
  uint32_t u[32];
  w32_draws(seed, ci, t, quad0, u);
  uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < 32; j += 2) mn = min(min(mn, u[j]), u[j + 1]);
  // T1 >= T2 >= T3: no word below T1 leaves the lower levels empty as well
  uint32_t F = acc | (k1 & w32_screened_lt(u, mn, T1));
  if (LEV >= 2) F |= k2 & w32_screened_lt(u, mn, T2);
  if (LEV >= 3) F |= k3 & w32_screened_lt(u, mn, T3);
  return F;
}

}  // namespace ising
