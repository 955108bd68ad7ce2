// Bit-sliced helpers shared by the kernels that keep one spin bit per
// (site, replica) lane of a 32-bit word.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace ising {

// Bit-sliced population count of DEG one-bit inputs per lane:
// u = u0 + 2 u1 + 4 u2 (DEG = 4 or 6).
template <int DEG>
__device__ __forceinline__ void bond_count3(const uint32_t* x, uint32_t& u0, uint32_t& u1, uint32_t& u2) {
  if (DEG == 4) {
    const uint32_t s1 = x[0] ^ x[1], c1 = x[0] & x[1];
    const uint32_t s2 = x[2] ^ x[3], c2 = x[2] & x[3];
    u0 = s1 ^ s2;
    const uint32_t k = s1 & s2;
    u1 = xor3(c1, c2, k);
    u2 = (c1 & c2) | (k & (c1 | c2));
  } else {
    const uint32_t s1 = xor3(x[0], x[1], x[2]);
    const uint32_t c1 = (x[0] & x[1]) | (x[2] & (x[0] | x[1]));
    const uint32_t s2 = xor3(x[3], x[4], x[5]);
    const uint32_t c2 = (x[3] & x[4]) | (x[5] & (x[3] | x[4]));
    u0 = s1 ^ s2;
    const uint32_t k = s1 & s2;
    u1 = xor3(c1, c2, k);
    u2 = (c1 & c2) | (k & (c1 | c2));
  }
}

// Number of leading nonzero threshold levels of a sweep (thresholds
// decrease with k, so the first zero ends the prefix).
template <int NDIM>
__device__ __forceinline__ int sweep_levels(uint32_t T1, uint32_t T2, uint32_t T3) {
  return T1 == 0u ? 0 : T2 == 0u ? 1 : (NDIM == 2 || T3 == 0u) ? 2 : 3;
}

// The four words of one Philox block shifted into LEV compare chains at once
// (word 3 first), word b against its own thresholds T_k[b] (the four
// replicas of a quad may run at different temperatures; all are uniform
// over the block): c_k = 16 c_k + bits (u_3 < T_k[3], ..., u_0 < T_k[0]).
// Each compare is two VALU instructions: the borrow of u - T, then an add
// with carry that doubles c_k and shifts the borrow in.  FIRST starts the
// chains instead: the first borrow of each level becomes c_k (a select of 0
// or 1), so no starting value has to be set.  One asm block per Philox block
// keeps the carry sequence free of inserted waits.
#define ISING_LT_SUB(T, U) "v_subrev_co_u32_e32 %0, vcc, %" #T ", %" #U "\n\t"
#define ISING_LT_ADD(C) "v_addc_co_u32_e32 %" #C ", vcc, %" #C ", %" #C ", vcc\n\t"
#define ISING_LT_SET(C) "v_cndmask_b32_e64 %" #C ", 0, 1, vcc\n\t"
template <int LEV, bool FIRST = false>
__device__ __forceinline__ void lt_shift_in4(uint32_t& c1, uint32_t& c2, uint32_t& c3, const uint32_t* u,
                                             const uint32_t* T1, const uint32_t* T2, const uint32_t* T3) {
  uint32_t d;
  if (LEV == 1) {
#define ISING_LT1(S1)                                                                                        \
  ISING_LT_SUB(2, 6) S1(1) ISING_LT_SUB(3, 7) ISING_LT_ADD(1) ISING_LT_SUB(4, 8) ISING_LT_ADD(1) ISING_LT_SUB(5, 9) \
  ISING_LT_ADD(1)
    if (FIRST)
      asm(ISING_LT1(ISING_LT_SET)
          : "=&v"(d), "=&v"(c1)
          : "s"(T1[3]), "s"(T1[2]), "s"(T1[1]), "s"(T1[0]), "v"(u[3]), "v"(u[2]), "v"(u[1]), "v"(u[0])
          : "vcc");
    else
      asm(ISING_LT1(ISING_LT_ADD)
          : "=&v"(d), "+v"(c1)
          : "s"(T1[3]), "s"(T1[2]), "s"(T1[1]), "s"(T1[0]), "v"(u[3]), "v"(u[2]), "v"(u[1]), "v"(u[0])
          : "vcc");
#undef ISING_LT1
  } else if (LEV == 2) {
#define ISING_LT2(S1)                                                                                      \
  ISING_LT_SUB(3, 11) S1(1) ISING_LT_SUB(7, 11) S1(2) ISING_LT_SUB(4, 12) ISING_LT_ADD(1) ISING_LT_SUB(8, 12) \
  ISING_LT_ADD(2) ISING_LT_SUB(5, 13) ISING_LT_ADD(1) ISING_LT_SUB(9, 13) ISING_LT_ADD(2) ISING_LT_SUB(6, 14)  \
  ISING_LT_ADD(1) ISING_LT_SUB(10, 14) ISING_LT_ADD(2)
    if (FIRST)
      asm(ISING_LT2(ISING_LT_SET)
          : "=&v"(d), "=&v"(c1), "=&v"(c2)
          : "s"(T1[3]), "s"(T1[2]), "s"(T1[1]), "s"(T1[0]), "s"(T2[3]), "s"(T2[2]), "s"(T2[1]), "s"(T2[0]),
            "v"(u[3]), "v"(u[2]), "v"(u[1]), "v"(u[0])
          : "vcc");
    else
      asm(ISING_LT2(ISING_LT_ADD)
          : "=&v"(d), "+v"(c1), "+v"(c2)
          : "s"(T1[3]), "s"(T1[2]), "s"(T1[1]), "s"(T1[0]), "s"(T2[3]), "s"(T2[2]), "s"(T2[1]), "s"(T2[0]),
            "v"(u[3]), "v"(u[2]), "v"(u[1]), "v"(u[0])
          : "vcc");
#undef ISING_LT2
  } else {
#define ISING_LT3(S1)                                                                                         \
  ISING_LT_SUB(4, 16) S1(1) ISING_LT_SUB(8, 16) S1(2) ISING_LT_SUB(12, 16) S1(3) ISING_LT_SUB(5, 17)            \
  ISING_LT_ADD(1) ISING_LT_SUB(9, 17) ISING_LT_ADD(2) ISING_LT_SUB(13, 17) ISING_LT_ADD(3) ISING_LT_SUB(6, 18)   \
  ISING_LT_ADD(1) ISING_LT_SUB(10, 18) ISING_LT_ADD(2) ISING_LT_SUB(14, 18) ISING_LT_ADD(3) ISING_LT_SUB(7, 19)  \
  ISING_LT_ADD(1) ISING_LT_SUB(11, 19) ISING_LT_ADD(2) ISING_LT_SUB(15, 19) ISING_LT_ADD(3)
    if (FIRST)
      asm(ISING_LT3(ISING_LT_SET)
          : "=&v"(d), "=&v"(c1), "=&v"(c2), "=&v"(c3)
          : "s"(T1[3]), "s"(T1[2]), "s"(T1[1]), "s"(T1[0]), "s"(T2[3]), "s"(T2[2]), "s"(T2[1]), "s"(T2[0]),
            "s"(T3[3]), "s"(T3[2]), "s"(T3[1]), "s"(T3[0]), "v"(u[3]), "v"(u[2]), "v"(u[1]), "v"(u[0])
          : "vcc");
    else
      asm(ISING_LT3(ISING_LT_ADD)
          : "=&v"(d), "+v"(c1), "+v"(c2), "+v"(c3)
          : "s"(T1[3]), "s"(T1[2]), "s"(T1[1]), "s"(T1[0]), "s"(T2[3]), "s"(T2[2]), "s"(T2[1]), "s"(T2[0]),
            "s"(T3[3]), "s"(T3[2]), "s"(T3[1]), "s"(T3[0]), "v"(u[3]), "v"(u[2]), "v"(u[1]), "v"(u[0])
          : "vcc");
#undef ISING_LT3
  }
}
#undef ISING_LT_SUB
#undef ISING_LT_ADD
#undef ISING_LT_SET

// The same with one threshold per level for all four words.
template <int LEV, bool FIRST = false>
__device__ __forceinline__ void lt_shift_in4(uint32_t& c1, uint32_t& c2, uint32_t& c3, const uint32_t* u, uint32_t T1,
                                             uint32_t T2, uint32_t T3) {
  const uint32_t t1[4] = {T1, T1, T1, T1}, t2[4] = {T2, T2, T2, T2}, t3[4] = {T3, T3, T3, T3};
  lt_shift_in4<LEV, FIRST>(c1, c2, c3, u, t1, t2, t3);
}

}  // namespace ising
