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
// One level of the above as volatile statements, for a chain that runs under
// a wave-uniform branch: plain asm counts as free of side effects, and the
// compiler may hoist the whole chain out of the branch.
template <bool FIRST = false>
__device__ __forceinline__ void lt_shift_in4_kept(uint32_t& c, const uint32_t* u, uint32_t T) {
  uint32_t d;
#define ISING_LT1(S1)                                                                                        \
  ISING_LT_SUB(2, 6) S1(1) ISING_LT_SUB(3, 7) ISING_LT_ADD(1) ISING_LT_SUB(4, 8) ISING_LT_ADD(1) ISING_LT_SUB(5, 9) \
  ISING_LT_ADD(1)
  if (FIRST)
    asm volatile(ISING_LT1(ISING_LT_SET)
                 : "=&v"(d), "=&v"(c)
                 : "s"(T), "s"(T), "s"(T), "s"(T), "v"(u[3]), "v"(u[2]), "v"(u[1]), "v"(u[0])
                 : "vcc");
  else
    asm volatile(ISING_LT1(ISING_LT_ADD)
                 : "=&v"(d), "+v"(c)
                 : "s"(T), "s"(T), "s"(T), "s"(T), "v"(u[3]), "v"(u[2]), "v"(u[1]), "v"(u[0])
                 : "vcc");
#undef ISING_LT1
}
// Bits (u_31 < T(31), ..., u_0 < T(0)) of 32 words, word j compared with
// T_hi where bit j of sel is set and with T_lo elsewhere: one chain for two
// levels.  The result register starts as sel; each add with carry shifts the
// previous word's borrow in at the bottom and the next word's selector bit
// out at the top, into the carry that picks the threshold.  Three
// instructions a word (select, borrow, add) against four for two chains, and
// the carry never leaves the block.
#define ISING_SEL_STEP(U)                      \
  "v_cndmask_b32_e32 %1, %3, %4, vcc\n\t"      \
  "v_sub_co_u32_e32 %2, vcc, %" #U ", %1\n\t" \
  "v_addc_co_u32_e32 %0, vcc, %0, %0, vcc\n\t"
__device__ __forceinline__ uint32_t lt_select32(const uint32_t* u, uint32_t sel, uint32_t T_lo, uint32_t T_hi) {
  uint32_t c = sel, t, d;
  asm("v_add_co_u32_e32 %0, vcc, %0, %0\n\t"
      ISING_SEL_STEP(36) ISING_SEL_STEP(35) ISING_SEL_STEP(34) ISING_SEL_STEP(33) ISING_SEL_STEP(32) ISING_SEL_STEP(31)
      ISING_SEL_STEP(30) ISING_SEL_STEP(29) ISING_SEL_STEP(28) ISING_SEL_STEP(27) ISING_SEL_STEP(26) ISING_SEL_STEP(25)
      ISING_SEL_STEP(24) ISING_SEL_STEP(23) ISING_SEL_STEP(22) ISING_SEL_STEP(21) ISING_SEL_STEP(20) ISING_SEL_STEP(19)
      ISING_SEL_STEP(18) ISING_SEL_STEP(17) ISING_SEL_STEP(16) ISING_SEL_STEP(15) ISING_SEL_STEP(14) ISING_SEL_STEP(13)
      ISING_SEL_STEP(12) ISING_SEL_STEP(11) ISING_SEL_STEP(10) ISING_SEL_STEP(9) ISING_SEL_STEP(8) ISING_SEL_STEP(7)
      ISING_SEL_STEP(6) ISING_SEL_STEP(5)
      : "+v"(c), "=&v"(t), "=&v"(d)
      : "v"(T_lo), "v"(T_hi), "v"(u[0]), "v"(u[1]), "v"(u[2]), "v"(u[3]), "v"(u[4]), "v"(u[5]), "v"(u[6]),
        "v"(u[7]), "v"(u[8]), "v"(u[9]), "v"(u[10]), "v"(u[11]), "v"(u[12]), "v"(u[13]), "v"(u[14]), "v"(u[15]),
        "v"(u[16]), "v"(u[17]), "v"(u[18]), "v"(u[19]), "v"(u[20]), "v"(u[21]), "v"(u[22]), "v"(u[23]),
        "v"(u[24]), "v"(u[25]), "v"(u[26]), "v"(u[27]), "v"(u[28]), "v"(u[29]), "v"(u[30]), "v"(u[31])
      : "vcc");
  return c;
}
// The same for three levels: bit j of sel3 picks T3, else bit j of sel2
// picks T2, else T1 (the two selector sets are disjoint).  sel3 rides in the
// result register as sel does above; sel2 is shifted out of its own register.
// Five instructions a word against six for three chains.
#define ISING_SEL3_STEP(U)                     \
  "v_cndmask_b32_e32 %2, %4, %6, vcc\n\t"      \
  "v_add_co_u32_e32 %1, vcc, %1, %1\n\t"       \
  "v_cndmask_b32_e32 %2, %2, %5, vcc\n\t"      \
  "v_sub_co_u32_e32 %3, vcc, %" #U ", %2\n\t" \
  "v_addc_co_u32_e32 %0, vcc, %0, %0, vcc\n\t"
__device__ __forceinline__ uint32_t lt_select32_3(const uint32_t* u, uint32_t sel2, uint32_t sel3, uint32_t T1,
                                                  uint32_t T2, uint32_t T3) {
  uint32_t c = sel3, s = sel2, t, d;
  asm("v_add_co_u32_e32 %0, vcc, %0, %0\n\t"
      ISING_SEL3_STEP(38) ISING_SEL3_STEP(37) ISING_SEL3_STEP(36) ISING_SEL3_STEP(35) ISING_SEL3_STEP(34)
      ISING_SEL3_STEP(33) ISING_SEL3_STEP(32) ISING_SEL3_STEP(31) ISING_SEL3_STEP(30) ISING_SEL3_STEP(29)
      ISING_SEL3_STEP(28) ISING_SEL3_STEP(27) ISING_SEL3_STEP(26) ISING_SEL3_STEP(25) ISING_SEL3_STEP(24)
      ISING_SEL3_STEP(23) ISING_SEL3_STEP(22) ISING_SEL3_STEP(21) ISING_SEL3_STEP(20) ISING_SEL3_STEP(19)
      ISING_SEL3_STEP(18) ISING_SEL3_STEP(17) ISING_SEL3_STEP(16) ISING_SEL3_STEP(15) ISING_SEL3_STEP(14)
      ISING_SEL3_STEP(13) ISING_SEL3_STEP(12) ISING_SEL3_STEP(11) ISING_SEL3_STEP(10) ISING_SEL3_STEP(9)
      ISING_SEL3_STEP(8) ISING_SEL3_STEP(7)
      : "+v"(c), "+v"(s), "=&v"(t), "=&v"(d)
      : "v"(T1), "v"(T2), "v"(T3), "v"(u[0]), "v"(u[1]), "v"(u[2]), "v"(u[3]), "v"(u[4]), "v"(u[5]), "v"(u[6]),
        "v"(u[7]), "v"(u[8]), "v"(u[9]), "v"(u[10]), "v"(u[11]), "v"(u[12]), "v"(u[13]), "v"(u[14]), "v"(u[15]),
        "v"(u[16]), "v"(u[17]), "v"(u[18]), "v"(u[19]), "v"(u[20]), "v"(u[21]), "v"(u[22]), "v"(u[23]),
        "v"(u[24]), "v"(u[25]), "v"(u[26]), "v"(u[27]), "v"(u[28]), "v"(u[29]), "v"(u[30]), "v"(u[31])
      : "vcc");
  return c;
}
#undef ISING_SEL3_STEP
#undef ISING_SEL_STEP
// The chains above for the 16 words of a four-replica word (word 4 j + r:
// site j, replica r), each replica with its own pair or triple of
// thresholds: T_lo[r] / T_hi[r], or T1[r] / T2[r] / T3[r].  The selector bits
// sit in bits 0..15 of sel (sel2, sel3) and results come out in bits 0..15.
#define ISING_SEL16_STEP(TL, TH, U)              \
  "v_cndmask_b32_e32 %1, %" #TL ", %" #TH ", vcc\n\t" \
  "v_sub_co_u32_e32 %2, vcc, %" #U ", %1\n\t"   \
  "v_addc_co_u32_e32 %0, vcc, %0, %0, vcc\n\t"
__device__ __forceinline__ uint32_t lt_select16(const uint32_t* u, uint32_t sel, const uint32_t* T_lo,
                                                const uint32_t* T_hi) {
  uint32_t c = sel << 16, t, d;
  asm("v_add_co_u32_e32 %0, vcc, %0, %0\n\t"
      ISING_SEL16_STEP(6, 10, 26) ISING_SEL16_STEP(5, 9, 25) ISING_SEL16_STEP(4, 8, 24) ISING_SEL16_STEP(3, 7, 23)
      ISING_SEL16_STEP(6, 10, 22) ISING_SEL16_STEP(5, 9, 21) ISING_SEL16_STEP(4, 8, 20) ISING_SEL16_STEP(3, 7, 19)
      ISING_SEL16_STEP(6, 10, 18) ISING_SEL16_STEP(5, 9, 17) ISING_SEL16_STEP(4, 8, 16) ISING_SEL16_STEP(3, 7, 15)
      ISING_SEL16_STEP(6, 10, 14) ISING_SEL16_STEP(5, 9, 13) ISING_SEL16_STEP(4, 8, 12) ISING_SEL16_STEP(3, 7, 11)
      : "+v"(c), "=&v"(t), "=&v"(d)
      : "v"(T_lo[0]), "v"(T_lo[1]), "v"(T_lo[2]), "v"(T_lo[3]), "v"(T_hi[0]), "v"(T_hi[1]), "v"(T_hi[2]),
        "v"(T_hi[3]), "v"(u[0]), "v"(u[1]), "v"(u[2]), "v"(u[3]), "v"(u[4]), "v"(u[5]), "v"(u[6]), "v"(u[7]),
        "v"(u[8]), "v"(u[9]), "v"(u[10]), "v"(u[11]), "v"(u[12]), "v"(u[13]), "v"(u[14]), "v"(u[15])
      : "vcc");
  return c;
}
#undef ISING_SEL16_STEP
#define ISING_SEL16_3_STEP(T1, T2, T3, U)         \
  "v_cndmask_b32_e32 %2, %" #T1 ", %" #T3 ", vcc\n\t" \
  "v_add_co_u32_e32 %1, vcc, %1, %1\n\t"          \
  "v_cndmask_b32_e32 %2, %2, %" #T2 ", vcc\n\t"   \
  "v_sub_co_u32_e32 %3, vcc, %" #U ", %2\n\t"    \
  "v_addc_co_u32_e32 %0, vcc, %0, %0, vcc\n\t"
__device__ __forceinline__ uint32_t lt_select16_3(const uint32_t* u, uint32_t sel2, uint32_t sel3, const uint32_t* T1,
                                                  const uint32_t* T2, const uint32_t* T3) {
  uint32_t c = sel3 << 16, s = sel2 << 16, t, d;
  asm("v_add_co_u32_e32 %0, vcc, %0, %0\n\t"
      ISING_SEL16_3_STEP(7, 11, 15, 31) ISING_SEL16_3_STEP(6, 10, 14, 30) ISING_SEL16_3_STEP(5, 9, 13, 29)
      ISING_SEL16_3_STEP(4, 8, 12, 28) ISING_SEL16_3_STEP(7, 11, 15, 27) ISING_SEL16_3_STEP(6, 10, 14, 26)
      ISING_SEL16_3_STEP(5, 9, 13, 25) ISING_SEL16_3_STEP(4, 8, 12, 24) ISING_SEL16_3_STEP(7, 11, 15, 23)
      ISING_SEL16_3_STEP(6, 10, 14, 22) ISING_SEL16_3_STEP(5, 9, 13, 21) ISING_SEL16_3_STEP(4, 8, 12, 20)
      ISING_SEL16_3_STEP(7, 11, 15, 19) ISING_SEL16_3_STEP(6, 10, 14, 18) ISING_SEL16_3_STEP(5, 9, 13, 17)
      ISING_SEL16_3_STEP(4, 8, 12, 16)
      : "+v"(c), "+v"(s), "=&v"(t), "=&v"(d)
      : "v"(T1[0]), "v"(T1[1]), "v"(T1[2]), "v"(T1[3]), "v"(T2[0]), "v"(T2[1]), "v"(T2[2]), "v"(T2[3]),
        "v"(T3[0]), "v"(T3[1]), "v"(T3[2]), "v"(T3[3]), "v"(u[0]), "v"(u[1]), "v"(u[2]), "v"(u[3]), "v"(u[4]),
        "v"(u[5]), "v"(u[6]), "v"(u[7]), "v"(u[8]), "v"(u[9]), "v"(u[10]), "v"(u[11]), "v"(u[12]), "v"(u[13]),
        "v"(u[14]), "v"(u[15])
      : "vcc");
  return c;
}
#undef ISING_SEL16_3_STEP
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
