// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
// written from its published definition: ten rounds, each forming the two
// 64-bit products M_a * x0 and M_b * x2, then
//   x' = (hi_b ^ x1 ^ k0, lo_b, hi_a ^ x3 ^ k1, lo_a),
// with the key advanced by the Weyl increments between rounds.
//
// Device forms: the 32x32->64 products are single v_mad_u64_u32 and each
// three-way xor of per-lane values is one v_bitop3_b32 (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeylB = 0xBB67AE85u;

constexpr uint32_t kTagMetropolis = 0u;
constexpr uint32_t kTagInit = 1u;
constexpr uint32_t kTagWeight = 2u;
constexpr uint32_t kTagExchange = 4u;  // replica-exchange decisions (3 keys the network's initial weights)

struct u32x4 {
  uint32_t v[4];
};

// Portable form (host code and any device code without a uniform key).
__host__ __device__ inline u32x4 philox_ref(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
    const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
    const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
  u32x4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// a ^ b ^ c in one VALU op (v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}

// Device form for a counter whose word c0 varies across the lanes of a wave
// while c1, c2, c3 and the key are wave-uniform (the sweep's (site, sweep,
// replica quad, tag) counters).  Bit-identical to philox_ref; the first two
// rounds are written so that their uniform halves stay on the scalar unit.
__device__ __forceinline__ u32x4 philox_lane_c0(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
  {  // round 1: M_b * c2 uniform
    const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
    const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
    const uint32_t n0 = ((uint32_t)(pb >> 32) ^ c1) ^ k0;
    const uint32_t n2 = (uint32_t)(pa >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
  {  // round 2: c0, c1 uniform
    const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
    const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
    const uint32_t n0 = (uint32_t)(pb >> 32) ^ (c1 ^ k0);
    const uint32_t n2 = ((uint32_t)(pa >> 32) ^ k1) ^ c3;
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
  {  // round 3: c3 uniform
    const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
    const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
    const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
    const uint32_t n2 = (uint32_t)(pa >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
#pragma unroll
  for (int r = 3; r < 10; ++r) {
    const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
    const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
    const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
  u32x4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// Two blocks of philox_lane_c0 whose counters differ in c0 only (ca, cb),
// computed round by round in lockstep: the two dependency chains interleave,
// which doubles the independent work a wave can issue between the products'
// latencies.  The uniform halves of the first two rounds are shared.
__device__ __forceinline__ void philox_lane_c0_x2(uint64_t key, uint32_t ca, uint32_t cb, uint32_t c1, uint32_t c2,
                                                  uint32_t c3, u32x4& outa, u32x4& outb) {
  uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
  uint32_t a0, a1, a2, a3, b0, b1, b2, b3;
  {  // round 1: M_b * c2 uniform, so the new words 0 and 1 are shared
    const uint64_t pa = (uint64_t)kPhiloxMulA * ca;
    const uint64_t pb = (uint64_t)kPhiloxMulA * cb;
    const uint64_t pu = (uint64_t)kPhiloxMulB * c2;
    const uint32_t n0 = ((uint32_t)(pu >> 32) ^ c1) ^ k0;
    const uint32_t ck = c3 ^ k1;
    a0 = n0;
    b0 = n0;
    a1 = (uint32_t)pu;
    b1 = (uint32_t)pu;
    a2 = (uint32_t)(pa >> 32) ^ ck;
    b2 = (uint32_t)(pb >> 32) ^ ck;
    a3 = (uint32_t)pa;
    b3 = (uint32_t)pb;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
  {  // round 2: words 0 and 1 uniform (shared)
    const uint64_t pu = (uint64_t)kPhiloxMulA * a0;
    const uint64_t qa = (uint64_t)kPhiloxMulB * a2;
    const uint64_t qb = (uint64_t)kPhiloxMulB * b2;
    const uint32_t ck = a1 ^ k0;
    const uint32_t hk = (uint32_t)(pu >> 32) ^ k1;
    const uint32_t na0 = (uint32_t)(qa >> 32) ^ ck;
    const uint32_t nb0 = (uint32_t)(qb >> 32) ^ ck;
    const uint32_t na2 = hk ^ a3;
    const uint32_t nb2 = hk ^ b3;
    a1 = (uint32_t)qa;
    b1 = (uint32_t)qb;
    a3 = (uint32_t)pu;
    b3 = (uint32_t)pu;
    a0 = na0;
    b0 = nb0;
    a2 = na2;
    b2 = nb2;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
  {  // round 3: word 3 uniform (shared)
    const uint64_t pa = (uint64_t)kPhiloxMulA * a0;
    const uint64_t pb = (uint64_t)kPhiloxMulA * b0;
    const uint64_t qa = (uint64_t)kPhiloxMulB * a2;
    const uint64_t qb = (uint64_t)kPhiloxMulB * b2;
    const uint32_t ck = a3 ^ k1;
    const uint32_t na0 = xor3((uint32_t)(qa >> 32), a1, k0);
    const uint32_t nb0 = xor3((uint32_t)(qb >> 32), b1, k0);
    const uint32_t na2 = (uint32_t)(pa >> 32) ^ ck;
    const uint32_t nb2 = (uint32_t)(pb >> 32) ^ ck;
    a1 = (uint32_t)qa;
    b1 = (uint32_t)qb;
    a3 = (uint32_t)pa;
    b3 = (uint32_t)pb;
    a0 = na0;
    b0 = nb0;
    a2 = na2;
    b2 = nb2;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
#pragma unroll
  for (int r = 3; r < 10; ++r) {
    const uint64_t pa = (uint64_t)kPhiloxMulA * a0;
    const uint64_t pb = (uint64_t)kPhiloxMulA * b0;
    const uint64_t qa = (uint64_t)kPhiloxMulB * a2;
    const uint64_t qb = (uint64_t)kPhiloxMulB * b2;
    const uint32_t na0 = xor3((uint32_t)(qa >> 32), a1, k0);
    const uint32_t nb0 = xor3((uint32_t)(qb >> 32), b1, k0);
    const uint32_t na2 = xor3((uint32_t)(pa >> 32), a3, k1);
    const uint32_t nb2 = xor3((uint32_t)(pb >> 32), b3, k1);
    a1 = (uint32_t)qa;
    b1 = (uint32_t)qb;
    a3 = (uint32_t)pa;
    b3 = (uint32_t)pb;
    a0 = na0;
    b0 = nb0;
    a2 = na2;
    b2 = nb2;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
  outa.v[0] = a0; outa.v[1] = a1; outa.v[2] = a2; outa.v[3] = a3;
  outb.v[0] = b0; outb.v[1] = b1; outb.v[2] = b2; outb.v[3] = b3;
}

// Device form for arbitrary (per-lane) counters; bit-identical to philox_ref.
__device__ __forceinline__ u32x4 philox_lanes(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
    const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
    const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxWeylA;
    k1 += kPhiloxWeylB;
  }
  u32x4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

}  // namespace ising
