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
