// Checkerboard Metropolis sweeps, 32 replicas per 32-bit LDS word.
//
// One block owns a group of 32 replicas for a whole window of sweeps.  The
// word of site (p, h) (colour-split order) holds bit j = spin of replica
// 32g + j (1: +1).  A second LDS array holds each site's weight signs (bit d
// set: weight of direction d is +1; order +x, -x, +y, -y, +z, -z).
//
// A visit of a site word (paper, Section III: the sweep visits every site
// once) computes for all 32 replicas at once which incident bonds are
// unsatisfied (w s_i s_j = +1, bit-parallel over replicas), adds them in a
// bit-sliced counter u (0..deg), and derives dE = 2 deg - 4u: replicas with
// u >= deg/2 (dE <= 0) flip, a replica with dE = 4k > 0 flips iff its Philox
// word of (site, sweep, replica >> 2, tag 0) is below T_k(sweep).  The eight
// Philox blocks of a word serve its eight replica quads.  Fields are
// recomputed from the neighbours' words at every visit, so nothing but spins
// lives on chip.  Same-colour sites are never neighbours on an even torus, so
// the parallel update equals the sequential sweep bit for bit.
//
// After the window: spins written back in canonical layout, accepted flips
// per replica (when requested), and energy H = sum_e w_e s_a s_b
// = 2 (#unsatisfied bonds) - |E| (eq. (2), J = -w, h = 0) with
// cut = (W_total - H) / 2 (eq. (1)).
#include <hip/hip_runtime.h>

#include "bitslice.hpp"
#include "internal.hpp"
#include "philox.hpp"
#include "reduce.hpp"

namespace ising {
namespace {

constexpr int kMaxBlock = 1024;
constexpr int kExtraWords = 112;  // [0,32) flips, [32,64) unsatisfied-bond counts, 64 invalid flags

struct BpArgs {
  Lattice lat;
  const uint8_t* wbits;  // colour-split order, bit d set: weight of direction d is -1
  int8_t* spins;
  const uint32_t* thr;
  int64_t* cut;
  int64_t* energy;
  uint32_t* flips;
  unsigned long long* stats;
  uint64_t seed;
  int64_t w_total;
  int32_t n_replicas;
  int32_t replica_offset;
  int32_t t_begin, t_end;
  int32_t init;
  int32_t lp;
  int32_t flush_every;  // sweeps between flushes of the 8-bit flip counters
};

// Bit-sliced population count of DEG one-bit inputs per lane: u = u0 + 2 u1 + 4 u2.
template <int DEG>
__device__ __forceinline__ void bond_count(const uint32_t* x, uint32_t& u0, uint32_t& u1, uint32_t& u2) {
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

// Per-lane value of a bit-sliced counter of NPLANES planes, added to LDS
// counters dst[0..31] (lanes below nvalid only): summed over the wave first,
// then one atomic per wave and counter.  Every thread of the block calls it.
template <int NPLANES>
__device__ __forceinline__ void flush_planes(uint32_t* planes, uint32_t* dst, int nvalid) {
  uint32_t any = 0u;
#pragma unroll
  for (int k = 0; k < NPLANES; ++k) any |= planes[k];
  if (__ballot(any != 0u) == 0ull) return;  // the whole wave has nothing to add
  for (int j = 0; j < nvalid; ++j) {
    uint32_t v = 0u;
#pragma unroll
    for (int k = 0; k < NPLANES; ++k) v |= ((planes[k] >> j) & 1u) << k;
    const uint32_t s = wave_total(v);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(&dst[j], s);
  }
#pragma unroll
  for (int k = 0; k < NPLANES; ++k) planes[k] = 0u;
}

// Add a 32-lane bit vector into a bit-sliced counter.
template <int NPLANES>
__device__ __forceinline__ void add_planes(uint32_t* planes, uint32_t x) {
#pragma unroll
  for (int k = 0; k < NPLANES; ++k) {
    const uint32_t c = planes[k] & x;
    planes[k] ^= x;
    x = c;
  }
}

// Threshold compares of the 32 replicas of a site word against the first LEV
// thresholds; bit j of c[k] = (Philox word of replica j) < T_{k+1}.
template <int LEV>
__device__ __forceinline__ void draw_compare(uint64_t seed, uint32_t ci, uint32_t t, uint32_t quad0, uint32_t T1,
                                             uint32_t T2, uint32_t T3, uint32_t& c1, uint32_t& c2, uint32_t& c3) {
#pragma unroll
  for (int q = 7; q >= 0; --q) {
    const u32x4 r = philox_lane_c0(seed, ci, t, quad0 + (uint32_t)q, kTagMetropolis);
    lt_shift_in4<LEV>(c1, c2, c3, r.v, T1, T2, T3);
  }
}

template <int NDIM, bool FLIPS, bool STATS>
__global__ void __launch_bounds__(kMaxBlock) k_sweep_bp32(BpArgs a) {
  extern __shared__ uint32_t lds[];
  constexpr int DEG = 2 * NDIM;
  const Lattice& L = a.lat;
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  uint32_t* extra = lds + L.n;
  uint8_t* wl = (uint8_t*)(extra + kExtraWords);  // [n] weight signs (bit set: +1)

  const int r0 = blockIdx.x * 32;
  const int nvalid = min(32, a.n_replicas - r0);
  const uint32_t quad0 = (uint32_t)(a.replica_offset + r0) >> 2;
  const size_t n = (size_t)L.n;

  for (int k = tid; k < kExtraWords; k += B) extra[k] = 0u;

  // ---- state in --------------------------------------------------------------
  uint32_t bad = 0u;
  for (uint32_t i = tid; i < (uint32_t)L.n; i += B) {
    int p;
    uint32_t h;
    site_to_split(L, i, p, h);
    const uint32_t slot = (uint32_t)p * (uint32_t)L.half + h;
    uint32_t word = 0u;
    if (a.init) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const u32x4 u = philox_lane_c0(a.seed, i, 0u, quad0 + q, kTagInit);
#pragma unroll
        for (int b = 0; b < 4; ++b) word |= (u.v[b] >> 31) << (4 * q + b);
      }
    } else {
      for (int j = 0; j < nvalid; ++j) {
        const int8_t v = a.spins[(size_t)(r0 + j) * n + i];
        word |= (v > 0 ? 1u : 0u) << j;
        bad |= (v != 1 && v != -1) ? (1u << j) : 0u;
      }
    }
    lds[slot] = word;
    wl[slot] = (uint8_t)(~a.wbits[slot] & ((1u << DEG) - 1u));
  }

  // ---- this thread's sites (as in the four-replica kernel) ------------------
  const uint32_t hx = (uint32_t)L.hx;
  const uint32_t m = (uint32_t)tid % hx;
  const uint32_t line0 = (uint32_t)tid / hx;
  const uint32_t m_up = (m + 1u == hx) ? 0u : m + 1u;
  const uint32_t m_dn = (m == 0u) ? hx - 1u : m - 1u;
  const uint32_t lp = (uint32_t)a.lp;
  const uint32_t Ly = (uint32_t)L.Ly, Lz = (uint32_t)L.Lz;
  const uint32_t lp_z = NDIM == 2 ? 0u : lp / Ly;
  const uint32_t lp_y = lp - lp_z * Ly;
  const uint32_t z0 = NDIM == 2 ? 0u : line0 / Ly;
  const uint32_t y0 = line0 - z0 * Ly;
  const bool active = tid < (int)(hx * lp);
  const uint32_t d_up = m_up - m, d_dn = m_dn - m;
  const uint32_t row = hx, plane = hx * Ly;
  const uint32_t dyp_wrap = row - plane, dym_wrap = plane - row;
  const uint32_t dzp_wrap = plane - plane * Lz, dzm_wrap = plane * Lz - plane;
  const uint32_t own_step = lp * hx;
  const uint32_t ci_step = lp * (uint32_t)L.Lx;
  __syncthreads();
  if (bad) atomicOr(&extra[64], bad);

  uint32_t fplanes[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) fplanes[k] = 0u;
  uint32_t n_blocks = 0u, n_draws = 0u;
  const uint32_t valid_lanes = nvalid == 32 ? 0xFFFFFFFFu : ((1u << nvalid) - 1u);

  for (int t = a.t_begin; t < a.t_end; ++t) {
    const uint32_t* tr = a.thr + (size_t)t * NDIM;
    const uint32_t T1 = tr[0], T2 = tr[1], T3 = NDIM == 3 ? tr[2] : 0u;
    for (int p = 0; p < 2; ++p) {
      if (active) {
        const uint32_t other = (uint32_t)(1 - 2 * p) * (uint32_t)L.half;
        uint32_t own = (uint32_t)p * (uint32_t)L.half + line0 * hx + m;
        uint32_t ci0 = line0 * (uint32_t)L.Lx + 2u * m;
        uint32_t y = y0, z = z0;
        for (uint32_t line = line0; line < (uint32_t)L.lines; line += lp) {
          const uint32_t o = (p + y + z) & 1u;
          const uint32_t base = own + other;
          uint32_t nb[DEG];
          nb[0] = base + (o ? d_up : 0u);
          nb[1] = base + (o ? 0u : d_dn);
          nb[2] = base + (y + 1u == Ly ? dyp_wrap : row);
          nb[3] = base + (y == 0u ? dym_wrap : 0u - row);
          if (NDIM == 3) {
            nb[DEG - 2] = base + (z + 1u == Lz ? dzp_wrap : plane);
            nb[DEG - 1] = base + (z == 0u ? dzm_wrap : 0u - plane);
          }
          const uint32_t ci = ci0 + o;
          const uint32_t s = lds[own];
          const uint32_t wp = wl[own];
          uint32_t x[DEG];
#pragma unroll
          for (int d = 0; d < DEG; ++d) {
            // unsatisfied bond: w s_i s_j = +1  <=>  (s_i == s_j) == (w == +1)
            const uint32_t plus = (uint32_t)__builtin_amdgcn_sbfe((int)wp, d, 1);  // all ones iff w = +1
            x[d] = xor3(s, lds[nb[d]], plus);
          }
          uint32_t u0, u1, u2;
          bond_count<DEG>(x, u0, u1, u2);
          // dE = 2 deg - 4u: flip when u >= deg/2; else k = deg/2 - u
          uint32_t acc, k1, k2, k3 = 0u;
          if (NDIM == 2) {
            acc = u1 | u2;        // u >= 2
            k1 = u0 & ~acc;       // u == 1
            k2 = ~(u0 | acc);     // u == 0
          } else {
            acc = u2 | (u1 & u0);           // u >= 3
            k1 = u1 & ~u0 & ~u2;            // u == 2
            k2 = u0 & ~u1 & ~u2;            // u == 1
            k3 = ~(u0 | u1 | u2);           // u == 0
          }
          uint32_t c1 = 0u, c2 = 0u, c3 = 0u;
          if (T1 != 0u) {
            // thresholds decrease with k, so the nonzero ones are a prefix
            if (T2 == 0u)
              draw_compare<1>(a.seed, ci, (uint32_t)t, quad0, T1, T2, T3, c1, c2, c3);
            else if (NDIM == 2 || T3 == 0u)
              draw_compare<2>(a.seed, ci, (uint32_t)t, quad0, T1, T2, T3, c1, c2, c3);
            else
              draw_compare<3>(a.seed, ci, (uint32_t)t, quad0, T1, T2, T3, c1, c2, c3);
            if (STATS) {
              const uint32_t need = k1 | (T2 ? k2 : 0u) | (T3 ? k3 : 0u);
              n_blocks += 8u;
              n_draws += __popc(need & valid_lanes);
            }
          }
          const uint32_t F = acc | (k1 & c1) | (k2 & c2) | (k3 & c3);
          if (F) lds[own] = s ^ F;
          if (FLIPS) add_planes<8>(fplanes, F);
          own += own_step;
          ci0 += ci_step;
          y += lp_y;
          z += lp_z;
          if (y >= Ly) {
            y -= Ly;
            z += 1u;
          }
        }
      }
      __syncthreads();
    }
    if (FLIPS && ((t - a.t_begin) % a.flush_every == a.flush_every - 1 || t + 1 == a.t_end))
      flush_planes<8>(fplanes, extra, nvalid);
  }

  // ---- unsatisfied bonds along +x, +y (+z): energy ---------------------------
  {
    uint32_t eplanes[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) eplanes[k] = 0u;
    if (active) {
      for (int p = 0; p < 2; ++p) {
        const uint32_t other = (uint32_t)(1 - 2 * p) * (uint32_t)L.half;
        uint32_t own = (uint32_t)p * (uint32_t)L.half + line0 * hx + m;
        uint32_t y = y0, z = z0;
        for (uint32_t line = line0; line < (uint32_t)L.lines; line += lp) {
          const uint32_t o = (p + y + z) & 1u;
          const uint32_t base = own + other;
          const uint32_t s = lds[own];
          const uint32_t wp = wl[own];
          uint32_t e = xor3(s, lds[base + (o ? d_up : 0u)], (uint32_t)__builtin_amdgcn_sbfe((int)wp, 0, 1));
          add_planes<12>(eplanes, e);
          e = xor3(s, lds[base + (y + 1u == Ly ? dyp_wrap : row)], (uint32_t)__builtin_amdgcn_sbfe((int)wp, 2, 1));
          add_planes<12>(eplanes, e);
          if (NDIM == 3) {
            e = xor3(s, lds[base + (z + 1u == Lz ? dzp_wrap : plane)], (uint32_t)__builtin_amdgcn_sbfe((int)wp, 4, 1));
            add_planes<12>(eplanes, e);
          }
          own += own_step;
          y += lp_y;
          z += lp_z;
          if (y >= Ly) {
            y -= Ly;
            z += 1u;
          }
        }
      }
    }
    flush_planes<12>(eplanes, extra + 32, nvalid);
  }
  // 64-bit totals (a block's can exceed 32 bits), one atomic per wave
  if (STATS) {
    const uint64_t nb = wave_total((uint64_t)n_blocks), nd = wave_total((uint64_t)n_draws);
    if ((tid & 63) == 0 && (nb | nd)) {
      atomicAdd(&a.stats[0], (unsigned long long)nb);
      atomicAdd(&a.stats[1], (unsigned long long)nd);
    }
  }
  __syncthreads();

  // ---- state out ------------------------------------------------------------
  for (uint32_t i = tid; i < (uint32_t)L.n; i += B) {
    int p;
    uint32_t h;
    site_to_split(L, i, p, h);
    const uint32_t word = lds[(uint32_t)p * (uint32_t)L.half + h];
    for (int j = 0; j < nvalid; ++j) a.spins[(size_t)(r0 + j) * n + i] = ((word >> j) & 1u) ? (int8_t)1 : (int8_t)-1;
  }
  const int64_t n_edges = (int64_t)NDIM * L.n;
  for (int j = tid; j < nvalid; j += B) {
    const int r = r0 + j;
    const bool invalid = (extra[64] >> j) & 1u;
    const int64_t h = 2 * (int64_t)extra[32 + j] - n_edges;
    if (a.flips) a.flips[r] = extra[j];
    if (a.energy) a.energy[r] = invalid ? INT64_MIN : h;
    if (a.cut) a.cut[r] = invalid ? INT64_MIN : (a.w_total - h) / 2;
  }
}

}  // namespace

size_t sweep_bp32_lds_bytes(const Lattice& L) { return (size_t)L.n * 5u + kExtraWords * 4u; }

int sweep_bp32_block(const Lattice& L, int requested) {
  if (L.hx > kMaxBlock) return 0;
  int max_lp = kMaxBlock / L.hx;
  if (max_lp > L.lines) max_lp = L.lines;
  int lp = max_lp;
  if (requested > 0) {
    lp = requested / L.hx;
    if (lp < 1) lp = 1;
    if (lp > max_lp) lp = max_lp;
  }
  // per-thread bit-sliced counters: <= 255 site words per sweep (8-bit flip
  // counters) and <= 4095 bonds per window pass (12-bit bond counters)
  const int words = 2 * L.lines;  // site words per thread per sweep when lp = 1
  int min_lp = (words + 254) / 255;
  const int min_lp_e = (words * L.ndim + 4094) / 4095;
  if (min_lp_e > min_lp) min_lp = min_lp_e;
  if (lp < min_lp) lp = min_lp;
  if (lp * L.hx > kMaxBlock) return 0;
  return lp * L.hx;
}

hipError_t launch_sweep_bp32(const ising_graph* g, const SweepLaunch& s, hipStream_t stream) {
  const Lattice& L = g->lat;
  const int block = sweep_bp32_block(L, s.block_threads);
  if (block <= 0) return hipErrorInvalidValue;
  BpArgs a;
  a.lat = L;
  a.wbits = g->d_wbits;
  a.spins = s.spins;
  a.thr = s.d_thr;
  a.cut = s.cut;
  a.energy = s.energy;
  a.flips = s.flips;
  a.stats = s.stats;
  a.seed = s.seed;
  a.w_total = g->w_total;
  a.n_replicas = s.n_replicas;
  a.replica_offset = s.replica_offset;
  a.t_begin = s.t_begin;
  a.t_end = s.t_end;
  a.init = s.init;
  a.lp = block / L.hx;
  // a thread visits 2 ceil(lines / lp) site words per sweep; 8-bit counters
  const int per_sweep = 2 * ((L.lines + a.lp - 1) / a.lp);
  a.flush_every = per_sweep >= 255 ? 1 : 255 / per_sweep;
  const size_t lds = sweep_bp32_lds_bytes(L);
  const int grid = (s.n_replicas + 31) / 32;
  auto go = [&](auto kernel) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, a);
    return hipSuccess;
  };
  const bool fl = s.flips != nullptr, st = s.stats != nullptr;
  hipError_t e;
  if (g->ndim == 2) {
    if (fl)
      e = st ? go(k_sweep_bp32<2, true, true>) : go(k_sweep_bp32<2, true, false>);
    else
      e = st ? go(k_sweep_bp32<2, false, true>) : go(k_sweep_bp32<2, false, false>);
  } else {
    if (fl)
      e = st ? go(k_sweep_bp32<3, true, true>) : go(k_sweep_bp32<3, true, false>);
    else
      e = st ? go(k_sweep_bp32<3, false, true>) : go(k_sweep_bp32<3, false, false>);
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace ising
