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
// Philox blocks of a word serve its eight replica quads; the decision and its
// compare chains are shared with the streamed kernel (word32.hpp).  Fields are
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
#include "word32.hpp"

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

// Add two bit vectors at once: a full adder on the lowest plane (sum = xor
// of the three, carry = their majority), then the carry rippled upwards --
// one ripple for two vectors.
template <int NPLANES>
__device__ __forceinline__ void add_planes2(uint32_t* planes, uint32_t a, uint32_t b) {
  uint32_t c[NPLANES];
  c[0] = __builtin_amdgcn_bitop3_b32(planes[0], a, b, 0xE8);  // majority: the carry into plane 1
#pragma unroll
  for (int k = 1; k + 1 < NPLANES; ++k) c[k] = planes[k] & c[k - 1];
  // in place: each plane keeps its register from visit to visit
  asm("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(planes[0]) : "v"(a), "v"(b));
#pragma unroll
  for (int k = 1; k < NPLANES; ++k) asm("v_xor_b32 %0, %0, %1" : "+v"(planes[k]) : "v"(c[k - 1]));
}

// Add four bit vectors at once: two full adders into the lowest plane (their
// carries have weight 2), a third adding both carries into the next plane,
// then its carry rippled upwards -- one ripple for four vectors.
template <int NPLANES>
__device__ __forceinline__ void add_planes4(uint32_t* planes, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  const uint32_t c1 = __builtin_amdgcn_bitop3_b32(planes[0], a, b, 0xE8);  // majority
  asm("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(planes[0]) : "v"(a), "v"(b));
  const uint32_t c2 = __builtin_amdgcn_bitop3_b32(planes[0], c, d, 0xE8);
  asm("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(planes[0]) : "v"(c), "v"(d));
  uint32_t e[NPLANES];
  e[1] = __builtin_amdgcn_bitop3_b32(planes[1], c1, c2, 0xE8);  // carry into plane 2
#pragma unroll
  for (int k = 2; k + 1 < NPLANES; ++k) e[k] = planes[k] & e[k - 1];
  asm("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(planes[1]) : "v"(c1), "v"(c2));
#pragma unroll
  for (int k = 2; k < NPLANES; ++k) asm("v_xor_b32 %0, %0, %1" : "+v"(planes[k]) : "v"(e[k - 1]));
}

// Per-thread constants of the walk over a colour's site words: column m of
// lines line0, line0 + lp, ... (as in the four-replica kernel).
struct BpWalk {
  uint32_t m, line0, lp, hx, Lx, Ly, Lz, half, lines;
  uint32_t lp_y, lp_z, y0, z0;
  uint32_t d_up, d_dn, row, plane, dyp_wrap, dym_wrap, dzp_wrap, dzm_wrap;
  uint32_t own_step, ci_step;
};

// One colour half-sweep of this thread's site words.  EVEN2D: a 2-D torus
// walked with an even number of lines per pass, so every line of the thread
// has the same x parity o and the x-shift neighbour sits at a fixed offset;
// otherwise the general walk (3-D, or an odd pass).  The word is written back
// unconditionally: no other thread reads it during this half-sweep.
template <int NDIM, int LEV, bool SCREEN, bool FLIPS, bool STATS, bool EVEN2D>
__device__ __forceinline__ void bp_half_sweep(uint32_t* lds, const uint8_t* wl, const BpWalk& w, uint32_t p,
                                              uint64_t seed, uint32_t t, uint32_t quad0, uint32_t T1, uint32_t T2,
                                              uint32_t T3, uint32_t valid_lanes, uint32_t* fplanes,
                                              uint32_t& n_words, uint32_t& n_draws) {
  constexpr int DEG = 2 * NDIM;
  const uint32_t other = (1u - 2u * p) * w.half;
  uint32_t own = p * w.half + w.line0 * w.hx + w.m;
  if (EVEN2D) {
    // lines y0, y0 + lp, ... < Ly; only the first (y = 0) and the last
    // (y = Ly - 1) can wrap in y, so those two run with per-lane offsets and
    // the lines between with fixed ones
    const uint32_t o = (p + w.y0) & 1u;
    // x-shift neighbour (+x when o = 1, -x when o = 0) and the weight-sign
    // bits of the shifted and the same-column bonds
    const uint32_t dx = o ? w.d_up : w.d_dn;
    const int bit_shift = o ? 0 : 1, bit_same = 1 - bit_shift;
    uint32_t ci = w.line0 * w.Lx + 2u * w.m + o;
    typedef __attribute__((address_space(3))) uint32_t lds_u32;
    typedef __attribute__((address_space(3))) const uint8_t lds_u8;
    // LDS byte addresses of the own word, its weight byte and the
    // same-column neighbour word, advanced by one pass per visit
    uint32_t a_own = (uint32_t)(uintptr_t)(lds_u32*)(lds + own);
    uint32_t a_wl = (uint32_t)(uintptr_t)(lds_u8*)(wl + own);
    uint32_t a_nb = (uint32_t)(uintptr_t)(lds_u32*)(lds + own + other);
    const uint32_t n_lines = (w.Ly - 1u - w.y0) / w.lp + 1u;  // this thread's lines (y0 < Ly)
    const uint32_t step = w.own_step, step4 = 4u * w.own_step;
    const uint32_t dx4 = 4u * dx;
    auto rd = [](uint32_t a) { return *(const lds_u32*)(uintptr_t)a; };
    auto visit = [&](uint32_t dyp, uint32_t dym) {
      // opaque to the compiler, so each address is its own induction
      // register and a read uses it directly (no base added per read)
      asm volatile("" : "+v"(a_own), "+v"(a_wl), "+v"(a_nb));
      const uint32_t s = rd(a_own);
      const uint32_t wp = *(lds_u8*)(uintptr_t)a_wl;
      uint32_t x[4];
      x[0] = xor3(s, rd(a_nb + dx4), (uint32_t)__builtin_amdgcn_sbfe((int)wp, bit_shift, 1));
      x[1] = xor3(s, rd(a_nb), (uint32_t)__builtin_amdgcn_sbfe((int)wp, bit_same, 1));
      x[2] = xor3(s, rd(a_nb + 4u * dyp), (uint32_t)__builtin_amdgcn_sbfe((int)wp, 2, 1));
      x[3] = xor3(s, rd(a_nb + 4u * dym), (uint32_t)__builtin_amdgcn_sbfe((int)wp, 3, 1));
      const uint32_t F =
          w32_decide<NDIM, LEV, SCREEN, STATS>(x, seed, ci, t, quad0, T1, T2, T3, valid_lanes, n_words, n_draws);
      *(lds_u32*)(uintptr_t)a_own = s ^ F;
      a_own += step4;
      a_wl += step;
      a_nb += step4;
      ci += w.ci_step;
      return F;
    };
    // first line; its flips are counted with the last line's
    const uint32_t F_first = visit(w.y0 + 1u == w.Ly ? w.dyp_wrap : w.row, w.y0 == 0u ? w.dym_wrap : 0u - w.row);
    if (n_lines == 1u) {
      if (FLIPS) add_planes<8>(fplanes, F_first);
      return;
    }
    // middle lines four at a time, their flips added together; then a pair
    // and a single line for what is left
    const uint32_t n_mid = n_lines - 2u;
    for (uint32_t k = 0u; k < n_mid / 4u; ++k) {
      const uint32_t Fa = visit(w.row, 0u - w.row);
      const uint32_t Fb = visit(w.row, 0u - w.row);
      const uint32_t Fc = visit(w.row, 0u - w.row);
      const uint32_t Fd = visit(w.row, 0u - w.row);
      if (FLIPS) add_planes4<8>(fplanes, Fa, Fb, Fc, Fd);
    }
    if (n_mid & 2u) {
      const uint32_t Fa = visit(w.row, 0u - w.row);
      const uint32_t Fb = visit(w.row, 0u - w.row);
      if (FLIPS) add_planes2<8>(fplanes, Fa, Fb);
    }
    if (n_mid & 1u) {
      const uint32_t F = visit(w.row, 0u - w.row);
      if (FLIPS) add_planes<8>(fplanes, F);
    }
    const uint32_t y_last = w.y0 + (n_lines - 1u) * w.lp;
    const uint32_t F_last = visit(y_last + 1u == w.Ly ? w.dyp_wrap : w.row, 0u - w.row);
    if (FLIPS) add_planes2<8>(fplanes, F_first, F_last);
    return;
  }
  uint32_t ci0 = w.line0 * w.Lx + 2u * w.m;
  uint32_t y = w.y0, z = w.z0;
  for (uint32_t line = w.line0; line < w.lines; line += w.lp) {
    const uint32_t o = (p + y + z) & 1u;
    const uint32_t base = own + other;
    uint32_t nb[DEG];
    nb[0] = base + (o ? w.d_up : 0u);
    nb[1] = base + (o ? 0u : w.d_dn);
    nb[2] = base + (y + 1u == w.Ly ? w.dyp_wrap : w.row);
    nb[3] = base + (y == 0u ? w.dym_wrap : 0u - w.row);
    if (NDIM == 3) {
      nb[DEG - 2] = base + (z + 1u == w.Lz ? w.dzp_wrap : w.plane);
      nb[DEG - 1] = base + (z == 0u ? w.dzm_wrap : 0u - w.plane);
    }
    const uint32_t s = lds[own];
    const uint32_t wp = wl[own];
    uint32_t x[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
      // unsatisfied bond: w s_i s_j = +1  <=>  (s_i == s_j) == (w == +1)
      const uint32_t plus = (uint32_t)__builtin_amdgcn_sbfe((int)wp, d, 1);  // all ones iff w = +1
      x[d] = xor3(s, lds[nb[d]], plus);
    }
    const uint32_t F =
        w32_decide<NDIM, LEV, SCREEN, STATS>(x, seed, ci0 + o, t, quad0, T1, T2, T3, valid_lanes, n_words, n_draws);
    lds[own] = s ^ F;
    if (FLIPS) add_planes<8>(fplanes, F);
    own += w.own_step;
    ci0 += w.ci_step;
    y += w.lp_y;
    z += w.lp_z;
    if (y >= w.Ly) {
      y -= w.Ly;
      z += 1u;
    }
  }
}

// Sweeps t, t + 1, ... of the window while their mode (w32_mode: number of
// nonzero threshold levels, screened or not) is 2 LEV + SCREEN; returns the
// first sweep not run.  The mode is the schedule's, the same for every thread
// of the block, so all of them leave at the same sweep and meet the same
// barriers.  One loop per mode keeps the flip-counter planes in the same
// registers from sweep to sweep.
template <int NDIM, int LEV, bool SCREEN, bool FLIPS, bool STATS, bool EVEN2D>
__device__ __forceinline__ int bp_sweeps(int t, const BpArgs& a, bool active, uint32_t* lds, const uint8_t* wl,
                                         const BpWalk& w, uint32_t quad0, uint32_t valid_lanes, uint32_t* fplanes,
                                         uint32_t* extra, int nvalid, uint32_t& n_words, uint32_t& n_draws) {
  for (; t < a.t_end; ++t) {
    const uint32_t* tr = a.thr + (size_t)t * NDIM;
    const uint32_t T1 = tr[0], T2 = tr[1], T3 = NDIM == 3 ? tr[2] : 0u;
    if (w32_mode<NDIM>(T1, T2, T3) != 2 * LEV + (SCREEN ? 1 : 0)) break;
    for (uint32_t p = 0; p < 2u; ++p) {
      if (active)
        bp_half_sweep<NDIM, LEV, SCREEN, FLIPS, STATS, EVEN2D>(lds, wl, w, p, a.seed, (uint32_t)t, quad0, T1, T2, T3,
                                                               valid_lanes, fplanes, n_words, n_draws);
      __syncthreads();
    }
    if (FLIPS && ((t - a.t_begin) % a.flush_every == a.flush_every - 1 || t + 1 == a.t_end))
      flush_planes<8>(fplanes, extra, nvalid);
  }
  return t;
}

template <int NDIM, bool FLIPS, bool STATS, bool EVEN2D>
__device__ __forceinline__ int bp_sweeps_mode(int mode, int t, const BpArgs& a, bool active, uint32_t* lds,
                                              const uint8_t* wl, const BpWalk& w, uint32_t quad0,
                                              uint32_t valid_lanes, uint32_t* fplanes, uint32_t* extra, int nvalid,
                                              uint32_t& n_words, uint32_t& n_draws) {
#define ISING_BP_SWEEPS(LEV, SCREEN)                                                                              \
  bp_sweeps<NDIM, LEV, SCREEN, FLIPS, STATS, EVEN2D>(t, a, active, lds, wl, w, quad0, valid_lanes, fplanes, extra, \
                                                     nvalid, n_words, n_draws)
  // the modes w32_mode returns: 0, 3, 5 and 4 (2-D) or 6, 7 (3-D)
  switch (mode) {
    case 0:
      return ISING_BP_SWEEPS(0, false);
    case 3:
      return ISING_BP_SWEEPS(1, true);
    case 5:
      return ISING_BP_SWEEPS(2, true);
  }
  if constexpr (NDIM == 2) {
    return ISING_BP_SWEEPS(2, false);
  } else {
    if (mode == 6) return ISING_BP_SWEEPS(3, false);
    return ISING_BP_SWEEPS(3, true);
  }
#undef ISING_BP_SWEEPS
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

  // ---- this thread's sites ---------------------------------------------------
  BpWalk w;
  const uint32_t hx = (uint32_t)L.hx;
  w.hx = hx;
  w.Lx = (uint32_t)L.Lx;
  w.half = (uint32_t)L.half;
  w.lines = (uint32_t)L.lines;
  w.m = (uint32_t)tid % hx;
  w.line0 = (uint32_t)tid / hx;
  const uint32_t m_up = (w.m + 1u == hx) ? 0u : w.m + 1u;
  const uint32_t m_dn = (w.m == 0u) ? hx - 1u : w.m - 1u;
  w.lp = (uint32_t)a.lp;
  w.Ly = (uint32_t)L.Ly;
  w.Lz = (uint32_t)L.Lz;
  w.lp_z = NDIM == 2 ? 0u : w.lp / w.Ly;
  w.lp_y = w.lp - w.lp_z * w.Ly;
  w.z0 = NDIM == 2 ? 0u : w.line0 / w.Ly;
  w.y0 = w.line0 - w.z0 * w.Ly;
  const bool active = tid < (int)(hx * w.lp);
  w.d_up = m_up - w.m;
  w.d_dn = m_dn - w.m;
  w.row = hx;
  w.plane = hx * w.Ly;
  w.dyp_wrap = w.row - w.plane;
  w.dym_wrap = w.plane - w.row;
  w.dzp_wrap = w.plane - w.plane * w.Lz;
  w.dzm_wrap = w.plane * w.Lz - w.plane;
  w.own_step = w.lp * hx;
  w.ci_step = w.lp * w.Lx;
  const bool even2d = NDIM == 2 && (w.lp & 1u) == 0u;
  __syncthreads();
  if (bad) atomicOr(&extra[64], bad);

  uint32_t fplanes[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) fplanes[k] = 0u;
  uint32_t n_words = 0u, n_draws = 0u;
  const uint32_t valid_lanes = nvalid == 32 ? 0xFFFFFFFFu : ((1u << nvalid) - 1u);

  int t = a.t_begin;
  while (t < a.t_end) {
    const uint32_t* tr = a.thr + (size_t)t * NDIM;
    const int mode = w32_mode<NDIM>(tr[0], tr[1], NDIM == 3 ? tr[2] : 0u);
    if (even2d)
      t = bp_sweeps_mode<NDIM, FLIPS, STATS, true>(mode, t, a, active, lds, wl, w, quad0, valid_lanes, fplanes, extra,
                                                   nvalid, n_words, n_draws);
    else
      t = bp_sweeps_mode<NDIM, FLIPS, STATS, false>(mode, t, a, active, lds, wl, w, quad0, valid_lanes, fplanes,
                                                    extra, nvalid, n_words, n_draws);
  }

  // ---- unsatisfied bonds along +x, +y (+z): energy ---------------------------
  {
    uint32_t eplanes[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) eplanes[k] = 0u;
    if (active) {
      for (uint32_t p = 0; p < 2u; ++p) {
        const uint32_t other = (1u - 2u * p) * w.half;
        uint32_t own = p * w.half + w.line0 * hx + w.m;
        uint32_t y = w.y0, z = w.z0;
        for (uint32_t line = w.line0; line < w.lines; line += w.lp) {
          const uint32_t o = (p + y + z) & 1u;
          const uint32_t base = own + other;
          const uint32_t s = lds[own];
          const uint32_t wp = wl[own];
          uint32_t e = xor3(s, lds[base + (o ? w.d_up : 0u)], (uint32_t)__builtin_amdgcn_sbfe((int)wp, 0, 1));
          add_planes<12>(eplanes, e);
          e = xor3(s, lds[base + (y + 1u == w.Ly ? w.dyp_wrap : w.row)], (uint32_t)__builtin_amdgcn_sbfe((int)wp, 2, 1));
          add_planes<12>(eplanes, e);
          if (NDIM == 3) {
            e = xor3(s, lds[base + (z + 1u == w.Lz ? w.dzp_wrap : w.plane)],
                     (uint32_t)__builtin_amdgcn_sbfe((int)wp, 4, 1));
            add_planes<12>(eplanes, e);
          }
          own += w.own_step;
          y += w.lp_y;
          z += w.lp_z;
          if (y >= w.Ly) {
            y -= w.Ly;
            z += 1u;
          }
        }
      }
    }
    flush_planes<12>(eplanes, extra + 32, nvalid);
  }
  // 64-bit totals (a block's can exceed 32 bits), one atomic per wave
  if (STATS) {
    // eight Philox blocks per word that drew
    const uint64_t nb = 8ull * wave_total((uint64_t)n_words), nd = wave_total((uint64_t)n_draws);
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
