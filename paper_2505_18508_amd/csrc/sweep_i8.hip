// Checkerboard Metropolis sweeps, four replicas per 32-bit LDS word.
//
// One block owns one replica quad (replicas 4q .. 4q+3) for a whole window of
// sweeps; the quad's state lives in LDS for the entire window.  Word of site
// (p, h) in colour-split order, byte b = replica 4q + b:
//   bit 7      spin (1: +1, 0: -1)
//   bits 0-3   maintained local field f + deg, f = sum_j w_ij s_j  (0..2 deg)
//   bits 4-6   of bytes 0 and 1: the site's weight signs, direction order
//              +x, -x, +y, -y, +z, -z (bit set: weight -1)
// A sweep (the paper's fundamental step, Section III) visits every colour-0
// site, then every colour-1 site.  A visit computes dE = -2 s_i f_i from the
// field byte; dE <= 0 flips without a draw, dE = 4k > 0 flips iff the Philox
// word of (site, sweep, quad, tag 0) for that replica is below T_k(sweep).
// An accepted flip rewrites the spin bit and adds -2 w_ij s_i(old) to the
// field byte of each neighbour with one packed ds_add_u32 per neighbour (the
// per-byte deltas form one signed integer; every field byte ends inside
// 0..2 deg, so the integer sum is exact whatever the order of the adds).
// Same-colour sites are never neighbours on an even torus, so the result is
// the sequential sweep's, bit for bit.
//
// After the window: spins written back in canonical layout, accepted flips
// per replica, and the energy H = 1/2 sum_i s_i f_i (eq. (2), J = -w, h = 0)
// with cut = (W_total - H) / 2 (eq. (1)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "philox.hpp"

namespace ising {
namespace {

constexpr int kMaxBlock = 1024;
constexpr int kExtraWords = 16;  // [0,4) flips, 4 invalid flags, [8,12) energy sums
constexpr int kLut = 144;        // threshold table entries: (spin bit << 7) | field, field <= 12

struct BatchItem {
  int32_t inst;  // instance
  int32_t r0;    // first local replica of the quad
};

struct I8Args {
  Lattice lat;
  const uint8_t* wbits;
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
  int32_t lp;  // lines per pass: block = hx * lp
};

// Neighbour word indices of colour-p site at (line, y, z, m), and its
// canonical index.  nb[] follows the direction order +x, -x, +y, -y, +z, -z.
template <int NDIM>
struct SiteGeom {
  uint32_t own, ci;
  uint32_t nb[2 * NDIM];
};

template <int NDIM>
__device__ __forceinline__ SiteGeom<NDIM> site_geom(const Lattice& L, int p, uint32_t line, uint32_t y, uint32_t z,
                                                    uint32_t m, uint32_t m_up, uint32_t m_dn) {
  SiteGeom<NDIM> s;
  const uint32_t o = (p + y + z) & 1u;
  const uint32_t hx = (uint32_t)L.hx;
  const uint32_t other = (uint32_t)(1 - p) * (uint32_t)L.half;
  s.own = (uint32_t)p * (uint32_t)L.half + line * hx + m;
  s.ci = line * (uint32_t)L.Lx + 2u * m + o;
  const uint32_t row = other + line * hx;
  s.nb[0] = row + (o ? m_up : m);
  s.nb[1] = row + (o ? m : m_dn);
  const uint32_t Ly = (uint32_t)L.Ly;
  const uint32_t lyp = (y + 1u == Ly) ? line + 1u - Ly : line + 1u;
  const uint32_t lym = (y == 0u) ? line + Ly - 1u : line - 1u;
  s.nb[2] = other + lyp * hx + m;
  s.nb[3] = other + lym * hx + m;
  if (NDIM == 3) {
    const uint32_t Lz = (uint32_t)L.Lz;
    const uint32_t lzp = (z + 1u == Lz) ? line - (Lz - 1u) * Ly : line + Ly;
    const uint32_t lzm = (z == 0u) ? line + (Lz - 1u) * Ly : line - Ly;
    s.nb[2 * NDIM - 2] = other + lzp * hx + m;
    s.nb[2 * NDIM - 1] = other + lzm * hx + m;
  }
  return s;
}

// Threshold for a replica whose field byte, seen from its own spin, is g =
// s f + deg < deg: dE = 2 (deg - g) = 4k with k = (deg - g) / 2.
template <int NDIM>
__device__ __forceinline__ uint32_t thr_for_g(uint32_t g, uint32_t t1, uint32_t t2, uint32_t t3) {
  if (NDIM == 2) return g == 0u ? t2 : t1;
  return g == 0u ? t3 : (g == 2u ? t2 : t1);
}

// One replica quad (local replicas r0 .. r0+3) for the window of a.  Called
// by every thread of a block; lds holds sweep_i8_lds_bytes(a.lat) bytes.
template <int NDIM, bool STATS>
__device__ __forceinline__ void i8_quad(const I8Args& a, const int r0, uint32_t* lds) {
  constexpr int DEG = 2 * NDIM;
  constexpr uint32_t kOnes = 0x01010101u;
  const Lattice& L = a.lat;
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  uint32_t* extra = lds + L.n;

  const int nvalid = min(4, a.n_replicas - r0);
  const uint32_t quad = (uint32_t)(a.replica_offset + r0) >> 2;
  const size_t n = (size_t)L.n;

  for (int k = tid; k < kExtraWords; k += B) extra[k] = 0u;

  // ---- state in: spin bits in colour-split order --------------------------
  uint32_t bad = 0u;
  for (uint32_t i = tid; i < (uint32_t)L.n; i += B) {
    int p;
    uint32_t h;
    site_to_split(L, i, p, h);
    uint32_t word = 0u;
    if (a.init) {
      const u32x4 u = philox_lane_c0(a.seed, i, 0u, quad, kTagInit);
#pragma unroll
      for (int b = 0; b < 4; ++b) word |= (u.v[b] >> 31) << (8 * b + 7);
    } else {
      for (int b = 0; b < nvalid; ++b) {
        const int8_t v = a.spins[(size_t)(r0 + b) * n + i];
        word |= (v > 0 ? 1u : 0u) << (8 * b + 7);
        bad |= (v != 1 && v != -1) ? (1u << b) : 0u;
      }
    }
    lds[(uint32_t)p * (uint32_t)L.half + h] = word;
  }
  __syncthreads();
  if (bad) atomicOr(&extra[4], bad);

  // ---- this thread's sites: fixed m, lines line0, line0 + lp, ... ---------
  const uint32_t hx = (uint32_t)L.hx;
  const uint32_t m = (uint32_t)tid % hx;
  const uint32_t line0 = (uint32_t)tid / hx;
  const uint32_t m_up = (m + 1u == hx) ? 0u : m + 1u;
  const uint32_t m_dn = (m == 0u) ? hx - 1u : m - 1u;
  const uint32_t lp = (uint32_t)a.lp;
  const uint32_t Ly = (uint32_t)L.Ly;
  const uint32_t lp_z = NDIM == 2 ? 0u : lp / Ly;
  const uint32_t lp_y = lp - lp_z * Ly;
  const uint32_t z0 = NDIM == 2 ? 0u : line0 / Ly;
  const uint32_t y0 = line0 - z0 * Ly;
  const bool active = tid < (int)(hx * lp);

  // ---- fields and weight bits ---------------------------------------------
  if (active) {
    for (int p = 0; p < 2; ++p) {
      uint32_t y = y0, z = z0;
      for (uint32_t line = line0; line < (uint32_t)L.lines; line += lp) {
        const SiteGeom<NDIM> s = site_geom<NDIM>(L, p, line, y, z, m, m_up, m_dn);
        const uint32_t wb = a.wbits[s.own];
        uint32_t cnt = 0u;  // per byte: neighbours with w s_j = +1
#pragma unroll
        for (int d = 0; d < DEG; ++d) {
          const uint32_t ns = (lds[s.nb[d]] >> 7) & kOnes;
          cnt += ((wb >> d) & 1u) ? (ns ^ kOnes) : ns;
        }
        // f + deg = 2 cnt; keep spin bits, add field and weight bits
        const uint32_t wordv = (lds[s.own] & 0x80808080u) | (2u * cnt) | ((wb & 7u) << 4) | (((wb >> 3) & 7u) << 12);
        lds[s.own] = wordv;
        y += lp_y;
        z += lp_z;
        if (y >= Ly) {
          y -= Ly;
          z += 1u;
        }
      }
    }
  }
  __syncthreads();

  // ---- the window of sweeps -----------------------------------------------
  // Per-sweep threshold table in LDS, double-buffered: entry (spin bit << 7 |
  // field byte) holds T_k(t) of that state when its dE = 4k > 0, else 0 (a
  // dE <= 0 state flips without a draw).  Sweep t+1's table is written during
  // sweep t's first half; two barriers separate it from its first reader.
  uint32_t* lut = extra + kExtraWords;
  auto fill_lut = [&](uint32_t* dst, int t) {
    const uint32_t* tr = a.thr + (size_t)t * NDIM;
    for (int idx = tid; idx < kLut; idx += B) {
      const uint32_t fb = (uint32_t)idx & 0xFu;
      uint32_t v = 0u;
      // only reachable states: weight bits clear, field even and <= 2 deg
      if ((idx & 0x70) == 0 && (fb & 1u) == 0u && fb <= 2u * DEG) {
        const int g = (idx & 0x80) ? (int)fb : 2 * DEG - (int)fb;  // s f + deg, even, 0..2 deg
        const int k = (DEG - g) / 2;                                 // dE = 4k
        if (k >= 1 && k <= NDIM) v = tr[k - 1];
      }
      dst[idx] = v;
    }
  };
  fill_lut(lut + (a.t_begin & 1) * kLut, a.t_begin);
  __syncthreads();

  // per-thread neighbour offsets (word index deltas, modulo 2^32)
  const uint32_t d_up = m_up - m, d_dn = m_dn - m;
  const uint32_t row = hx, plane = hx * Ly;
  const uint32_t dyp_wrap = row - plane, dym_wrap = plane - row;
  const uint32_t Lz = (uint32_t)L.Lz;
  const uint32_t dzp_wrap = plane - plane * Lz, dzm_wrap = plane * Lz - plane;
  const uint32_t own_step = lp * hx;
  const uint32_t ci_step = lp * (uint32_t)L.Lx;

  uint32_t fl0 = 0u, fl1 = 0u, fl2 = 0u, fl3 = 0u;
  uint32_t n_blocks = 0u, n_draws = 0u;  // RNG statistics (STATS only)
  const uint32_t valid_mask = (1u << nvalid) - 1u;
  constexpr uint32_t kGeBias = (uint32_t)(0x80 - DEG) * kOnes;  // + fb: bit 7 iff fb >= deg
  constexpr uint32_t kLeBias = (uint32_t)(0x80 + DEG) * kOnes;  // - fb: bit 7 iff fb <= deg
  for (int t = a.t_begin; t < a.t_end; ++t) {
    const uint32_t* cur = lut + (t & 1) * kLut;
    uint32_t fc_lo = 0u, fc_hi = 0u;  // flips, packed 16-bit lanes (bytes 0,2 / 1,3)
    for (int p = 0; p < 2; ++p) {
      if (p == 0 && t + 1 < a.t_end) fill_lut(lut + ((t + 1) & 1) * kLut, t + 1);
      uint32_t fc8 = 0u;  // flips this half-sweep, packed bytes
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
          const uint32_t w = lds[own];
          // dE <= 0 per byte: fb >= deg for spin +1, fb <= deg for spin -1
          const uint32_t fb = w & 0x0F0F0F0Fu;
          const uint32_t ge = fb + kGeBias, le = kLeBias - fb;
          const uint32_t acc = ((w & ge) | (~w & le)) & 0x80808080u;
          uint32_t F = acc >> 7;
          const uint32_t T0 = cur[w & 0x8Fu];
          const uint32_t T1 = cur[(w >> 8) & 0x8Fu];
          const uint32_t T2 = cur[(w >> 16) & 0x8Fu];
          const uint32_t T3 = cur[(w >> 24) & 0x8Fu];
          const bool need = (T0 | T1 | T2 | T3) != 0u;
          if (STATS && need) {
            const uint32_t nm = (T0 ? 1u : 0u) | (T1 ? 2u : 0u) | (T2 ? 4u : 0u) | (T3 ? 8u : 0u);
            n_blocks += 1u;
            n_draws += __popc(nm & valid_mask);
          }
          if (need) {
            const u32x4 u = philox_lane_c0(a.seed, ci, (uint32_t)t, quad, kTagMetropolis);
            const uint32_t m4 = (u.v[0] < T0 ? 1u : 0u) | (u.v[1] < T1 ? 2u : 0u) | (u.v[2] < T2 ? 4u : 0u) |
                                (u.v[3] < T3 ? 8u : 0u);
            F |= (m4 * 0x00204081u) & kOnes;  // bit b -> bit 8b
          }
          if (F) {
            lds[own] = w ^ (F << 7);
            // field change of a neighbour over a +1 edge: -2 s_i(old) per flipped byte
            const uint32_t up = (w >> 7) & F;  // flipped bytes whose old spin was +1
            const uint32_t D = 2u * (F - 2u * up);
            const uint32_t wb = ((w >> 4) & 7u) | ((w >> 9) & 0x38u);
#pragma unroll
            for (int d = 0; d < DEG; ++d) atomicAdd(&lds[nb[d]], ((wb >> d) & 1u) ? 0u - D : D);
            fc8 += F;
          }
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
      fc_lo += fc8 & 0x00FF00FFu;
      fc_hi += (fc8 >> 8) & 0x00FF00FFu;
      __syncthreads();
    }
    fl0 += fc_lo & 0xFFFFu;
    fl2 += fc_lo >> 16;
    fl1 += fc_hi & 0xFFFFu;
    fl3 += fc_hi >> 16;
  }

  // ---- energy from the maintained fields ----------------------------------
  constexpr uint32_t kTwoDeg = (uint32_t)(2 * DEG) * kOnes;
  uint32_t e0 = 0u, e1 = 0u, e2 = 0u, e3 = 0u;
  if (active) {
    for (int p = 0; p < 2; ++p) {
      for (uint32_t line = line0; line < (uint32_t)L.lines; line += lp) {
        const uint32_t w = lds[(uint32_t)p * (uint32_t)L.half + line * hx + m];
        const uint32_t fb = w & 0x0F0F0F0Fu;
        const uint32_t spm = (w >> 7) & kOnes;
        const uint32_t negm = (spm ^ kOnes) * 0xFFu;
        const uint32_t g = (fb & ~negm) | ((kTwoDeg - fb) & negm);
        e0 += g & 0xFFu;
        e1 += (g >> 8) & 0xFFu;
        e2 += (g >> 16) & 0xFFu;
        e3 += g >> 24;
      }
    }
    atomicAdd(&extra[0], fl0);
    atomicAdd(&extra[1], fl1);
    atomicAdd(&extra[2], fl2);
    atomicAdd(&extra[3], fl3);
    atomicAdd(&extra[8], e0);
    atomicAdd(&extra[9], e1);
    atomicAdd(&extra[10], e2);
    atomicAdd(&extra[11], e3);
    // per-thread totals go straight to the 64-bit outputs (a block's total can
    // exceed 32 bits)
    if (STATS && (n_blocks | n_draws)) {
      atomicAdd(&a.stats[0], (unsigned long long)n_blocks);
      atomicAdd(&a.stats[1], (unsigned long long)n_draws);
    }
  }
  __syncthreads();

  // ---- state out ----------------------------------------------------------
  for (uint32_t i = tid; i < (uint32_t)L.n; i += B) {
    int p;
    uint32_t h;
    site_to_split(L, i, p, h);
    const uint32_t word = lds[(uint32_t)p * (uint32_t)L.half + h];
    for (int b = 0; b < nvalid; ++b)
      a.spins[(size_t)(r0 + b) * n + i] = ((word >> (8 * b + 7)) & 1u) ? (int8_t)1 : (int8_t)-1;
  }
  for (int b = tid; b < nvalid; b += B) {
    const int r = r0 + b;
    const bool invalid = (extra[4] >> b) & 1u;
    // sum_i (g_i - deg) = sum_i s_i f_i = 2 H
    const int64_t twice_h = (int64_t)extra[8 + b] - (int64_t)DEG * (int64_t)L.n;
    const int64_t h = twice_h / 2;
    if (a.flips) a.flips[r] = extra[b];
    if (a.energy) a.energy[r] = invalid ? INT64_MIN : h;
    if (a.cut) a.cut[r] = invalid ? INT64_MIN : (a.w_total - h) / 2;
  }
}

template <int NDIM, bool STATS>
__global__ void __launch_bounds__(kMaxBlock) k_sweep_i8(I8Args a) {
  extern __shared__ uint32_t lds[];
  i8_quad<NDIM, STATS>(a, blockIdx.x * 4, lds);
}

// Persistent launch over a queue of (instance, quad) items, costliest
// first: each block takes the next item from a global counter until the
// queue is empty, so every block reaches the exit.
template <int NDIM>
__global__ void __launch_bounds__(kMaxBlock) k_sweep_i8_batch(const I8Args* inst, const BatchItem* items, int n_items,
                                                              unsigned int* counter) {
  extern __shared__ uint32_t lds[];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = next;
    __syncthreads();
    if (it >= n_items) break;
    const BatchItem bi = items[it];
    i8_quad<NDIM, false>(inst[bi.inst], bi.r0, lds);
    __syncthreads();
  }
}

__global__ void k_reset_counter(unsigned int* counter) { *counter = 0u; }

}  // namespace

size_t sweep_i8_lds_bytes(const Lattice& L) { return ((size_t)L.n + kExtraWords + 2 * kLut) * 4u; }

int sweep_i8_block(const Lattice& L, int requested) {
  if (L.hx > kMaxBlock) return 0;
  int max_lp = kMaxBlock / L.hx;
  if (max_lp > L.lines) max_lp = L.lines;
  int lp = max_lp;
  if (requested > 0) {
    lp = requested / L.hx;
    if (lp < 1) lp = 1;
    if (lp > max_lp) lp = max_lp;
  }
  // a thread visits ceil(lines / lp) sites per half-sweep; flip counters are
  // packed bytes, so keep that <= 255
  const int min_lp = (L.lines + 254) / 255;
  if (lp < min_lp) lp = min_lp;
  if (lp * L.hx > kMaxBlock) return 0;
  return lp * L.hx;
}

hipError_t launch_sweep_i8(const ising_graph* g, const SweepLaunch& s, hipStream_t stream) {
  const Lattice& L = g->lat;
  const int block = sweep_i8_block(L, s.block_threads);
  if (block <= 0) return hipErrorInvalidValue;
  I8Args a;
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
  const size_t lds = sweep_i8_lds_bytes(L);
  const int grid = (s.n_replicas + 3) / 4;
  auto go = [&](auto kernel) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, a);
    return hipSuccess;
  };
  hipError_t e;
  if (g->ndim == 2)
    e = s.stats ? go(k_sweep_i8<2, true>) : go(k_sweep_i8<2, false>);
  else
    e = s.stats ? go(k_sweep_i8<3, true>) : go(k_sweep_i8<3, false>);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace ising

namespace ising {

hipError_t build_i8_batch(const ising_graph* const* graphs, const SweepLaunch* launches, int n_inst, I8BatchPlan* plan) {
  plan->ndim = graphs[0]->ndim;
  std::vector<I8Args> inst((size_t)n_inst);
  std::vector<std::pair<int64_t, BatchItem>> items;
  size_t lds = 0;
  for (int k = 0; k < n_inst; ++k) {
    const ising_graph* g = graphs[k];
    const SweepLaunch& s = launches[k];
    const Lattice& L = g->lat;
    const int block = sweep_i8_block(L, kMaxBlock);
    if (block <= 0) return hipErrorInvalidValue;
    I8Args& a = inst[(size_t)k];
    a.lat = L;
    a.wbits = g->d_wbits;
    a.spins = s.spins;
    a.thr = s.d_thr;
    a.cut = s.cut;
    a.energy = s.energy;
    a.flips = s.flips;
    a.stats = nullptr;
    a.seed = s.seed;
    a.w_total = g->w_total;
    a.n_replicas = s.n_replicas;
    a.replica_offset = s.replica_offset;
    a.t_begin = s.t_begin;
    a.t_end = s.t_end;
    a.init = s.init;
    a.lp = block / L.hx;
    const size_t b = sweep_i8_lds_bytes(L);
    if (b > lds) lds = b;
    const int64_t cost = (int64_t)L.n * (s.t_end - s.t_begin);
    for (int r0 = 0; r0 < s.n_replicas; r0 += 4) items.push_back({cost * std::min(4, s.n_replicas - r0), BatchItem{k, r0}});
  }
  // costliest first; ties in instance and replica order
  std::stable_sort(items.begin(), items.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  std::vector<BatchItem> order(items.size());
  for (size_t i = 0; i < items.size(); ++i) order[i] = items[i].second;
  plan->n_items = (int)order.size();
  plan->lds = lds;
  plan->block = kMaxBlock;
  const void* kernel = plan->ndim == 2 ? (const void*)k_sweep_i8_batch<2> : (const void*)k_sweep_i8_batch<3>;
  hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0, dev = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kMaxBlock, lds);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  plan->grid = std::min(plan->n_items, per_cu * cus);
  e = hipMalloc(&plan->d_inst, sizeof(I8Args) * (size_t)n_inst);
  if (e == hipSuccess) e = hipMalloc(&plan->d_items, sizeof(BatchItem) * order.size());
  if (e == hipSuccess) e = hipMalloc((void**)&plan->d_counter, sizeof(unsigned int));
  if (e == hipSuccess) e = hipMemcpy(plan->d_inst, inst.data(), sizeof(I8Args) * (size_t)n_inst, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(plan->d_items, order.data(), sizeof(BatchItem) * order.size(), hipMemcpyHostToDevice);
  return e;
}

hipError_t run_i8_batch(const I8BatchPlan& plan, hipStream_t stream) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, stream, plan.d_counter);
  if (plan.ndim == 2)
    hipLaunchKernelGGL(k_sweep_i8_batch<2>, dim3(plan.grid), dim3(plan.block), plan.lds, stream,
                       (const I8Args*)plan.d_inst, (const BatchItem*)plan.d_items, plan.n_items, plan.d_counter);
  else
    hipLaunchKernelGGL(k_sweep_i8_batch<3>, dim3(plan.grid), dim3(plan.block), plan.lds, stream,
                       (const I8Args*)plan.d_inst, (const BatchItem*)plan.d_items, plan.n_items, plan.d_counter);
  return hipGetLastError();
}

void free_i8_batch(I8BatchPlan& plan) {
  (void)hipFree(plan.d_inst);
  (void)hipFree(plan.d_items);
  (void)hipFree(plan.d_counter);
  plan.d_inst = plan.d_items = nullptr;
  plan.d_counter = nullptr;
}

}  // namespace ising
