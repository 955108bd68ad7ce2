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

#include "internal.hpp"
#include "philox.hpp"

namespace ising {
namespace {

constexpr int kMaxBlock = 1024;
constexpr int kExtraWords = 16;  // [0,4) flips, 4 invalid flags, [8,12) energy sums, 12-13 stats

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

template <int NDIM, bool STATS>
__global__ void __launch_bounds__(kMaxBlock) k_sweep_i8(I8Args a) {
  extern __shared__ uint32_t lds[];
  constexpr int DEG = 2 * NDIM;
  constexpr uint32_t kOnes = 0x01010101u;
  const Lattice& L = a.lat;
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  uint32_t* extra = lds + L.n;

  const int r0 = blockIdx.x * 4;                     // first local replica of this quad
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
  uint32_t fl0 = 0u, fl1 = 0u, fl2 = 0u, fl3 = 0u;
  uint32_t n_blocks = 0u, n_draws = 0u;  // RNG statistics (STATS only)
  const uint32_t valid_mask = (1u << nvalid) - 1u;
  constexpr uint32_t kTwoDeg = (uint32_t)(2 * DEG) * kOnes;
  constexpr uint32_t kAccBias = (uint32_t)(0x80 - DEG) * kOnes;
  for (int t = a.t_begin; t < a.t_end; ++t) {
    const uint32_t* tr = a.thr + (size_t)t * NDIM;
    const uint32_t t1 = tr[0], t2 = tr[1], t3 = NDIM == 3 ? tr[2] : 0u;
    uint32_t fc_lo = 0u, fc_hi = 0u;  // packed 16-bit flip counters
    for (int p = 0; p < 2; ++p) {
      if (active) {
        uint32_t y = y0, z = z0;
        for (uint32_t line = line0; line < (uint32_t)L.lines; line += lp) {
          const SiteGeom<NDIM> s = site_geom<NDIM>(L, p, line, y, z, m, m_up, m_dn);
          y += lp_y;
          z += lp_z;
          if (y >= Ly) {
            y -= Ly;
            z += 1u;
          }
          const uint32_t w = lds[s.own];
          const uint32_t fb = w & 0x0F0F0F0Fu;
          const uint32_t spm = (w >> 7) & kOnes;
          const uint32_t negm = (spm ^ kOnes) * 0xFFu;
          const uint32_t g = (fb & ~negm) | ((kTwoDeg - fb) & negm);  // s f + deg per byte
          const uint32_t acc = (g + kAccBias) & 0x80808080u;           // dE <= 0
          uint32_t F = acc >> 7;
          if (acc != 0x80808080u) {
            uint32_t tb[4];
            bool need = false;
            uint32_t need_mask = 0u;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const uint32_t gb = (g >> (8 * b)) & 0xFFu;
              tb[b] = ((acc >> (8 * b + 7)) & 1u) ? 0u : thr_for_g<NDIM>(gb, t1, t2, t3);
              need |= tb[b] != 0u;
              if (STATS) need_mask |= (tb[b] != 0u ? 1u : 0u) << b;
            }
            if (STATS && need) {
              n_blocks += 1u;
              n_draws += __popc(need_mask & valid_mask);
            }
            if (need) {
              const u32x4 u = philox_lane_c0(a.seed, s.ci, (uint32_t)t, quad, kTagMetropolis);
#pragma unroll
              for (int b = 0; b < 4; ++b) F |= (u.v[b] < tb[b] ? 1u : 0u) << (8 * b);
            }
          }
          if (F) {
            lds[s.own] = w ^ (F << 7);
            const uint32_t D = 2u * ((F & ~spm) - (F & spm));
            const uint32_t wb = ((w >> 4) & 7u) | ((w >> 9) & 0x38u);
#pragma unroll
            for (int d = 0; d < DEG; ++d) atomicAdd(&lds[s.nb[d]], ((wb >> d) & 1u) ? 0u - D : D);
            fc_lo += F & 0x00FF00FFu;
            fc_hi += (F >> 8) & 0x00FF00FFu;
          }
        }
      }
      __syncthreads();
    }
    fl0 += fc_lo & 0xFFFFu;
    fl2 += fc_lo >> 16;
    fl1 += fc_hi & 0xFFFFu;
    fl3 += fc_hi >> 16;
  }

  // ---- energy from the maintained fields ----------------------------------
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
    if (STATS) {
      atomicAdd(&extra[12], n_blocks);
      atomicAdd(&extra[13], n_draws);
    }
  }
  __syncthreads();
  if (STATS && tid == 0) {
    atomicAdd(&a.stats[0], (unsigned long long)extra[12]);
    atomicAdd(&a.stats[1], (unsigned long long)extra[13]);
  }

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

}  // namespace

size_t sweep_i8_lds_bytes(const Lattice& L) { return (size_t)L.n * 4u + kExtraWords * 4u; }

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
