// Checkerboard Metropolis sweeps, four replicas per 32-bit LDS word.
//
// One block owns one replica quad (replicas 4q .. 4q+3) for a whole window of
// sweeps; the quad's state lives in LDS for the entire window.  Word of site
// (p, h) in colour-split order, byte b = replica 4q + b:
//   bit 6      spin (1: +1, 0: -1)
//   bits 2-4   maintained count c of neighbours j with w_ij s_j = +1
//              (0..deg), so the local field is f = 2 c - deg
//   bits 0, 1, 5, 7 of byte 0 and bits 0, 1 of byte 1: the site's weight
//              signs (bit set: weight -1) in slot order x-same, x-shift,
//              +y, -y, +z, -z, where x-same is the x neighbour stored under
//              the same column index m in the other colour and x-shift the
//              one at m + 1 or m - 1
// Byte & 0x5C is then directly the byte offset of the replica's entry in the
// per-sweep threshold table (24 words: spin << 4 | c).
//
// A sweep (the paper's fundamental step, Section III) visits every colour-0
// site, then every colour-1 site.  A visit flips a replica whose energy
// change dE = -2 s_i f_i is <= 0, and otherwise flips it iff the Philox word
// of (site, sweep, quad, tag 0) for that replica is below T_k(sweep), dE =
// 4k.  An accepted flip rewrites the spin bit and moves the count of each
// neighbour by -+1 with one packed ds_add_u32 per neighbour (the per-byte
// deltas form one signed integer; every count stays inside 0..deg after each
// add, so the packed sum is exact whatever the order of the adds).
// Same-colour sites are never neighbours on an even torus, so the result is
// the sequential sweep's, bit for bit.
//
// After the window: spins written back in canonical layout, accepted flips
// per replica, and the energy H = 1/2 sum_i s_i f_i (eq. (2), J = -w, h = 0)
// with cut = (W_total - H) / 2 (eq. (1)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"
#include "philox.hpp"
#include "reduce.hpp"

namespace ising {
namespace i8q {

constexpr int kMaxBlock = 1024;
constexpr int kExtraWords = 16;        // [0,4) flips, 4 invalid flags, [8,12) energy sums
constexpr int kSpinBit = 6;
constexpr uint32_t kOnes = 0x01010101u;
constexpr uint32_t kSpin = kOnes << kSpinBit;  // spin bits of the four bytes
constexpr uint32_t kCnt = 0x1C1C1C1Cu;         // neighbour counts, bits 2-4
constexpr uint32_t kLutSel = 0x5C5C5C5Cu;      // spin | count: LUT byte offsets
constexpr int kLutWords = 24;                  // (0x5C >> 2) + 1
// bit of the word holding the weight sign of direction slot d
constexpr int kWPos[6] = {0, 1, 5, 7, 8, 9};
// LDS beside the state words: threshold tables, counters, a queue slot
constexpr int kLutSet = 4 * kLutWords;         // one table per replica byte
constexpr size_t kStaticLds = (2 * kLutSet + kExtraWords + 4) * 4;


struct I8Args {
  Lattice lat;
  const uint8_t* wbits;
  int8_t* spins;
  const uint32_t* thr;      // schedule thresholds [S][NDIM]
  const uint32_t* rep_thr;  // or per-replica fixed thresholds [R][NDIM]
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

// What one thread needs to walk its sites: a fixed column m and the lines
// line0, line0 + lp, ... (byte addresses into the state array).
struct I8Walk {
  uint32_t own0, own1;    // byte address of the first site, colour 0 / 1
  uint32_t odelta0;       // own site -> same-column word of the other colour (colour 0; colour 1: the negation)
  uint32_t ci0;       // canonical index of (line0, column 2m), before + o
  uint32_t y0, z0;
  uint32_t d_up4, d_dn4;        // x-shift neighbour offset when o = 1 / o = 0
  uint32_t dym_first, dyp_last; // 2-D uniform walk: -y offset on the first line, +y on the last
  uint32_t nl;                  // lines this thread visits per half-sweep
};

template <int NDIM>
__device__ __forceinline__ uint32_t slot_weights(uint32_t wb, uint32_t o) {
  // direction order +x, -x, +y, -y, +z, -z -> slot order x-same, x-shift, ...
  const uint32_t ws = o ? ((wb & ~3u) | ((wb & 1u) << 1) | ((wb >> 1) & 1u)) : wb;
  uint32_t v = 0u;
#pragma unroll
  for (int d = 0; d < 2 * NDIM; ++d) v |= ((ws >> d) & 1u) << kWPos[d];
  return v;
}

// One half-sweep of colour p over this thread's sites; returns the accepted
// flips as packed bytes.  BUF selects the threshold buffer, UNIFORM the 2-D
// walk where every thread visits lines / lp lines and o is fixed.
template <int NDIM, bool STATS, int BUF, bool UNIFORM>
__device__ __forceinline__ uint32_t i8_half(const I8Args& a, const I8Walk& wk, uint32_t* lds, const uint32_t* lut,
                                            int p, int t, uint32_t quad, uint32_t valid_mask, uint32_t& n_blocks,
                                            uint32_t& n_draws) {
  constexpr int DEG = 2 * NDIM;
  constexpr uint32_t kGeBias = (uint32_t)((1 << kSpinBit) - 2 * DEG) * kOnes;  // + 4c: spin bit iff c >= deg/2
  constexpr uint32_t kLeBias = (uint32_t)((1 << kSpinBit) + 2 * DEG) * kOnes;  // - 4c: spin bit iff c <= deg/2
  const Lattice& L = a.lat;
  const char* tab = (const char*)(lut + BUF * kLutSet);  // then byte b's table at + 4 b kLutWords bytes
  char* st = (char*)lds;
  const uint32_t hx = (uint32_t)L.hx, Ly = (uint32_t)L.Ly, Lz = (uint32_t)L.Lz;
  const uint32_t lp = (uint32_t)a.lp;
  const uint32_t row4 = 4u * hx, plane4 = 4u * hx * Ly;
  const uint32_t step4 = lp * row4, ci_step = lp * (uint32_t)L.Lx;
  const uint32_t lp_z = NDIM == 2 ? 0u : lp / Ly;
  const uint32_t lp_y = lp - lp_z * Ly;
  const uint32_t od = p ? 0u - wk.odelta0 : wk.odelta0;
  uint32_t own = p ? wk.own1 : wk.own0;
  uint32_t ci = wk.ci0;
  uint32_t y = wk.y0, z = wk.z0;
  uint32_t dsh = 0u;
  if (UNIFORM) {
    const uint32_t o = (p + wk.y0) & 1u;
    ci += o;
    dsh = o ? wk.d_up4 : wk.d_dn4;
  }
  const uint32_t nl = UNIFORM ? (uint32_t)L.lines / lp : wk.nl;
  uint32_t fc8 = 0u;
  for (uint32_t i = 0; i < nl; ++i) {
    uint32_t cie = ci;
    if (!UNIFORM) {
      const uint32_t o = (p + y + z) & 1u;
      cie += o;
      dsh = o ? wk.d_up4 : wk.d_dn4;
    }
    const uint32_t w = *(const uint32_t*)(st + own);
    const uint32_t wm = w & kLutSel;
    const uint32_t T0 = *(const uint32_t*)(tab + (wm & 0xFFu));
    const uint32_t T1 = *(const uint32_t*)(tab + 4 * kLutWords + ((wm >> 8) & 0xFFu));
    const uint32_t T2 = *(const uint32_t*)(tab + 8 * kLutWords + ((wm >> 16) & 0xFFu));
    const uint32_t T3 = *(const uint32_t*)(tab + 12 * kLutWords + (wm >> 24));
    // dE <= 0: c >= deg/2 for spin +1, c <= deg/2 for spin -1
    const uint32_t c4 = w & kCnt;
    const uint32_t ge = c4 + kGeBias, le = kLeBias - c4;
    uint32_t F = ((w & ge) | (~w & le)) & kSpin;
    if (STATS) {
      const uint32_t nm = (T0 ? 1u : 0u) | (T1 ? 2u : 0u) | (T2 ? 4u : 0u) | (T3 ? 8u : 0u);
      n_blocks += nm ? 1u : 0u;
      n_draws += __popc(nm & valid_mask);
    }
    // the word is drawn whether or not a replica needs it: a draw is a pure
    // function of its counter, so skipping it would change nothing else
    const u32x4 u = philox_lane_c0(a.seed, cie, (uint32_t)t, quad, kTagMetropolis);
    F |= (u.v[0] < T0 ? (1u << kSpinBit) : 0u) | (u.v[1] < T1 ? (1u << (kSpinBit + 8)) : 0u) |
         (u.v[2] < T2 ? (1u << (kSpinBit + 16)) : 0u) | (u.v[3] < T3 ? (1u << (kSpinBit + 24)) : 0u);
    if (F) {
      *(uint32_t*)(st + own) = w ^ F;
      const uint32_t F1 = F >> kSpinBit;
      // neighbour count change over a +1 edge: +4 per flipped byte, -8 more
      // where the old spin was +1 (count unit = 4 at bits 2-4)
      const uint32_t D = (F1 << 2) - ((w & F) >> (kSpinBit - 3));
      const uint32_t nD = 0u - D;
      fc8 += F1;
      const uint32_t nbs = own + od;
      uint32_t dyp, dym;
      if (UNIFORM) {
        dym = (i == 0u) ? wk.dym_first : 0u - row4;
        dyp = (i + 1u == nl) ? wk.dyp_last : row4;
      } else {
        dyp = (y + 1u == Ly) ? row4 - plane4 : row4;
        dym = (y == 0u) ? plane4 - row4 : 0u - row4;
      }
      uint32_t addr[DEG];
      addr[0] = nbs;
      addr[1] = nbs + dsh;
      addr[2] = nbs + dyp;
      addr[3] = nbs + dym;
      if (NDIM == 3) {
        addr[DEG - 2] = nbs + ((z + 1u == Lz) ? plane4 - Lz * plane4 : plane4);
        addr[DEG - 1] = nbs + ((z == 0u) ? Lz * plane4 - plane4 : 0u - plane4);
      }
#pragma unroll
      for (int d = 0; d < DEG; ++d) {
        const uint32_t neg = (uint32_t)__builtin_amdgcn_sbfe((int32_t)w, kWPos[d], 1);  // all ones iff w = -1
        atomicAdd((uint32_t*)(st + addr[d]), __builtin_amdgcn_bitop3_b32(neg, nD, D, 0xCA));  // neg ? nD : D
      }
    }
    own += step4;
    ci += ci_step;
    if (!UNIFORM) {
      y += lp_y;
      z += lp_z;
      if (y >= Ly) {
        y -= Ly;
        z += 1u;
      }
    }
  }
  return fc8;
}

// One replica quad (local replicas r0 .. r0+3) for the window of a.  Called
// by every thread of a block; lds holds the n state words, lut 2 kLutSet
// threshold words and extra kExtraWords words.
template <int NDIM, bool STATS>
__device__ __forceinline__ void i8_quad(const I8Args& a, const int r0, uint32_t* lds, uint32_t* lut,
                                        uint32_t* extra) {
  constexpr int DEG = 2 * NDIM;
  const Lattice& L = a.lat;
  const int tid = threadIdx.x;
  const int B = blockDim.x;

  const int nvalid = min(4, a.n_replicas - r0);
  const uint32_t quad = (uint32_t)(a.replica_offset + r0) >> 2;
  const size_t n = (size_t)L.n;

  for (int k = tid; k < kExtraWords; k += B) extra[k] = 0u;

  // ---- state in: spin bits in colour-split order --------------------------
  // Two sites per step and every replica row loaded before any is used: rows
  // past the last valid replica repeat that replica's row and are masked out.
  uint32_t bad = 0u;
  const size_t row[4] = {(size_t)r0 * n, (size_t)(r0 + min(1, nvalid - 1)) * n,
                         (size_t)(r0 + min(2, nvalid - 1)) * n, (size_t)(r0 + min(3, nvalid - 1)) * n};
  const uint32_t nn = (uint32_t)L.n;
  for (uint32_t i0 = tid; i0 < nn; i0 += 2u * (uint32_t)B) {
    const uint32_t i1 = i0 + (uint32_t)B;
    const bool has1 = i1 < nn;
    const uint32_t ii[2] = {i0, has1 ? i1 : i0};
    uint32_t word[2] = {0u, 0u};
    if (a.init) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const u32x4 u = philox_lane_c0(a.seed, ii[e], 0u, quad, kTagInit);
#pragma unroll
        for (int b = 0; b < 4; ++b) word[e] |= (u.v[b] >> 31) << (8 * b + kSpinBit);
      }
    } else {
      int8_t v[2][4];
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int b = 0; b < 4; ++b) v[e][b] = a.spins[row[b] + ii[e]];
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const bool keep = b < nvalid;
          word[e] |= (keep && v[e][b] > 0 ? 1u : 0u) << (8 * b + kSpinBit);
          bad |= (keep && v[e][b] != 1 && v[e][b] != -1) ? (1u << b) : 0u;
        }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (e == 0 || has1) {
        int p;
        uint32_t h;
        site_to_split(L, ii[e], p, h);
        lds[(uint32_t)p * (uint32_t)L.half + h] = word[e];
      }
    }
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

  // ---- counts and weight bits ---------------------------------------------
  if (active) {
    for (int p = 0; p < 2; ++p) {
      uint32_t y = y0, z = z0;
      for (uint32_t line = line0; line < (uint32_t)L.lines; line += lp) {
        const SiteGeom<NDIM> s = site_geom<NDIM>(L, p, line, y, z, m, m_up, m_dn);
        const uint32_t wb = a.wbits[s.own];
        uint32_t cnt = 0u;  // per byte: neighbours with w s_j = +1
#pragma unroll
        for (int d = 0; d < DEG; ++d) {
          const uint32_t ns = (lds[s.nb[d]] >> kSpinBit) & kOnes;
          cnt += ((wb >> d) & 1u) ? (ns ^ kOnes) : ns;
        }
        const uint32_t o = (p + y + z) & 1u;
        lds[s.own] = (lds[s.own] & kSpin) | (cnt << 2) | slot_weights<NDIM>(wb, o);
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
  // Per-sweep threshold tables, one per replica byte, double-buffered: entry
  // spin << 4 | c of byte b's table holds that replica's T_k(t) when the
  // state's dE = 4k > 0, else 0 (a dE <= 0 state flips without a draw).
  // Under a schedule the four tables are equal; with per-replica fixed
  // thresholds they differ and do not change.  Sweep t+1's tables are
  // written during sweep t's first half; two barriers separate them from
  // their first reader.
  auto fill_lut = [&](uint32_t* dst, int t) {
    for (int idx = tid; idx < kLutSet; idx += B) {
      const int b = idx / kLutWords, e = idx - b * kLutWords;
      const uint32_t* tr = a.rep_thr ? a.rep_thr + (size_t)(r0 + min(b, nvalid - 1)) * NDIM
                                     : a.thr + (size_t)t * NDIM;
      uint32_t v = 0u;
      const int c = e & 7;
      if ((e & 8) == 0 && c <= DEG) {
        const int k = (e & 16) ? NDIM - c : c - NDIM;  // dE = 4k
        if (k >= 1 && k <= NDIM) v = tr[k - 1];
      }
      dst[idx] = v;
    }
  };
  fill_lut(lut + (a.t_begin & 1) * kLutSet, a.t_begin);
  __syncthreads();

  I8Walk wk;
  const uint32_t half4 = 4u * (uint32_t)L.half;
  wk.own0 = 4u * (line0 * hx + m);
  wk.own1 = half4 + wk.own0;
  wk.odelta0 = half4;
  wk.ci0 = line0 * (uint32_t)L.Lx + 2u * m;
  wk.y0 = y0;
  wk.z0 = z0;
  wk.d_up4 = 4u * (m_up - m);
  wk.d_dn4 = 4u * (m_dn - m);
  const uint32_t row4 = 4u * hx, plane4 = row4 * Ly;
  wk.nl = line0 < (uint32_t)L.lines ? ((uint32_t)L.lines - 1u - line0) / lp + 1u : 0u;
  wk.dym_first = (line0 == 0u) ? plane4 - row4 : 0u - row4;
  wk.dyp_last = (line0 + (wk.nl - 1u) * lp + 1u == Ly) ? row4 - plane4 : row4;
  // 2-D, lp even and dividing the lines: every thread walks the same number
  // of lines and keeps its x parity o, so the walk needs no per-line tests
  const bool uniform = NDIM == 2 && (lp & 1u) == 0u && (uint32_t)L.lines % lp == 0u;

  uint32_t fl0 = 0u, fl1 = 0u, fl2 = 0u, fl3 = 0u;
  uint32_t n_blocks = 0u, n_draws = 0u;  // RNG statistics (STATS only)
  const uint32_t valid_mask = (1u << nvalid) - 1u;
  for (int t = a.t_begin; t < a.t_end; ++t) {
    uint32_t fc_lo = 0u, fc_hi = 0u;  // flips, packed 16-bit lanes (bytes 0,2 / 1,3)
    for (int p = 0; p < 2; ++p) {
      if (p == 0 && t + 1 < a.t_end) fill_lut(lut + ((t + 1) & 1) * kLutSet, t + 1);
      uint32_t fc8 = 0u;  // flips this half-sweep, packed bytes
      if (active) {
        if constexpr (NDIM == 2) {
          if (uniform) {
            fc8 = (t & 1) ? i8_half<NDIM, STATS, 1, true>(a, wk, lds, lut, p, t, quad, valid_mask, n_blocks, n_draws)
                          : i8_half<NDIM, STATS, 0, true>(a, wk, lds, lut, p, t, quad, valid_mask, n_blocks, n_draws);
          } else {
            fc8 = (t & 1) ? i8_half<NDIM, STATS, 1, false>(a, wk, lds, lut, p, t, quad, valid_mask, n_blocks, n_draws)
                          : i8_half<NDIM, STATS, 0, false>(a, wk, lds, lut, p, t, quad, valid_mask, n_blocks, n_draws);
          }
        } else {
          fc8 = (t & 1) ? i8_half<NDIM, STATS, 1, false>(a, wk, lds, lut, p, t, quad, valid_mask, n_blocks, n_draws)
                        : i8_half<NDIM, STATS, 0, false>(a, wk, lds, lut, p, t, quad, valid_mask, n_blocks, n_draws);
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

  // ---- energy from the maintained counts ----------------------------------
  // per byte e = c for spin +1, deg - c for spin -1, so s f = 2 e - deg
  constexpr uint32_t kDeg = (uint32_t)DEG * kOnes;
  uint32_t e0 = 0u, e1 = 0u, e2 = 0u, e3 = 0u;
  if (active) {
    for (int p = 0; p < 2; ++p) {
      for (uint32_t line = line0; line < (uint32_t)L.lines; line += lp) {
        const uint32_t w = lds[(uint32_t)p * (uint32_t)L.half + line * hx + m];
        const uint32_t c = (w >> 2) & 0x07070707u;
        const uint32_t down = (((w >> kSpinBit) & kOnes) ^ kOnes) * 0xFFu;  // 0xFF where spin -1
        const uint32_t g = (c & ~down) | ((kDeg - c) & down);
        e0 += g & 0xFFu;
        e1 += (g >> 8) & 0xFFu;
        e2 += (g >> 16) & 0xFFu;
        e3 += g >> 24;
      }
    }
  }
  // wave totals first, then one atomic per wave and counter
  {
    const uint32_t v[8] = {fl0, fl1, fl2, fl3, e0, e1, e2, e3};
    const int slot[8] = {0, 1, 2, 3, 8, 9, 10, 11};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t s = wave_total(v[k]);
      if ((tid & 63) == 0) atomicAdd(&extra[slot[k]], s);
    }
  }
  if (STATS) {  // 64-bit: a block's totals can exceed 32 bits
    const uint64_t nb = wave_total((uint64_t)n_blocks), nd = wave_total((uint64_t)n_draws);
    if ((tid & 63) == 0 && (nb | nd)) {
      atomicAdd(&a.stats[0], (unsigned long long)nb);
      atomicAdd(&a.stats[1], (unsigned long long)nd);
    }
  }
  __syncthreads();

  // ---- state out ----------------------------------------------------------
  for (uint32_t i = tid; i < (uint32_t)L.n; i += B) {
    int p;
    uint32_t h;
    site_to_split(L, i, p, h);
    const uint32_t word = lds[(uint32_t)p * (uint32_t)L.half + h];
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (b < nvalid) a.spins[row[b] + i] = ((word >> (8 * b + kSpinBit)) & 1u) ? (int8_t)1 : (int8_t)-1;
  }
  for (int b = tid; b < nvalid; b += B) {
    const int r = r0 + b;
    const bool invalid = (extra[4] >> b) & 1u;
    // sum_i s_i f_i = 2 sum_i e_i - deg n = 2 H
    const int64_t h = (int64_t)extra[8 + b] - (int64_t)NDIM * (int64_t)L.n;
    if (a.flips) a.flips[r] = extra[b];
    if (a.energy) a.energy[r] = invalid ? INT64_MIN : h;
    if (a.cut) a.cut[r] = invalid ? INT64_MIN : (a.w_total - h) / 2;
  }
}

}  // namespace i8q
}  // namespace ising
