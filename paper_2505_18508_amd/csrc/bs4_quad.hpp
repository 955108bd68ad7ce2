// Checkerboard Metropolis sweeps, bit-sliced over 4 replicas x 4 sites per
// 16-bit LDS word.
//
// For replica counts too small to fill the chip with 32-replica groups, a
// block owns one replica quad (4q .. 4q+3), as the byte-per-replica kernel
// does, but keeps only spin bits on chip and packs four sites of one colour
// with each replica quad into one 16-bit word, so that the bond logic of a
// visit serves 16 (site, replica) attempts at once.
//
// Word g = gl * hx + m of colour p, gl = z LY4 + Y (LY4 = ceil(Ly / 4) word
// lines per plane), holds the colour-p sites at column m (x = 2m + o) of
// rows y = 4Y .. 4Y + 3 of plane z; bit 4 j + r is the spin (1: +1) of
// replica 4q + r at row 4Y + j.  When Ly = 2 mod 4 (variant PART) the last
// word line of every plane holds two rows: its nibbles 2 and 3 are padding,
// held at 0 and never flipped, and the y neighbours across the wrap are
// shifted in by one nibble instead of three.  LDS holds one record of
// 32-bit entries per g: the colour-0 and colour-1 words, then per colour one
// weight mask per direction slot (nibble j all ones iff that bond of site j
// has weight +1); the record stride is odd, so a wave's records fall in
// distinct banks.  The neighbours of lane (j, r), all in the other colour:
//   x-same   word g, same lane (the x neighbour stored under column m)
//   x-shift  column m + 1 where o = 1, m - 1 where o = 0; o alternates with
//            j, so the two column words are merged by a nibble mask
//   +y, -y   word g shifted by one nibble, the nibble shifted in taken from
//            the next / previous word of the same plane (torus wrap in y)
//   +z, -z   word g of the next / previous plane
// A visit finds the unsatisfied bonds (w s_i s_j = +1) of all 16 lanes with
// one three-way xor per slot, counts them bit-sliced (u = 0..deg) and flips
// lanes with u >= deg/2 (dE <= 0) and lanes with dE = 4k > 0 whose Philox
// word of (site, sweep, quad, tag 0) for that replica is below T_k(sweep)
// (Section III's sweep: colour 0, then colour 1; same-colour sites are never
// neighbours on an even torus, so the result is the sequential sweep's bit
// for bit).
//
// After the window: spins written back in canonical layout, accepted flips
// per replica, and the energy H = sum over colour-0 sites of s_i f_i =
// 2 (unsatisfied bonds at colour-0 sites) - |E| (eq. (2), J = -w, h = 0),
// cut = (W_total - H) / 2 (eq. (1)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bitslice.hpp"
#include "lattice.hpp"
#include "philox.hpp"
#include "reduce.hpp"

namespace ising {
namespace bs4q {

constexpr int kMaxBlock = 1024;
constexpr int kExtraWords = 16;  // [0,4) flips, 4 invalid flags, [8,12) unsatisfied bonds at colour 0

// 32-bit entries per record: 2 spin words + 2 colours x deg weight masks,
// padded to an odd count
template <int NDIM>
constexpr int rec_words() {
  return NDIM == 2 ? 11 : 15;
}

struct Bs4Args {
  Lattice lat;
  const uint8_t* wbits;  // colour-split order, bit d set: weight of direction d (+x,-x,+y,-y,+z,-z) is -1
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
  int32_t lp;  // word lines per pass: block = hx * lp
};

// What one thread needs to walk its words: fixed column m, word lines
// gl0, gl0 + lp, ...; byte offsets between records.
struct Bs4Walk {
  uint32_t base0;          // record of (gl0, m)
  uint32_t du, dd;         // record of column m + 1 / m - 1, relative
  uint32_t step;           // records of lp word lines
  uint32_t row, plane;     // records of one word line / one plane
  uint32_t Y0, z0, lp_y, lp_z, LY4, Lz;
  uint32_t ci0, ci_step;   // canonical index of (first line of word line gl0, x = 2m), per pass
  uint32_t ci_m;           // 2m
  uint32_t GL, gl0, lp;
  // 2-D: word lines visited per half-sweep and, for the first and last
  // visits (only those can wrap), the +-y offsets, the shifts that bring the
  // +y / -y neighbour rows in (12, or 4 across the wrap of a plane whose last
  // word line holds two rows) and the lanes of real sites
  uint32_t nv, dyp_first, dym_first, dyp_last;
  uint32_t shp_first, shm_first, shp_last, rows_first, rows_last;
};

// Unsatisfied bonds of the 16 lanes of a colour-P word, counted bit-sliced:
// u = u0 + 2 u1 + 4 u2.  rd(off) reads the word at byte offset off (modulo
// 2^32) from the word's record; the +y and -y neighbour records are at dyp
// and dym, their rows come in shifted by shp and shm nibble bits (PART; else
// 12), z is the word line's plane.
template <int NDIM, int P, bool PART, class Rd>
__device__ __forceinline__ void bs4_bonds_rd(Rd rd, const Bs4Walk& wk, uint32_t dyp, uint32_t dym, uint32_t shp,
                                             uint32_t shm, uint32_t z, uint32_t& own, uint32_t& u0, uint32_t& u1,
                                             uint32_t& u2) {
  constexpr int DEG = 2 * NDIM;
  constexpr uint32_t O4 = 4u * (1u - (uint32_t)P);
  own = rd(4u * (uint32_t)P);
  const uint32_t xs = rd(O4);
  const uint32_t xu = rd(wk.du + O4);
  const uint32_t xd = rd(wk.dd + O4);
  const uint32_t yn = rd(dyp + O4);
  const uint32_t yv = rd(dym + O4);
  const uint32_t q = ((uint32_t)P + z) & 1u;      // o of the word's first site
  const uint32_t sel = q ? 0x0F0Fu : 0xF0F0u;     // nibbles whose x-shift neighbour is at m + 1
  uint32_t nb[DEG];
  nb[0] = xs;
  nb[1] = (xu & sel) | (xd & ~sel);
  if (PART) {
    // row Ly - 1 is nibble 1 of the last word line, so the wrap shifts by one nibble
    nb[2] = (xs >> 4) | (yn << shp);
    nb[3] = (xs << 4) | (yv >> shm);
  } else {
    nb[2] = (xs >> 4) | (yn << 12);
    nb[3] = (xs << 4) | (yv >> 12);
  }
  if (NDIM == 3) {
    const uint32_t vol = wk.plane * wk.Lz;
    nb[DEG - 2] = rd(((z + 1u == wk.Lz) ? wk.plane - vol : wk.plane) + O4);
    nb[DEG - 1] = rd(((z == 0u) ? vol - wk.plane : 0u - wk.plane) + O4);
  }
  uint32_t x[DEG];
#pragma unroll
  for (int d = 0; d < DEG; ++d) x[d] = xor3(own, nb[d], rd(4u * (2u + (uint32_t)(P * DEG + d))));
  bond_count3<DEG>(x, u0, u1, u2);
}

// The same for the word at record `base` of lds, its y neighbours found
// from its word line Y (wrapping at the plane's ends).
template <int NDIM, int P, bool PART = false>
__device__ __forceinline__ void bs4_bonds(const char* lds, uint32_t base, const Bs4Walk& wk, uint32_t Y, uint32_t z,
                                          uint32_t& own, uint32_t& u0, uint32_t& u1, uint32_t& u2) {
  const uint32_t dyp = (Y + 1u == wk.LY4) ? wk.row - wk.plane : wk.row;
  const uint32_t dym = (Y == 0u) ? wk.plane - wk.row : 0u - wk.row;
  const uint32_t shp = (PART && Y + 1u == wk.LY4) ? 4u : 12u;
  const uint32_t shm = (PART && Y == 0u) ? 4u : 12u;
  auto rd = [&](uint32_t off) { return *(const uint32_t*)(lds + (uint32_t)(base + off)); };
  bs4_bonds_rd<NDIM, P, PART>(rd, wk, dyp, dym, shp, shm, z, own, u0, u1, u2);
}

// Thresholds of the quad's four replicas for one sweep: T[k-1][b] for
// dE = 4k and replica b (equal for all b under a schedule); lev = length of
// the prefix of levels with a nonzero threshold for some replica (thresholds
// decrease with k); m[k-1] = lanes 4 j + b of the replicas with T[k-1][b] != 0.
struct QuadThr {
  uint32_t T[3][4];
  uint32_t m[3];
  int lev;
};

__device__ __forceinline__ void quad_thr_finish(QuadThr& th) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t mk = 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b) mk |= th.T[k][b] ? (0x1111u << b) : 0u;
    th.m[k] = mk;
  }
  th.lev = th.m[0] ? (th.m[1] ? (th.m[2] ? 3 : 2) : 1) : 0;
}

// The draws of a word's four sites and their compares against the first LEV
// thresholds: bit 4 j + r of c_k = (Philox word r of site j) < T_k of
// replica r.  Site j's canonical index: line 4 gl + j, x = 2m + (q ^ (j & 1)).
// PT: one threshold per replica (th); else one for all four (T1, T2, T3).
template <int LEV, bool PT>
__device__ __forceinline__ void bs4_draws(uint64_t seed, uint32_t ci0, uint32_t Lx, uint32_t q, uint32_t t,
                                          uint32_t quad, const QuadThr& th, uint32_t T1, uint32_t T2,
                                          uint32_t T3, uint32_t& c1, uint32_t& c2, uint32_t& c3) {
  // sites 3 and 2, then 1 and 0: two Philox blocks in lockstep, shifted in
  // site 3 (1) before site 2 (0)
#pragma unroll
  for (int j = 3; j >= 1; j -= 2) {
    const uint32_t cia = ci0 + (uint32_t)j * Lx + (q ^ 1u);
    const uint32_t cib = ci0 + (uint32_t)(j - 1) * Lx + q;
    u32x4 ra, rb;
    philox_lane_c0_x2(seed, cia, cib, t, quad, kTagMetropolis, ra, rb);
    // the first compares of the word start the chains
    const uint32_t* t1 = th.T[0];
    const uint32_t* t2 = th.T[1];
    const uint32_t* t3 = th.T[2];
    const uint32_t s1[4] = {T1, T1, T1, T1}, s2[4] = {T2, T2, T2, T2}, s3[4] = {T3, T3, T3, T3};
    if (!PT) {
      t1 = s1;
      t2 = s2;
      t3 = s3;
    }
    if (j == 3)
      lt_shift_in4<LEV, true>(c1, c2, c3, ra.v, t1, t2, t3);
    else
      lt_shift_in4<LEV>(c1, c2, c3, ra.v, t1, t2, t3);
    lt_shift_in4<LEV>(c1, c2, c3, rb.v, t1, t2, t3);
  }
}

// The 16 Philox words of a word's four sites: u[4 j + r] = word r of site j
// (sites 3 and 2, then 1 and 0, two blocks in lockstep).
__device__ __forceinline__ void bs4_words(uint64_t seed, uint32_t ci0, uint32_t Lx, uint32_t q, uint32_t t,
                                          uint32_t quad, uint32_t* u) {
#pragma unroll
  for (int j = 3; j >= 1; j -= 2) {
    u32x4 ra, rb;
    philox_lane_c0_x2(seed, ci0 + (uint32_t)j * Lx + (q ^ 1u), ci0 + (uint32_t)(j - 1) * Lx + q, t, quad,
                      kTagMetropolis, ra, rb);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      u[4 * j + r] = ra.v[r];
      u[4 * (j - 1) + r] = rb.v[r];
    }
  }
}

// Flip mask of a word from its bond counts: dE = 2 deg - 4u, flip when
// u >= deg/2, else k = deg/2 - u and the replica flips iff its draw is below
// T_k.  rows masks the lanes of real sites, q is o of the word's first site.
template <int NDIM, int LEV, bool STATS, bool PT>
__device__ __forceinline__ uint32_t bs4_decide(uint32_t u0, uint32_t u1, uint32_t u2, uint32_t rows, uint32_t q,
                                               uint32_t ci0, uint32_t Lx, const Bs4Args& a, int t, uint32_t quad,
                                               const QuadThr& th, uint32_t T1, uint32_t T2, uint32_t T3,
                                               uint32_t valid16, uint32_t& n_blocks, uint32_t& n_draws) {
  uint32_t acc, k1, k2, k3 = 0u;
  if (NDIM == 2) {
    acc = u1 | u2;
    k1 = u0 & ~acc;
    k2 = ~(u0 | acc);
  } else {
    acc = u2 | (u1 & u0);
    k1 = u1 & ~u0 & ~u2;
    k2 = u0 & ~u1 & ~u2;
    k3 = ~(u0 | u1 | u2);
  }
  if (LEV >= 2) {  // the levels share one chain; each replica's level bits pick its threshold
    const uint32_t need = k1 | k2 | (LEV >= 3 ? k3 : 0u);
    if (STATS) {
      n_blocks += 4u;
      n_draws += __popc(need & valid16 & rows);
    }
    uint32_t u[16];
    bs4_words(a.seed, ci0, Lx, q, (uint32_t)t, quad, u);
    const uint32_t s1[4] = {T1, T1, T1, T1}, s2[4] = {T2, T2, T2, T2}, s3[4] = {T3, T3, T3, T3};
    const uint32_t* t1 = PT ? th.T[0] : s1;
    const uint32_t* t2 = PT ? th.T[1] : s2;
    const uint32_t* t3 = PT ? th.T[2] : s3;
    const uint32_t c = LEV == 2 ? lt_select16(u, k2, t1, t2) : lt_select16_3(u, k2, k3, t1, t2, t3);
    return (acc | (need & c)) & rows;
  }
  uint32_t c1 = 0u, c2 = 0u, c3 = 0u;
  if (LEV > 0) {
    bs4_draws<(LEV > 0 ? LEV : 1), PT>(a.seed, ci0, Lx, q, (uint32_t)t, quad, th, T1, T2, T3, c1, c2, c3);
    if (STATS) {  // schedule only: per-replica thresholds reject statistics
      const uint32_t need = (k1 | (LEV >= 2 ? k2 : 0u) | (LEV >= 3 ? k3 : 0u)) & valid16 & rows;
      n_blocks += 4u;
      n_draws += __popc(need);
    }
  }
  return (acc | (k1 & c1) | (LEV >= 2 ? k2 & c2 : 0u) | (LEV >= 3 ? k3 & c3 : 0u)) & rows;
}

// Accepted flips of a word added to the four replicas' counters (replica b
// owns lanes 4 j + b).
template <bool FLIPS>
__device__ __forceinline__ void bs4_count_flips(uint32_t* fl, uint32_t F) {
  if (FLIPS) {
#pragma unroll
    for (int b = 0; b < 4; ++b) fl[b] += __popc(F & (0x1111u << b));
  }
}

// One half-sweep of colour P over this thread's words, with the first LEV
// threshold levels nonzero (0: no draws at all).  The word is written back
// unconditionally: no thread reads a colour-P word during this half-sweep.
template <int NDIM, int P, int LEV, bool FLIPS, bool STATS, bool PT, bool PART>
__device__ __forceinline__ void bs4_half(char* lds, const Bs4Walk& wk, const Bs4Args& a, int t, uint32_t quad,
                                         const QuadThr& th, uint32_t T1, uint32_t T2, uint32_t T3,
                                         uint32_t valid16, uint32_t* fl, uint32_t& n_blocks,
                                         uint32_t& n_draws) {
  const uint32_t Lx = (uint32_t)a.lat.Lx;
  if (NDIM == 2) {
    // one plane: fixed +-y offsets and shifts on every visit but the first
    // and the last, and the record's LDS byte address kept in a register of
    // its own from visit to visit
    typedef __attribute__((address_space(3))) uint32_t lds_u32;
    uint32_t r = (uint32_t)(uintptr_t)(lds_u32*)(lds + wk.base0);
    uint32_t ci0 = wk.ci0;
    auto visit = [&](uint32_t dyp, uint32_t dym, uint32_t shp, uint32_t shm, uint32_t rows) {
      asm("" : "+v"(r));  // opaque: r stays the induction register the reads use
      auto rd = [&](uint32_t off) { return *(const lds_u32*)(uintptr_t)(r + off); };
      uint32_t s, u0, u1, u2;
      bs4_bonds_rd<NDIM, P, PART>(rd, wk, dyp, dym, shp, shm, 0u, s, u0, u1, u2);
      const uint32_t F = bs4_decide<NDIM, LEV, STATS, PT>(u0, u1, u2, rows, (uint32_t)P, ci0, Lx, a, t, quad, th,
                                                          T1, T2, T3, valid16, n_blocks, n_draws);
      *(lds_u32*)(uintptr_t)(r + 4u * (uint32_t)P) = s ^ F;
      bs4_count_flips<FLIPS>(fl, F);
      r += wk.step;
      ci0 += wk.ci_step;
    };
    if (wk.nv == 0u) return;
    const uint32_t r_last = r + (wk.nv - 1u) * wk.step;  // record of the last visit
    visit(wk.dyp_first, wk.dym_first, wk.shp_first, wk.shm_first, wk.rows_first);
    if (wk.nv >= 2u) {
      while (r != r_last) visit(wk.row, 0u - wk.row, 12u, 12u, 0xFFFFu);
      visit(wk.dyp_last, 0u - wk.row, wk.shp_last, 12u, wk.rows_last);
    }
    return;
  }
  uint32_t base = wk.base0, ci0 = wk.ci0;
  uint32_t Y = wk.Y0, z = wk.z0;
  for (uint32_t gl = wk.gl0; gl < wk.GL; gl += wk.lp) {
    if (NDIM == 2) {  // one plane: the word line is the row, z = 0
      Y = gl;
      z = 0u;
    }
    uint32_t s, u0, u1, u2;
    bs4_bonds<NDIM, P, PART>(lds, base, wk, Y, z, s, u0, u1, u2);
    const uint32_t rows = (PART && Y + 1u == wk.LY4) ? 0x00FFu : 0xFFFFu;  // lanes of real sites
    const uint32_t F = bs4_decide<NDIM, LEV, STATS, PT>(u0, u1, u2, rows, ((uint32_t)P + z) & 1u, ci0, Lx, a, t, quad,
                                                        th, T1, T2, T3, valid16, n_blocks, n_draws);
    ((uint32_t*)(lds + base))[P] = s ^ F;
    bs4_count_flips<FLIPS>(fl, F);
    base += wk.step;
    if (NDIM == 3) {
      Y += wk.lp_y;
      z += wk.lp_z;
      if (Y >= wk.LY4) {
        Y -= wk.LY4;
        z += 1u;
      }
    }
    if (NDIM == 3 && PART)  // planes of Ly = 4 LY4 - 2 lines: the first line of word line (z, Y)
      ci0 = (z * (uint32_t)a.lat.Ly + 4u * Y) * Lx + wk.ci_m;
    else
      ci0 += wk.ci_step;
  }
}

// Sweeps t, t + 1, ... of the window while their number of nonzero levels
// is LEV (under PT the replicas' fixed thresholds: every sweep); returns the
// first sweep not run.  The level is the same for every thread of the block,
// so all of them leave at the same sweep and meet the same barriers.  One
// loop per level keeps the flip counters in the same registers from sweep to
// sweep; they move only where the level changes.
template <int NDIM, int LEV, bool FLIPS, bool STATS, bool PT, bool PART>
__device__ __forceinline__ int bs4_sweeps(int t, bool active, char* lds, const Bs4Walk& wk, const Bs4Args& a,
                                          uint32_t quad, const QuadThr& th, uint32_t valid16, uint32_t* fl,
                                          uint32_t& n_blocks, uint32_t& n_draws) {
  for (; t < a.t_end; ++t) {
    uint32_t T1 = 0u, T2 = 0u, T3 = 0u;
    if (!PT) {
      const uint32_t* tr = a.thr + (size_t)t * NDIM;
      T1 = tr[0];
      T2 = tr[1];
      T3 = NDIM == 3 ? tr[2] : 0u;
      if (sweep_levels<NDIM>(T1, T2, T3) != LEV) break;
    }
    if (active)
      bs4_half<NDIM, 0, LEV, FLIPS, STATS, PT, PART>(lds, wk, a, t, quad, th, T1, T2, T3, valid16, fl, n_blocks,
                                                     n_draws);
    __syncthreads();
    if (active)
      bs4_half<NDIM, 1, LEV, FLIPS, STATS, PT, PART>(lds, wk, a, t, quad, th, T1, T2, T3, valid16, fl, n_blocks,
                                                     n_draws);
    __syncthreads();
  }
  return t;
}

// One replica quad (local replicas r0 .. r0+3) for the window of a.  Called
// by every thread of a block; lds holds sweep_bs4_lds_bytes(a.lat) - 64
// bytes of records and extra kExtraWords words.
// PT: the replicas run at their own fixed temperatures (a.rep_thr) instead
// of the schedule's (a.thr).
// PART: Ly = 2 mod 4 (the last word line of every plane holds two rows).
template <int NDIM, bool FLIPS, bool STATS, bool PT = false, bool PART = false>
__device__ __forceinline__ void bs4_quad(const Bs4Args& a, const int r0, uint32_t* lds, uint32_t* extra) {
  constexpr int DEG = 2 * NDIM;
  constexpr uint32_t RS = (uint32_t)rec_words<NDIM>();
  const Lattice& L = a.lat;
  const uint32_t hx = (uint32_t)L.hx, Ly = (uint32_t)L.Ly, Lz = (uint32_t)L.Lz, Lx = (uint32_t)L.Lx;
  const uint32_t LY4 = (Ly + 3u) / 4u;        // word lines per plane
  const uint32_t GL = LY4 * Lz;                // word lines
  const uint32_t G = GL * hx;                  // records
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  const int nvalid = min(4, a.n_replicas - r0);
  const uint32_t quad = (uint32_t)(a.replica_offset + r0) >> 2;
  const size_t n = (size_t)L.n;

  for (int k = tid; k < kExtraWords; k += B) extra[k] = 0u;

  // ---- state and weight masks in, one record (both colours) per step ----------
  // Every load of a step is issued before any is used: rows past the last
  // valid replica repeat that replica's row and are masked out.
  uint32_t bad = 0u;
  const size_t row[4] = {(size_t)r0 * n, (size_t)(r0 + min(1, nvalid - 1)) * n,
                         (size_t)(r0 + min(2, nvalid - 1)) * n, (size_t)(r0 + min(3, nvalid - 1)) * n};
  for (uint32_t g = tid; g < G; g += B) {
    const uint32_t gl = g / hx, m = g - gl * hx;
    const uint32_t z = gl / LY4;
    uint32_t w0 = 0u, w1 = 0u;  // spin words of colours 0 and 1
    uint32_t wm0[DEG], wm1[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) wm0[d] = wm1[d] = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t y = 4u * (gl - z * LY4) + (uint32_t)j;
      const bool real = !PART || y < Ly;  // else a padding row of a two-row word line
      const uint32_t line = z * Ly + (real ? y : y - 2u);  // padding rows load row y - 2 and drop it
      const uint32_t o0 = (y + z) & 1u;  // colour 0 sits at x = 2m + o0, colour 1 at 2m + 1 - o0
      const uint32_t cb = line * Lx + 2u * m;
      const uint32_t wb0 = real ? a.wbits[line * hx + m] : 0xFFu;
      const uint32_t wb1 = real ? a.wbits[(uint32_t)L.half + line * hx + m] : 0xFFu;
      // direction order -> slot order: x-same is +x at x offset 0, -x at offset 1
      const uint32_t ws0 = o0 ? ((wb0 & ~3u) | ((wb0 & 1u) << 1) | ((wb0 >> 1) & 1u)) : wb0;
      const uint32_t ws1 = o0 ? wb1 : ((wb1 & ~3u) | ((wb1 & 1u) << 1) | ((wb1 >> 1) & 1u));
#pragma unroll
      for (int d = 0; d < DEG; ++d) {
        if (!((ws0 >> d) & 1u)) wm0[d] |= 0xFu << (4 * j);
        if (!((ws1 >> d) & 1u)) wm1[d] |= 0xFu << (4 * j);
      }
      if (a.init) {
        const u32x4 r0v = philox_lane_c0(a.seed, cb + o0, 0u, quad, kTagInit);
        const u32x4 r1v = philox_lane_c0(a.seed, cb + 1u - o0, 0u, quad, kTagInit);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          w0 |= (real ? r0v.v[b] >> 31 : 0u) << (4 * j + b);
          w1 |= (real ? r1v.v[b] >> 31 : 0u) << (4 * j + b);
        }
      } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int8_t ve = a.spins[row[b] + cb], vo = a.spins[row[b] + cb + 1u];  // x = 2m, 2m + 1
          const uint32_t keep = (b < nvalid && real) ? 1u : 0u;
          const uint32_t ue = ve > 0 ? keep : 0u, uo = vo > 0 ? keep : 0u;
          w0 |= (o0 ? uo : ue) << (4 * j + b);
          w1 |= (o0 ? ue : uo) << (4 * j + b);
          const bool off = (ve != 1 && ve != -1) || (vo != 1 && vo != -1);
          bad |= (off && keep) ? (1u << b) : 0u;
        }
      }
    }
    uint32_t* rec = lds + g * RS;
    rec[0] = w0;
    rec[1] = w1;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
      rec[2u + (uint32_t)d] = wm0[d];
      rec[2u + DEG + (uint32_t)d] = wm1[d];
    }
    rec[RS - 1u] = 0u;  // padding entry
  }
  __syncthreads();
  if (bad) atomicOr(&extra[4], bad);

  // ---- this thread's words --------------------------------------------------------
  const uint32_t m = (uint32_t)tid % hx;
  const uint32_t gl0 = (uint32_t)tid / hx;
  const uint32_t m_up = (m + 1u == hx) ? 0u : m + 1u;
  const uint32_t m_dn = (m == 0u) ? hx - 1u : m - 1u;
  const uint32_t lp = (uint32_t)a.lp;
  Bs4Walk wk;
  wk.LY4 = LY4;
  wk.Lz = Lz;
  wk.lp_z = NDIM == 2 ? 0u : lp / LY4;
  wk.lp_y = lp - wk.lp_z * LY4;
  wk.z0 = NDIM == 2 ? 0u : gl0 / LY4;
  wk.Y0 = gl0 - wk.z0 * LY4;
  wk.base0 = (gl0 * hx + m) * RS * 4u;
  wk.du = (m_up - m) * RS * 4u;
  wk.dd = (m_dn - m) * RS * 4u;
  wk.step = lp * hx * RS * 4u;
  wk.row = hx * RS * 4u;
  wk.plane = LY4 * wk.row;
  wk.ci0 = (wk.z0 * Ly + 4u * wk.Y0) * Lx + 2u * m;  // = 4 gl0 Lx + 2m when Ly = 4 LY4
  wk.ci_step = 4u * lp * Lx;
  wk.ci_m = 2u * m;
  wk.GL = GL;
  wk.gl0 = gl0;
  wk.lp = lp;
  wk.nv = gl0 < GL ? (GL - 1u - gl0) / lp + 1u : 0u;
  {
    const uint32_t gl_last = gl0 + (wk.nv > 0u ? wk.nv - 1u : 0u) * lp;  // 2-D: word line = Y
    const bool wrap_p = gl_last + 1u == LY4, wrap_m = gl0 == 0u;
    wk.dyp_last = wrap_p ? wk.row - wk.plane : wk.row;
    wk.shp_last = (PART && wrap_p) ? 4u : 12u;
    wk.rows_last = (PART && wrap_p) ? 0x00FFu : 0xFFFFu;
    wk.dym_first = wrap_m ? wk.plane - wk.row : 0u - wk.row;
    wk.shm_first = (PART && wrap_m) ? 4u : 12u;
    wk.dyp_first = (wk.nv == 1u) ? wk.dyp_last : wk.row;
    wk.shp_first = (wk.nv == 1u) ? wk.shp_last : 12u;
    wk.rows_first = (wk.nv == 1u) ? wk.rows_last : 0xFFFFu;
  }
  const bool active = tid < (int)(hx * lp);
  const uint32_t valid16 = 0x1111u * ((1u << nvalid) - 1u);
  char* lb = (char*)lds;

  uint32_t fl[4] = {0u, 0u, 0u, 0u};
  uint32_t n_blocks = 0u, n_draws = 0u;  // RNG statistics (STATS only)

  QuadThr th{};
  if (PT) {  // each replica at its own temperature for the whole window
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        th.T[k][b] = (k < NDIM && b < nvalid) ? a.rep_thr[(size_t)(r0 + b) * NDIM + k] : 0u;
    quad_thr_finish(th);
  }
  int t = a.t_begin;
  while (t < a.t_end) {
    int lev = th.lev;
    if (!PT) {
      const uint32_t* tr = a.thr + (size_t)t * NDIM;
      lev = sweep_levels<NDIM>(tr[0], tr[1], NDIM == 3 ? tr[2] : 0u);
    }
    if (lev == 0)
      t = bs4_sweeps<NDIM, 0, FLIPS, STATS, PT, PART>(t, active, lb, wk, a, quad, th, valid16, fl, n_blocks, n_draws);
    else if (lev == 1)
      t = bs4_sweeps<NDIM, 1, FLIPS, STATS, PT, PART>(t, active, lb, wk, a, quad, th, valid16, fl, n_blocks, n_draws);
    else if (NDIM == 2 || lev == 2)
      t = bs4_sweeps<NDIM, 2, FLIPS, STATS, PT, PART>(t, active, lb, wk, a, quad, th, valid16, fl, n_blocks, n_draws);
    else
      t = bs4_sweeps<NDIM, 3, FLIPS, STATS, PT, PART>(t, active, lb, wk, a, quad, th, valid16, fl, n_blocks, n_draws);
  }

  // ---- unsatisfied bonds of the colour-0 sites: energy -----------------------
  uint32_t e[4] = {0u, 0u, 0u, 0u};
  if (active) {
    uint32_t base = wk.base0;
    uint32_t Y = wk.Y0, z = wk.z0;
    for (uint32_t gl = gl0; gl < GL; gl += lp) {
      if (NDIM == 2) {
        Y = gl;
        z = 0u;
      }
      uint32_t s, u0, u1, u2;
      bs4_bonds<NDIM, 0, PART>(lb, base, wk, Y, z, s, u0, u1, u2);
      const uint32_t rows = (PART && Y + 1u == LY4) ? 0x00FFu : 0xFFFFu;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t mr = (0x1111u << b) & rows;
        e[b] += __popc(u0 & mr) + 2u * __popc(u1 & mr) + 4u * __popc(u2 & mr);
      }
      base += wk.step;
      if (NDIM == 3) {
        Y += wk.lp_y;
        z += wk.lp_z;
        if (Y >= LY4) {
          Y -= LY4;
          z += 1u;
        }
      }
    }
  }
  // wave totals first, then one atomic per wave and counter
  const bool lane0 = (tid & 63) == 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t es = wave_total(e[b]);
    const uint32_t fs = FLIPS ? wave_total(fl[b]) : 0u;
    if (lane0) {
      atomicAdd(&extra[8 + b], es);
      if (FLIPS) atomicAdd(&extra[b], fs);
    }
  }
  if (STATS) {  // 64-bit: a block's totals can exceed 32 bits
    const uint64_t nb = wave_total((uint64_t)n_blocks), nd = wave_total((uint64_t)n_draws);
    if (lane0 && (nb | nd)) {
      atomicAdd(&a.stats[0], (unsigned long long)nb);
      atomicAdd(&a.stats[1], (unsigned long long)nd);
    }
  }
  __syncthreads();

  // ---- state out, one record (both colours) per step ----------------------------
  for (uint32_t g = tid; g < G; g += B) {
    const uint32_t gl = g / hx, m = g - gl * hx;
    const uint32_t z = gl / LY4;
    const uint32_t w0 = lds[g * RS], w1 = lds[g * RS + 1u];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t y = 4u * (gl - z * LY4) + (uint32_t)j;
      const bool real = !PART || y < Ly;
      const uint32_t line = z * Ly + y;
      const uint32_t o0 = (y + z) & 1u;
      const uint32_t cb = line * Lx + 2u * m;
      const uint32_t we = o0 ? w1 : w0, wo = o0 ? w0 : w1;  // words holding x = 2m and 2m + 1
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (b < nvalid && real) {
          const uint32_t sh = 4u * (uint32_t)j + (uint32_t)b;
          a.spins[row[b] + cb] = ((we >> sh) & 1u) ? (int8_t)1 : (int8_t)-1;
          a.spins[row[b] + cb + 1u] = ((wo >> sh) & 1u) ? (int8_t)1 : (int8_t)-1;
        }
      }
    }
  }
  const int64_t n_edges = (int64_t)NDIM * L.n;
  for (int b = tid; b < nvalid; b += B) {
    const int r = r0 + b;
    const bool invalid = (extra[4] >> b) & 1u;
    const int64_t h = 2 * (int64_t)extra[8 + b] - n_edges;
    if (a.flips) a.flips[r] = extra[b];
    if (a.energy) a.energy[r] = invalid ? INT64_MIN : h;
    if (a.cut) a.cut[r] = invalid ? INT64_MIN : (a.w_total - h) / 2;
  }
}


}  // namespace bs4q
}  // namespace ising
