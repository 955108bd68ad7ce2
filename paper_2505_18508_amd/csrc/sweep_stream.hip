// Checkerboard Metropolis sweeps for lattices too large for one block's LDS:
// 32 replicas per 32-bit word (as the on-chip bit-packed kernel), state in
// HBM, one launch per colour half-sweep.  A colour-p launch only reads
// colour-(1-p) words and only writes colour-p words, so the launch boundary
// is the only synchronisation the checkerboard needs, and the result is the
// sequential sweep's bit for bit.
//
// State: words [group][2][n/2] in colour-split order (word bit j = spin of
// replica 32 g + j).  Per half-sweep a word costs its own read and write and
// the reads of its neighbours' words (12 bytes per word per sweep, 0.375
// bytes per spin-update attempt).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bitslice.hpp"
#include "internal.hpp"
#include "philox.hpp"
#include "word32.hpp"

namespace ising {
namespace {

constexpr int kStreamBlock = 256;

struct StreamArgs {
  Lattice lat;
  const uint8_t* wbits;  // colour-split, bit d set: weight of direction d is -1
  uint32_t* words;       // [groups][n]
  const uint32_t* thr;
  uint32_t* part;        // [groups][blocks_x][32] block-owned flip counts, or null
  unsigned long long* spart;  // [groups][blocks_x][2] block-owned RNG counts (STATS)
  uint64_t seed;
  int32_t n_replicas, replica_offset, groups;
  FastDiv div_hx;  // division by the words per line of one colour
  FastDiv div_bx;  // division by the blocks per replica group (gridDim.x)
};

// One stage of a 32 x 32 bit transpose across the 32 lanes of a half-wave
// (row = lane, column = bit), the partner being lane ^ J: a lane whose bit J
// is clear keeps the low J-bit half of every 2J-bit block and takes the
// partner's low halves into its high halves; a lane whose bit J is set keeps
// its high halves and takes the partner's high halves into its low halves.
// m = the low halves of the 2J-bit blocks.  After the stages J = 16, 8, 4,
// 2, 1, bit k of lane j holds what bit j of lane k held.
template <int J>
__device__ __forceinline__ uint32_t transpose_stage(uint32_t x, uint32_t lane, uint32_t m) {
  const uint32_t y = (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x1F | (J << 10));  // lane ^ J within 32
  const uint32_t lo = (x & m) | ((y << J) & ~m);
  const uint32_t hi = (x & ~m) | ((y >> J) & m);
  const uint32_t upper = 0u - ((lane / (uint32_t)J) & 1u);  // all ones where lane bit J is set
  return (hi & upper) | (lo & ~upper);                    // select without a branch
}

// A thread's strip: column m of K consecutive lines l0 .. l0+K-1 of one
// plane (fewer for the last strip of a 2-D torus).  Going up the strip, the
// other colour's word of the line just visited becomes the next line's -y
// neighbour and its +y neighbour becomes the next line's same-column
// neighbour, so a visit loads its own word, its weight signs, the x-shift
// and +y neighbours (and, in 3-D, the +-z ones).  Flips are added into
// bit-sliced counters fp[0..NP) (count = sum 2^b fp[b]).
template <int NDIM, bool STATS, int K, int LEV, bool SCREEN, int NP>
__device__ __forceinline__ void stream_strip(const StreamArgs& a, uint32_t* w, int p, uint32_t t, uint32_t strip,
                                             uint32_t m, uint32_t quad0, uint32_t lanes, uint32_t T1, uint32_t T2,
                                             uint32_t T3, uint32_t* fp, uint32_t& n_words, uint32_t& n_draws) {
  constexpr int DEG = 2 * NDIM;
  const Lattice& L = a.lat;
  const uint32_t hx = (uint32_t)L.hx, Ly = (uint32_t)L.Ly, Lz = (uint32_t)L.Lz, Lx = (uint32_t)L.Lx;
  const uint32_t lines = (uint32_t)L.lines, half = (uint32_t)L.half;
  const uint32_t plane = hx * Ly;
  const uint32_t l0 = strip * (uint32_t)K;
  const uint32_t z = NDIM == 2 ? 0u : fdiv(l0, L.div_ly);
  uint32_t y = l0 - z * Ly;
  const uint32_t m_up = (m + 1u == hx) ? 0u : m + 1u;
  const uint32_t m_dn = (m == 0u) ? hx - 1u : m - 1u;
  uint32_t own = (uint32_t)p * half + l0 * hx + m;
  uint32_t oth = (uint32_t)(1 - p) * half + l0 * hx;  // the other colour's words of line l0
  uint32_t omask = 0u - (((uint32_t)p + y + z) & 1u);  // all ones where x = 2m + 1 (o = 1)
  uint32_t ci = l0 * Lx + 2u * m + (omask & 1u);
  // z neighbours: same offsets for every line of the strip (one plane)
  const uint32_t dzp = (z + 1u == Lz) ? 0u - (Lz - 1u) * plane : plane;
  const uint32_t dzm = (z == 0u) ? (Lz - 1u) * plane : 0u - plane;
  uint32_t ym = w[oth + (y == 0u ? plane - hx : 0u - hx) + m];
  uint32_t x0 = w[oth + m];
  // the loads of line k + 1 are issued before line k is decided (software
  // pipelining): they touch the other colour's words, which this launch
  // never writes, and the next own word, which line k does not write
  auto load_line = [&](uint32_t o_own, uint32_t o_oth, uint32_t yy, uint32_t om, uint32_t* v) {
    v[0] = w[o_oth + (yy + 1u == Ly ? 0u - (Ly - 1u) * hx : hx) + m];  // +y
    v[1] = w[o_oth + (om ? m_up : m_dn)];                               // x-shift
    v[2] = w[o_own];                                                    // own word
    v[3] = a.wbits[o_own];                                              // weight signs
    if (NDIM == 3) {
      v[4] = w[o_oth + dzp + m];
      v[5] = w[o_oth + dzm + m];
    }
  };
  uint32_t cur[6], nxt[6];
  uint32_t Fk[K];  // accepted flips of each line of the strip (0 past the lattice's last line)
#pragma unroll
  for (int k = 0; k < K; ++k) Fk[k] = 0u;
  load_line(own, oth, y, omask, cur);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (l0 + (uint32_t)k >= lines) break;
    const bool more = k + 1 < K && l0 + (uint32_t)k + 1u < lines;
    if (more) load_line(own + hx, oth + hx, y + 1u, ~omask, nxt);
    const uint32_t yp = cur[0], xs = cur[1], s = cur[2], wb = cur[3];
    uint32_t nb[DEG];
    nb[0] = (omask & xs) | (~omask & x0);  // +x: column m + 1 where o = 1, m where o = 0
    nb[1] = (omask & x0) | (~omask & xs);  // -x
    nb[2] = yp;
    nb[3] = ym;
    if (NDIM == 3) {
      nb[DEG - 2] = cur[4];
      nb[DEG - 1] = cur[5];
    }
    uint32_t x[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
      const uint32_t plus = ((wb >> d) & 1u) ? 0u : 0xFFFFFFFFu;  // all ones iff w = +1
      x[d] = xor3(s, nb[d], plus);                                // unsatisfied bonds
    }
    const uint32_t F =
        w32_decide<NDIM, LEV, SCREEN, STATS>(x, a.seed, ci, t, quad0, T1, T2, T3, lanes, n_words, n_draws);
    w[own] = s ^ F;
    Fk[k] = F;
    ym = x0;
    x0 = yp;
    own += hx;
    oth += hx;
    y += 1u;
    omask = ~omask;
    ci += Lx + ((omask & 2u) - 1u);  // next line, x parity flipped: +Lx +1 if o becomes 1, +Lx -1 if 0
#pragma unroll
    for (int e = 0; e < 6; ++e) cur[e] = nxt[e];
  }
  // the strip's flips per replica, bit-sliced (fp starts at zero: one strip
  // per thread and launch)
  if constexpr (K == 1) {
    fp[0] = Fk[0];
  } else if constexpr (K == 2) {
    fp[0] = Fk[0] ^ Fk[1];
    fp[1] = Fk[0] & Fk[1];
  } else if constexpr (K == 4) {
    bond_count3<4>(Fk, fp[0], fp[1], fp[2]);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      uint32_t c = Fk[k];
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        const uint32_t carry = fp[b] & c;
        fp[b] ^= c;
        c = carry;
      }
    }
  }
}

// One launch per colour half-sweep.  Each thread walks a strip of K lines
// (stream_strip); blocks are taken in an XCD-aware order.
template <int NDIM, bool STATS, int K>
__global__ void __launch_bounds__(kStreamBlock) k_halfsweep_stream(StreamArgs a, int p, int t) {
  constexpr int NP = K <= 1 ? 1 : K <= 3 ? 2 : 3;  // planes of a count up to K
  const Lattice& L = a.lat;
  // The dispatcher deals consecutive blocks to the 8 XCDs in turn; the blocks
  // one XCD receives take consecutive logical indices, so the strips that
  // share rows of words (neighbouring lines and columns) meet in one L2.
  const uint32_t nblk = gridDim.x * gridDim.y;
  const uint32_t lin = blockIdx.x + blockIdx.y * gridDim.x;
  const uint32_t per = nblk / 8u, rem = nblk % 8u, xcd = lin % 8u;
  const uint32_t logical = xcd * per + (xcd < rem ? xcd : rem) + lin / 8u;
  const int g = (int)fdiv(logical, a.div_bx);
  const uint32_t bx = logical - (uint32_t)g * gridDim.x;
  const uint32_t hx = (uint32_t)L.hx;
  const uint32_t n_items = hx * (((uint32_t)L.lines + (uint32_t)K - 1u) / (uint32_t)K);
  const uint32_t item = bx * kStreamBlock + threadIdx.x;
  const int r0 = 32 * g;
  const int nvalid = min(32, a.n_replicas - r0);
  const uint32_t lanes = nvalid == 32 ? 0xFFFFFFFFu : ((1u << nvalid) - 1u);
  const uint32_t* tr = a.thr + (size_t)t * NDIM;
  const uint32_t T1 = tr[0], T2 = tr[1], T3 = NDIM == 3 ? tr[2] : 0u;
  const int mode = w32_mode<NDIM>(T1, T2, T3);
  uint32_t fp[NP];
#pragma unroll
  for (int b = 0; b < NP; ++b) fp[b] = 0u;
  uint32_t n_words = 0u, n_draws = 0u;
  if (item < n_items) {
    const uint32_t strip = fdiv(item, a.div_hx);
    const uint32_t m = item - strip * hx;
    uint32_t* w = a.words + (size_t)g * L.n;
    const uint32_t quad0 = (uint32_t)(a.replica_offset + r0) >> 2;
#define ISING_STRIP(LEV, SCREEN)                                                                                 \
  stream_strip<NDIM, STATS, K, LEV, SCREEN, NP>(a, w, p, (uint32_t)t, strip, m, quad0, lanes, T1, T2, T3, fp, \
                                                n_words, n_draws)
    // the modes w32_mode returns: 0, 3, 5 and 4 (2-D) or 6, 7 (3-D)
    if (mode == 0) {
      ISING_STRIP(0, false);
    } else if (mode == 3) {
      ISING_STRIP(1, true);
    } else if (mode == 5) {
      ISING_STRIP(2, true);
    } else if constexpr (NDIM == 2) {
      ISING_STRIP(2, false);
    } else if (mode == 6) {
      ISING_STRIP(3, false);
    } else {
      ISING_STRIP(3, true);
    }
#undef ISING_STRIP
  }
  if (STATS) {  // block totals of Philox blocks (8 per word that drew) and draws, kept in the block's slot
    __shared__ uint32_t ws[kStreamBlock / 64][2];
    uint32_t d = n_draws, nw = n_words;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      d += __shfl_xor(d, off, 64);
      nw += __shfl_xor(nw, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      ws[threadIdx.x >> 6][0] = nw;
      ws[threadIdx.x >> 6][1] = d;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      unsigned long long c = 0ull;
#pragma unroll
      for (int k = 0; k < kStreamBlock / 64; ++k) c += ws[k][threadIdx.x];
      if (threadIdx.x == 0) c *= 8ull;
      a.spart[((size_t)g * gridDim.x + bx) * 2 + threadIdx.x] += c;
    }
  }
  // flips per replica: transposing the 32 x 32 bit matrix of each half-wave
  // (row = lane, column = replica bit) of every counter plane leaves in lane j
  // the half-wave's counts of replica j; the block adds its half-waves and
  // keeps a running total in its own slot (the same logical block owns the
  // same slot in every launch: no atomics)
  if (a.part) {
    __shared__ uint32_t wc[kStreamBlock / 32][32];
    const uint32_t lane = threadIdx.x & 31u;
    uint32_t cnt = 0u;
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      uint32_t x = fp[b];
      x = transpose_stage<16>(x, lane, 0x0000FFFFu);
      x = transpose_stage<8>(x, lane, 0x00FF00FFu);
      x = transpose_stage<4>(x, lane, 0x0F0F0F0Fu);
      x = transpose_stage<2>(x, lane, 0x33333333u);
      x = transpose_stage<1>(x, lane, 0x55555555u);
      cnt += (uint32_t)__popc(x) << b;
    }
    wc[threadIdx.x >> 5][lane] = cnt;
    __syncthreads();
    if (threadIdx.x < 32) {
      uint32_t c = 0u;
#pragma unroll
      for (int k = 0; k < kStreamBlock / 32; ++k) c += wc[k][threadIdx.x];
      uint32_t* slot = a.part + ((size_t)g * gridDim.x + bx) * 32 + threadIdx.x;
      *slot += c;
    }
  }
}

__global__ void k_reduce_flips(const uint32_t* part, int blocks_x, int32_t R, uint32_t* flips) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int g = r / 32, j = r % 32;
  uint32_t c = 0u;
  for (int b = 0; b < blocks_x; ++b) c += part[((size_t)g * blocks_x + b) * 32 + j];
  flips[r] = c;
}

// adds the block slots of the RNG counters to the caller's two totals (one block)
__global__ void k_reduce_stats(const unsigned long long* spart, int64_t n_slots, unsigned long long* stats) {
  __shared__ unsigned long long red[2][256];
  unsigned long long c0 = 0ull, c1 = 0ull;
  for (int64_t i = threadIdx.x; i < n_slots; i += blockDim.x) {
    c0 += spart[2 * i];
    c1 += spart[2 * i + 1];
  }
  red[0][threadIdx.x] = c0;
  red[1][threadIdx.x] = c1;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] += red[0][0];
    stats[1] += red[1][0];
  }
}

__global__ void k_zero_u64(unsigned long long* x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0ull;
}

// canonical int8 [R][n] <-> words [groups][n]; bad values flagged per replica
__global__ void k_pack(Lattice L, const int8_t* spins, int32_t R, uint32_t* words, uint32_t* bad) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (i >= (uint32_t)L.n) return;
  int p;
  uint32_t h;
  site_to_split(L, i, p, h);
  const int r0 = 32 * g, nvalid = min(32, R - r0);
  uint32_t word = 0u, flag = 0u;
  for (int j = 0; j < nvalid; ++j) {
    const int8_t v = spins[(size_t)(r0 + j) * L.n + i];
    word |= (v > 0 ? 1u : 0u) << j;
    flag |= (v != 1 && v != -1) ? (1u << j) : 0u;
  }
  words[(size_t)g * L.n + (uint32_t)p * (uint32_t)L.half + h] = word;
  if (flag) atomicOr(&bad[g], flag);
}

__global__ void k_init_words(Lattice L, uint64_t seed, int32_t replica_offset, uint32_t* words) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (i >= (uint32_t)L.n) return;
  int p;
  uint32_t h;
  site_to_split(L, i, p, h);
  const uint32_t quad0 = (uint32_t)(replica_offset + 32 * g) >> 2;
  uint32_t word = 0u;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const u32x4 u = philox_lane_c0(seed, i, 0u, quad0 + q, kTagInit);
#pragma unroll
    for (int b = 0; b < 4; ++b) word |= (u.v[b] >> 31) << (4 * q + b);
  }
  words[(size_t)g * L.n + (uint32_t)p * (uint32_t)L.half + h] = word;
}

__global__ void k_unpack(Lattice L, const uint32_t* words, int32_t R, int8_t* spins) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (i >= (uint32_t)L.n) return;
  int p;
  uint32_t h;
  site_to_split(L, i, p, h);
  const uint32_t word = words[(size_t)g * L.n + (uint32_t)p * (uint32_t)L.half + h];
  const int r0 = 32 * g, nvalid = min(32, R - r0);
  for (int j = 0; j < nvalid; ++j) spins[(size_t)(r0 + j) * L.n + i] = ((word >> j) & 1u) ? (int8_t)1 : (int8_t)-1;
}

__global__ void k_zero_u32(uint32_t* x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0u;
}

// replicas whose input held a value other than +/-1: cut and energy invalid
__global__ void k_mark_invalid(const uint32_t* bad, int32_t R, int64_t* cut, int64_t* energy) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  if ((bad[r / 32] >> (r % 32)) & 1u) {
    if (cut) cut[r] = INT64_MIN;
    if (energy) energy[r] = INT64_MIN;
  }
}

}  // namespace

// Lines per thread: the largest of 4, 2 whose strips still give at least
// 16 waves per CU of a 256-CU device over all groups (and, in 3-D, that
// divides Ly, so that no strip leaves its plane); else 1.  Longer strips
// hold more loads in flight than registers allow at full occupancy.
static int stream_lines_per_thread(const Lattice& L, int groups) {
  for (int k = 4; k > 1; k >>= 1) {
    if (L.ndim == 3 && L.Ly % k != 0) continue;
    const int64_t strips = ((int64_t)L.lines + k - 1) / k;
    if ((int64_t)L.hx * strips * groups >= (int64_t)256 * 16 * 64) return k;
  }
  return 1;
}

static int stream_blocks_x(const Lattice& L, int groups) {
  const int k = stream_lines_per_thread(L, groups);
  const int64_t items = (int64_t)L.hx * (((int64_t)L.lines + k - 1) / k);
  return (int)((items + kStreamBlock - 1) / kStreamBlock);
}

size_t stream_words_bytes(const Lattice& L, int n_replicas) {
  return sizeof(uint32_t) * (size_t)L.n * (size_t)((n_replicas + 31) / 32);
}

size_t stream_part_bytes(const Lattice& L, int n_replicas, bool flips, bool stats) {
  const int groups = (n_replicas + 31) / 32;
  const size_t slots = (size_t)stream_blocks_x(L, groups) * (size_t)groups;
  return (flips ? sizeof(uint32_t) * 32 * slots : 0) + (stats ? sizeof(unsigned long long) * 2 * slots : 0);
}

hipError_t launch_sweep_stream(const ising_graph* g, const SweepLaunch& s, uint32_t* words, uint32_t* bad,
                               uint32_t* part, hipStream_t stream, int64_t* cut_part) {
  const Lattice& L = g->lat;
  const int groups = (s.n_replicas + 31) / 32;
  const int bx = stream_blocks_x(L, groups);
  const int K = stream_lines_per_thread(L, groups);
  const dim3 site_grid((unsigned)((L.n + 255) / 256), (unsigned)groups);
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, stream, bad, (int64_t)groups);
  const int64_t n_slots = (int64_t)bx * groups;
  // part: flip slots (u32 [slots][32]) first, then RNG-count slots (u64 [slots][2])
  unsigned long long* spart =
      s.stats ? (unsigned long long*)(part + (s.flips ? 32 * n_slots : 0)) : nullptr;
  if (s.flips)
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((32 * n_slots + 255) / 256)), dim3(256), 0, stream, part,
                       32 * n_slots);
  if (s.stats)
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((2 * n_slots + 255) / 256)), dim3(256), 0, stream, spart,
                       2 * n_slots);
  if (s.init)
    hipLaunchKernelGGL(k_init_words, site_grid, dim3(256), 0, stream, L, s.seed, s.replica_offset, words);
  else
    hipLaunchKernelGGL(k_pack, site_grid, dim3(256), 0, stream, L, s.spins, s.n_replicas, words, bad);
  StreamArgs a;
  a.lat = L;
  a.wbits = g->d_wbits;
  a.words = words;
  a.thr = s.d_thr;
  a.part = s.flips ? part : nullptr;
  a.spart = spart;
  a.seed = s.seed;
  a.n_replicas = s.n_replicas;
  a.replica_offset = s.replica_offset;
  a.groups = groups;
  a.div_hx = make_fastdiv((uint32_t)L.hx);
  a.div_bx = make_fastdiv((uint32_t)bx);
  const dim3 grid((unsigned)bx, (unsigned)groups);
  auto go = [&](auto kernel) {
    for (int t = s.t_begin; t < s.t_end; ++t)
      for (int p = 0; p < 2; ++p) hipLaunchKernelGGL(kernel, grid, dim3(kStreamBlock), 0, stream, a, p, t);
  };
  auto pick = [&](auto nd, auto st) {
    constexpr int ND = decltype(nd)::value;
    constexpr bool ST = decltype(st)::value;
    if (K == 4) go(k_halfsweep_stream<ND, ST, 4>);
    else if (K == 2) go(k_halfsweep_stream<ND, ST, 2>);
    else go(k_halfsweep_stream<ND, ST, 1>);
  };
  using ND2 = std::integral_constant<int, 2>;
  using ND3 = std::integral_constant<int, 3>;
  using STY = std::integral_constant<bool, true>;
  using STN = std::integral_constant<bool, false>;
  if (g->ndim == 2) {
    if (s.stats) pick(ND2(), STY()); else pick(ND2(), STN());
  } else {
    if (s.stats) pick(ND3(), STY()); else pick(ND3(), STN());
  }
  hipLaunchKernelGGL(k_unpack, site_grid, dim3(256), 0, stream, L, words, s.n_replicas, s.spins);
  if (s.flips)
    hipLaunchKernelGGL(k_reduce_flips, dim3((unsigned)((s.n_replicas + 255) / 256)), dim3(256), 0, stream, part, bx,
                       s.n_replicas, s.flips);
  if (s.stats) hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(256), 0, stream, spart, n_slots, s.stats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (s.cut || s.energy) {
    e = launch_cut_energy(g, s.spins, s.n_replicas, s.cut, s.energy, stream, cut_part);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mark_invalid, dim3((unsigned)((s.n_replicas + 255) / 256)), dim3(256), 0, stream, bad,
                       s.n_replicas, s.cut, s.energy);
  }
  return hipGetLastError();
}

}  // namespace ising
