// Checkerboard Metropolis sweeps, bit-sliced over 4 replicas x 4 sites per
// word: the single-instance launch (one block per replica quad).  The word
// layout and the per-quad work are described in bs4_quad.hpp.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bs4_quad.hpp"
#include "internal.hpp"

namespace ising {
namespace {

using namespace bs4q;

template <int NDIM, bool FLIPS, bool STATS, bool PT, bool PART>
__global__ void __launch_bounds__(kMaxBlock) k_sweep_bs4(Bs4Args a) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t extra[kExtraWords];
  bs4_quad<NDIM, FLIPS, STATS, PT, PART>(a, blockIdx.x * 4, lds, extra);
}

// word lines per plane: rows / 4, or (rows + 2) / 4 with a last two-row line
int word_lines(const Lattice& L) { return (L.Ly + 3) / 4 * L.Lz; }

}  // namespace

// every even torus: Ly = 2 mod 4 takes the variant whose last word line of a
// plane holds two rows
bool sweep_bs4_supported(const Lattice& L) { return L.hx >= 1 && L.Ly % 2 == 0; }

size_t sweep_bs4_dyn_lds(const Lattice& L) {
  const size_t rs = L.ndim == 2 ? (size_t)rec_words<2>() : (size_t)rec_words<3>();
  return (size_t)word_lines(L) * (size_t)L.hx * rs * 4u;
}

size_t sweep_bs4_lds_bytes(const Lattice& L) { return sweep_bs4_dyn_lds(L) + kExtraWords * 4u; }

int sweep_bs4_block(const Lattice& L, int requested) {
  if (!sweep_bs4_supported(L) || L.hx > kMaxBlock) return 0;
  const int GL = word_lines(L);
  int max_lp = kMaxBlock / L.hx;
  if (max_lp > GL) max_lp = GL;
  int lp = max_lp;
  if (requested > 0) {
    lp = requested / L.hx;
    if (lp < 1) lp = 1;
    if (lp > max_lp) lp = max_lp;
  }
  return lp * L.hx;
}

int sweep_bs4_default_block(const Lattice& L, int n_replicas, int cus, size_t lds_per_cu) {
  const int full = sweep_bs4_block(L, 0);
  const int quads = (n_replicas + 3) / 4;
  if (full <= 0 || quads < 4 * cus || 2 * sweep_bs4_lds_bytes(L) > lds_per_cu) return full;
  // four or more quads per compute unit: blocks of at most 512 threads (8
  // waves: the kernel's registers leave a CU 16 wave slots, four waves per
  // SIMD, so two such blocks fit where a 9-wave block leaves room for one),
  // whose co-resident blocks overlap each other's barriers better than the
  // largest block does
  const int lp = 512 / L.hx;
  return sweep_bs4_block(L, (lp < 1 ? 1 : lp) * L.hx);
}

hipError_t launch_sweep_bs4(const ising_graph* g, const SweepLaunch& s, hipStream_t stream) {
  const Lattice& L = g->lat;
  const int block = sweep_bs4_block(L, s.block_threads);
  if (block <= 0) return hipErrorInvalidValue;
  Bs4Args a;
  a.lat = L;
  a.wbits = g->d_wbits;
  a.spins = s.spins;
  a.thr = s.d_thr;
  a.rep_thr = s.rep_thr;
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
  const size_t lds = sweep_bs4_dyn_lds(L);
  const int grid = (s.n_replicas + 3) / 4;
  auto go = [&](auto kernel) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, a);
    return hipSuccess;
  };
  const bool fl = s.flips != nullptr, st = s.stats != nullptr;
  hipError_t e;
  // PART selects the two-row last word line (Ly = 2 mod 4)
  auto pick = [&](auto ndim, auto part) -> hipError_t {
    constexpr int D = decltype(ndim)::value;
    constexpr bool P = decltype(part)::value;
    if (s.rep_thr)  // replica exchange: no RNG statistics variant
      return fl ? go(k_sweep_bs4<D, true, false, true, P>) : go(k_sweep_bs4<D, false, false, true, P>);
    if (st) return fl ? go(k_sweep_bs4<D, true, true, false, P>) : go(k_sweep_bs4<D, false, true, false, P>);
    return fl ? go(k_sweep_bs4<D, true, false, false, P>) : go(k_sweep_bs4<D, false, false, false, P>);
  };
  using two = std::integral_constant<int, 2>;
  using three = std::integral_constant<int, 3>;
  const bool part = L.Ly % 4 != 0;
  if (g->ndim == 2)
    e = part ? pick(two(), std::true_type()) : pick(two(), std::false_type());
  else
    e = part ? pick(three(), std::true_type()) : pick(three(), std::false_type());
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace ising
