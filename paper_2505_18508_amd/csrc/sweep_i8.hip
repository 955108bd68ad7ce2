// Checkerboard Metropolis sweeps, four replicas per 32-bit LDS word: the
// single-instance launch (one block per replica quad).  The per-quad work
// and the word layout are described in i8_quad.hpp.
#include <hip/hip_runtime.h>

#include "i8_quad.hpp"
#include "internal.hpp"

namespace ising {
namespace {

using namespace i8q;

template <int NDIM, bool STATS>
__global__ void __launch_bounds__(kMaxBlock) k_sweep_i8(I8Args a) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t lut[2 * kLutSet];
  __shared__ uint32_t extra[kExtraWords];
  i8_quad<NDIM, STATS>(a, blockIdx.x * 4, lds, lut, extra);
}

}  // namespace

// dynamic part (the state words) and the whole block's LDS with the static tables
size_t sweep_i8_dyn_lds(const Lattice& L) { return (size_t)L.n * 4u; }
size_t sweep_i8_lds_bytes(const Lattice& L) { return sweep_i8_dyn_lds(L) + kStaticLds; }

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
  const size_t lds = sweep_i8_dyn_lds(L);
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
