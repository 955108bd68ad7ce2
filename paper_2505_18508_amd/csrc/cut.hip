// Exact cut and energy of R states (paper, Section II): for every edge e =
// (a, b), counted once, cut += w_e [s_a != s_b] (eq. (1)) and
// H += w_e s_a s_b (eq. (2) with J = -w, h = 0).  One block per replica, or
// per 65,536-site chunk of a replica on large lattices; integer arithmetic
// throughout.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "philox.hpp"
#include "reduce.hpp"

namespace ising {
namespace {

constexpr int kCutBlock = 256;
constexpr uint32_t kCutChunk = 65536;  // sites per block on large lattices

// Sums of one chunk [i0, i1) of one replica: cut, energy and the count of
// values other than +1 / -1.  part == nullptr: the chunk is the whole
// replica and the block writes the outputs itself.
template <int NDIM>
__global__ void __launch_bounds__(kCutBlock) k_cut_energy(Lattice L, const int8_t* w, const int8_t* spins,
                                                          uint32_t chunk, uint32_t n_chunks, int64_t* part,
                                                          int64_t* cut, int64_t* energy) {
  const size_t n = (size_t)L.n;
  const uint32_t r = blockIdx.x / n_chunks, ch = blockIdx.x - r * n_chunks;
  const int8_t* s = spins + (size_t)r * n;
  const uint32_t Lx = (uint32_t)L.Lx, Ly = (uint32_t)L.Ly, Lz = (uint32_t)L.Lz;
  const uint32_t plane = Lx * Ly;
  const uint32_t i0 = ch * chunk;
  const uint32_t i1 = min((uint32_t)L.n, i0 + chunk);
  int32_t c = 0, h = 0, bad = 0;
  for (uint32_t i = i0 + threadIdx.x; i < i1; i += kCutBlock) {
    const uint32_t line = fdiv(i, L.div_lx);
    const uint32_t x = i - line * Lx;
    const uint32_t z = NDIM == 2 ? 0u : fdiv(line, L.div_ly);
    const uint32_t y = line - z * Ly;
    const int si = s[i];
    bad += (si != 1 && si != -1) ? 1 : 0;
    uint32_t nb[NDIM];
    nb[0] = (x + 1u == Lx) ? i + 1u - Lx : i + 1u;
    nb[1] = (y + 1u == Ly) ? i + Lx - plane : i + Lx;
    if (NDIM == 3) nb[NDIM - 1] = (z + 1u == Lz) ? i - (Lz - 1u) * plane : i + plane;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const int sj = s[nb[d]];
      const int we = w[(size_t)NDIM * i + d];
      h += we * si * sj;
      c += (si != sj) ? we : 0;
    }
  }
  const int64_t ct = block_sum<kCutBlock>((int64_t)c);
  const int64_t ht = block_sum<kCutBlock>((int64_t)h);
  const int64_t bt = block_sum<kCutBlock>((int64_t)bad);
  if (threadIdx.x == 0) {
    if (part) {
      int64_t* q = part + 3 * (size_t)blockIdx.x;
      q[0] = ct;
      q[1] = ht;
      q[2] = bt;
    } else {
      if (cut) cut[r] = bt ? INT64_MIN : ct;
      if (energy) energy[r] = bt ? INT64_MIN : ht;
    }
  }
}

// Per replica, the chunk sums in chunk order (exact integers: the result
// does not depend on how the lattice was split).
__global__ void k_cut_finish(const int64_t* part, uint32_t n_chunks, int64_t n_replicas, int64_t* cut,
                             int64_t* energy) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_replicas) return;
  int64_t c = 0, h = 0, b = 0;
  for (uint32_t k = 0; k < n_chunks; ++k) {
    const int64_t* q = part + 3 * ((size_t)r * n_chunks + k);
    c += q[0];
    h += q[1];
    b += q[2];
  }
  if (cut) cut[r] = b ? INT64_MIN : c;
  if (energy) energy[r] = b ? INT64_MIN : h;
}

__global__ void k_philox_dump(uint64_t key, const uint32_t* ctr, int64_t m, uint32_t* out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const uint32_t* c = ctr + 4 * k;
  const u32x4 o = philox_lanes(key, c[0], c[1], c[2], c[3]);
  out[4 * k + 0] = o.v[0];
  out[4 * k + 1] = o.v[1];
  out[4 * k + 2] = o.v[2];
  out[4 * k + 3] = o.v[3];
}

}  // namespace

size_t cut_part_bytes(const Lattice& L, int64_t n_replicas) {
  const uint32_t n_chunks = ((uint32_t)L.n + kCutChunk - 1) / kCutChunk;
  return n_chunks > 1 ? sizeof(int64_t) * 3 * (size_t)n_chunks * (size_t)n_replicas : 0;
}

hipError_t launch_cut_energy(const ising_graph* g, const int8_t* spins, int64_t n_replicas, int64_t* cut,
                             int64_t* energy, hipStream_t stream, int64_t* part_scratch) {
  if (n_replicas == 0 || (!cut && !energy)) return hipSuccess;
  // large lattices: several blocks per replica, so that enough loads are in
  // flight; their sums go through the caller's scratch (every entry written
  // before it is read) or a stream-ordered array
  const uint32_t n = (uint32_t)g->lat.n;
  const uint32_t n_chunks = (n + kCutChunk - 1) / kCutChunk;
  const uint32_t chunk = n_chunks == 1 ? n : kCutChunk;
  if ((int64_t)n_chunks * n_replicas > INT32_MAX) return hipErrorInvalidValue;
  int64_t* part = nullptr;
  const bool own = n_chunks > 1 && !part_scratch;
  if (n_chunks > 1) part = part_scratch;
  if (own) {
    hipError_t e = hipMallocAsync((void**)&part, cut_part_bytes(g->lat, n_replicas), stream);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((unsigned)(n_chunks * n_replicas));
  if (g->ndim == 2)
    hipLaunchKernelGGL(k_cut_energy<2>, grid, dim3(kCutBlock), 0, stream, g->lat, g->d_w, spins, chunk, n_chunks,
                       part, cut, energy);
  else
    hipLaunchKernelGGL(k_cut_energy<3>, grid, dim3(kCutBlock), 0, stream, g->lat, g->d_w, spins, chunk, n_chunks,
                       part, cut, energy);
  if (part) {
    hipLaunchKernelGGL(k_cut_finish, dim3((unsigned)((n_replicas + 255) / 256)), dim3(256), 0, stream, part, n_chunks,
                       n_replicas, cut, energy);
    if (own) (void)hipFreeAsync(part, stream);
  }
  return hipGetLastError();
}

hipError_t launch_philox_dump(uint64_t key, const uint32_t* ctr, int64_t m, uint32_t* out, hipStream_t stream) {
  if (m == 0) return hipSuccess;
  const int block = 256;
  const int64_t grid = (m + block - 1) / block;
  hipLaunchKernelGGL(k_philox_dump, dim3((unsigned)grid), dim3(block), 0, stream, key, ctr, m, out);
  return hipGetLastError();
}

}  // namespace ising
