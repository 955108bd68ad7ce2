// Replica exchange (parallel tempering) on the sweep kernels.
//
// L ladders of K inverse temperatures; replica slot r = l K + i starts at
// temperature i of ladder l and keeps its spins: only temperature labels
// move.  A round runs its sweeps with every replica at its own temperature
// (the sweep kernels' per-replica thresholds), then k_pt_exchange makes one
// pass over the adjacent pairs (k, k+1) with k of the round's parity: the
// replicas at beta_k and beta_{k+1} swap temperatures with probability
// min(1, exp((beta_k - beta_{k+1}) (H_a - H_b))) (Swendsen & Wang, 1986;
// Hukushima & Nemoto, 1996), which keeps the product of the K Boltzmann
// distributions stationary.  The decision is integer, as for the sweeps: on
// an even-degree torus H_a - H_b = 4m; m <= 0 or equal temperatures accept
// without a draw, else accept iff word 0 of Philox(seed, (k, round, l, tag 4))
// is below min(2^32 - 1, floor(2^32 exp(-(beta_{k+1} - beta_k) 4m))), a
// table computed on the host.  Everything of a round is queued on the
// caller's stream; nothing synchronises.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "internal.hpp"
#include "ising.h"
#include "philox.hpp"

struct ising_pt {
  const ising_graph* g = nullptr;
  int32_t K = 0, L = 0, R = 0, kmax = 0;
  uint64_t seed = 0;
  int device = 0;
  int32_t xmax = 0;                 // entries per pair in the exchange table
  uint32_t* d_metro = nullptr;      // [K][kmax] Metropolis thresholds of each temperature
  uint32_t* d_xthr = nullptr;       // [K-1][xmax] exchange thresholds, m = 1..xlen[k]
  int32_t* d_xlen = nullptr;        // [K-1]; -1: equal temperatures (always swap)
  int32_t* d_kidx = nullptr;        // [R] temperature index of each slot
  int32_t* d_pos = nullptr;         // [L][K] slot holding each temperature
  uint32_t* d_rep_thr = nullptr;    // [R][kmax] thresholds of each slot's current temperature
  int64_t* d_energy = nullptr;      // [R] energies after the last round's sweeps
  unsigned long long* d_acc = nullptr;  // [K-1] accepted exchanges per pair
};

namespace ising {
namespace {

constexpr int32_t kMaxExchangeEntries = 65536;

__global__ void k_pt_exchange(int32_t K, int32_t L, uint32_t round, uint64_t seed, int32_t kmax,
                              const int64_t* energy, int32_t* kidx, int32_t* pos, uint32_t* rep_thr,
                              const uint32_t* metro, const uint32_t* xthr, const int32_t* xlen, int32_t xmax,
                              unsigned long long* acc) {
  const int32_t first = (int32_t)(round & 1u);
  const int32_t npairs = (K - first) / 2;  // pairs k = first, first + 2, ... <= K - 2
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (npairs <= 0 || idx >= (int64_t)L * npairs) return;
  const int32_t l = (int32_t)(idx / npairs);
  const int32_t k = first + 2 * (int32_t)(idx - (int64_t)l * npairs);
  int32_t* P = pos + (size_t)l * K;
  const int32_t a = P[k], b = P[k + 1];
  const int64_t ha = energy[a], hb = energy[b];
  if (ha == INT64_MIN || hb == INT64_MIN) return;  // flagged input: no exchange
  const int64_t d = ha - hb;
  bool swap;
  if (d <= 0 || xlen[k] < 0) {
    swap = true;
  } else {
    const int64_t m = d >> 2;  // energies of an even-degree torus differ by multiples of 4
    if (m > xlen[k]) {
      swap = false;
    } else {
      const u32x4 u = philox_ref(seed, (uint32_t)k, round, (uint32_t)l, kTagExchange);
      swap = u.v[0] < xthr[(size_t)k * xmax + (size_t)(m - 1)];
    }
  }
  if (!swap) return;
  P[k] = b;
  P[k + 1] = a;
  kidx[a] = k + 1;
  kidx[b] = k;
  for (int j = 0; j < kmax; ++j) {
    rep_thr[(size_t)a * kmax + j] = metro[(size_t)(k + 1) * kmax + j];
    rep_thr[(size_t)b * kmax + j] = metro[(size_t)k * kmax + j];
  }
  atomicAdd(&acc[k], 1ull);
}

__global__ void k_copy_i64(const int64_t* src, int64_t* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_copy_i32(const int32_t* src, int32_t* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

void free_pt(ising_pt* pt) {
  if (!pt) return;
  (void)hipFree(pt->d_metro);
  (void)hipFree(pt->d_xthr);
  (void)hipFree(pt->d_xlen);
  (void)hipFree(pt->d_kidx);
  (void)hipFree(pt->d_pos);
  (void)hipFree(pt->d_rep_thr);
  (void)hipFree(pt->d_energy);
  (void)hipFree(pt->d_acc);
  delete pt;
}

}  // namespace
}  // namespace ising

extern "C" {

int ising_pt_create(const ising_graph* g, int32_t n_temps, const double* betas, int32_t n_ladders, uint64_t seed,
                    ising_pt** out) {
  using namespace ising;
  if (!out) return fail(ISING_E_ARG, "out is NULL");
  *out = nullptr;
  if (!g) return fail(ISING_E_ARG, "graph is NULL");
  if (n_temps < 2 || !betas) return fail(ISING_E_ARG, "need n_temps >= 2 and betas");
  if (n_ladders < 1 || (int64_t)n_ladders * n_temps > INT32_MAX) return fail(ISING_E_ARG, "n_ladders out of range");
  for (int32_t k = 0; k < n_temps; ++k) {
    if (!(betas[k] >= 0.0) || !std::isfinite(betas[k])) return fail(ISING_E_ARG, "betas[%d] must be finite, >= 0", k);
    if (k > 0 && betas[k] < betas[k - 1]) return fail(ISING_E_ARG, "betas must be non-decreasing");
  }
  int rc = check_device(g);
  if (rc) return rc;
  const int32_t K = n_temps, kmax = g->ndim;
  // host tables
  std::vector<uint32_t> metro((size_t)K * kmax);
  for (int32_t i = 0; i < K; ++i)
    for (int32_t k = 1; k <= kmax; ++k) metro[(size_t)i * kmax + (k - 1)] = accept_threshold(betas[i], k);
  std::vector<int32_t> xlen((size_t)K - 1);
  std::vector<std::vector<uint32_t>> rows((size_t)K - 1);
  int32_t xmax = 1;
  for (int32_t k = 0; k + 1 < K; ++k) {
    const double db = betas[k + 1] - betas[k];
    if (db == 0.0) {
      xlen[(size_t)k] = -1;
      continue;
    }
    for (int64_t m = 1;; ++m) {
      const double scaled = std::ldexp(std::exp(-(db * (4.0 * (double)m))), 32);
      const uint32_t T = scaled >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)std::floor(scaled);
      if (T == 0u) break;
      if (m > kMaxExchangeEntries)
        return fail(ISING_E_ARG, "temperatures %d and %d are too close (beta gap %g)", k, k + 1, db);
      rows[(size_t)k].push_back(T);
    }
    xlen[(size_t)k] = (int32_t)rows[(size_t)k].size();
    if (xlen[(size_t)k] > xmax) xmax = xlen[(size_t)k];
  }
  std::vector<uint32_t> xthr((size_t)(K - 1) * xmax, 0u);
  for (int32_t k = 0; k + 1 < K; ++k)
    for (size_t m = 0; m < rows[(size_t)k].size(); ++m) xthr[(size_t)k * xmax + m] = rows[(size_t)k][m];
  const int32_t L = n_ladders, R = L * K;
  std::vector<int32_t> kidx((size_t)R), pos((size_t)R);
  std::vector<uint32_t> rep((size_t)R * kmax);
  for (int32_t r = 0; r < R; ++r) {
    kidx[(size_t)r] = r % K;
    pos[(size_t)r] = r;  // pos[l][k] = l K + k
    for (int32_t j = 0; j < kmax; ++j) rep[(size_t)r * kmax + j] = metro[(size_t)(r % K) * kmax + j];
  }
  ising_pt* pt = new (std::nothrow) ising_pt();
  if (!pt) return fail(ISING_E_NOMEM, "replica-exchange handle");
  pt->g = g;
  pt->K = K;
  pt->L = L;
  pt->R = R;
  pt->kmax = kmax;
  pt->seed = seed;
  pt->device = g->device;
  pt->xmax = xmax;
  hipError_t e = hipMalloc((void**)&pt->d_metro, sizeof(uint32_t) * metro.size());
  if (e == hipSuccess) e = hipMalloc((void**)&pt->d_xthr, sizeof(uint32_t) * xthr.size());
  if (e == hipSuccess) e = hipMalloc((void**)&pt->d_xlen, sizeof(int32_t) * xlen.size());
  if (e == hipSuccess) e = hipMalloc((void**)&pt->d_kidx, sizeof(int32_t) * (size_t)R);
  if (e == hipSuccess) e = hipMalloc((void**)&pt->d_pos, sizeof(int32_t) * (size_t)R);
  if (e == hipSuccess) e = hipMalloc((void**)&pt->d_rep_thr, sizeof(uint32_t) * rep.size());
  if (e == hipSuccess) e = hipMalloc((void**)&pt->d_energy, sizeof(int64_t) * (size_t)R);
  if (e == hipSuccess) e = hipMalloc((void**)&pt->d_acc, sizeof(unsigned long long) * (size_t)(K - 1));
  if (e != hipSuccess) {
    free_pt(pt);
    return fail(ISING_E_NOMEM, "replica-exchange tables: %s", hipGetErrorString(e));
  }
  std::vector<unsigned long long> zero((size_t)(K - 1), 0ull);
  e = hipMemcpy(pt->d_metro, metro.data(), sizeof(uint32_t) * metro.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pt->d_xthr, xthr.data(), sizeof(uint32_t) * xthr.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pt->d_xlen, xlen.data(), sizeof(int32_t) * xlen.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pt->d_kidx, kidx.data(), sizeof(int32_t) * (size_t)R, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pt->d_pos, pos.data(), sizeof(int32_t) * (size_t)R, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pt->d_rep_thr, rep.data(), sizeof(uint32_t) * rep.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pt->d_acc, zero.data(), sizeof(unsigned long long) * zero.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_pt(pt);
    return fail_hip(e, "replica-exchange table upload");
  }
  *out = pt;
  return ISING_OK;
}

int ising_pt_run(ising_pt* pt, int8_t* spins, int32_t init_spins, int32_t round_begin, int32_t n_rounds,
                 int32_t sweeps_per_round, int64_t* cut_out, int64_t* energy_out, void* stream) {
  using namespace ising;
  if (!pt) return fail(ISING_E_ARG, "handle is NULL");
  if (!spins) return fail(ISING_E_ARG, "spins is NULL");
  if (round_begin < 0 || n_rounds < 0 || sweeps_per_round < 1)
    return fail(ISING_E_ARG, "need round_begin >= 0, n_rounds >= 0, sweeps_per_round >= 1");
  if (init_spins && round_begin != 0) return fail(ISING_E_ARG, "init_spins needs round_begin == 0");
  if ((int64_t)(round_begin + (int64_t)n_rounds) * sweeps_per_round > INT32_MAX)
    return fail(ISING_E_ARG, "sweep indices exceed 2^31 - 1");
  int rc = check_device(pt->g);
  if (rc) return rc;
  if (n_rounds == 0) return ISING_OK;
  hipStream_t st = (hipStream_t)stream;
  const int32_t end_round = round_begin + n_rounds;
  for (int32_t q = round_begin; q < end_round; ++q) {
    ising_run_params p{};
    p.struct_size = sizeof(ising_run_params);
    p.layout = ISING_LAYOUT_AUTO;
    p.seed = pt->seed;
    p.n_replicas = pt->R;
    p.n_sweeps = end_round * sweeps_per_round;  // sweep indices key the Philox streams
    p.sweep_begin = q * sweeps_per_round;
    p.sweep_end = (q + 1) * sweeps_per_round;
    p.schedule = ISING_SCHED_LINEAR;
    p.beta0 = p.beta1 = 0.0;  // unused: per-replica thresholds
    p.init_spins = (init_spins && q == 0) ? 1 : 0;
    p.replica_thresholds = pt->d_rep_thr;
    rc = ising_run_trials(pt->g, &p, spins, q + 1 == end_round ? cut_out : nullptr, pt->d_energy, nullptr, st);
    if (rc) return rc;
    const int32_t npairs = (pt->K - (q & 1)) / 2;
    const int64_t threads = (int64_t)pt->L * npairs;
    if (threads > 0)
      hipLaunchKernelGGL(k_pt_exchange, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, pt->K, pt->L,
                         (uint32_t)q, pt->seed, pt->kmax, (const int64_t*)pt->d_energy, pt->d_kidx, pt->d_pos,
                         pt->d_rep_thr, (const uint32_t*)pt->d_metro, (const uint32_t*)pt->d_xthr,
                         (const int32_t*)pt->d_xlen, pt->xmax, pt->d_acc);
  }
  if (energy_out)
    hipLaunchKernelGGL(k_copy_i64, dim3((unsigned)((pt->R + 255) / 256)), dim3(256), 0, st,
                       (const int64_t*)pt->d_energy, energy_out, (int64_t)pt->R);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(e, "replica-exchange launch");
  return ISING_OK;
}

int ising_pt_state(const ising_pt* pt, int32_t* temp_index_out, uint64_t* accepted_out, void* stream) {
  using namespace ising;
  if (!pt) return fail(ISING_E_ARG, "handle is NULL");
  int rc = check_device(pt->g);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (temp_index_out)
    hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)((pt->R + 255) / 256)), dim3(256), 0, st,
                       (const int32_t*)pt->d_kidx, temp_index_out, (int64_t)pt->R);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && accepted_out) {
    e = hipStreamSynchronize(st);
    if (e == hipSuccess)
      e = hipMemcpy(accepted_out, pt->d_acc, sizeof(unsigned long long) * (size_t)(pt->K - 1), hipMemcpyDeviceToHost);
  }
  if (e != hipSuccess) return fail_hip(e, "replica-exchange state");
  return ISING_OK;
}

void ising_pt_destroy(ising_pt* pt) { ising::free_pt(pt); }

}  // extern "C"
