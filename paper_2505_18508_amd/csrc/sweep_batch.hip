// Uneven instances in one persistent launch.
//
// Every (instance, replica quad) pair is a work item.  Resident blocks take
// items from a device queue, costliest first (sites x sweeps x replicas,
// weighted by the packing's cost per attempt), until the queue is empty, so
// every block reaches the exit.  Each instance keeps the four-replica packing
// that suits its lattice: bit-sliced 4 x 4 sites per word where the
// second-fastest axis is a multiple of 4, else one byte per replica with
// maintained fields; a block runs either routine on the same LDS.  Each
// replica's trajectory is the one a single-instance launch gives.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "bs4_quad.hpp"
#include "i8_quad.hpp"
#include "internal.hpp"
#include "ising.h"

namespace ising {
namespace {

constexpr int kBatchBlock = 1024;
static_assert(bs4q::kExtraWords == i8q::kExtraWords, "both routines share the block's counter words");
static_assert(bs4q::kMaxBlock == kBatchBlock && i8q::kMaxBlock == kBatchBlock, "one block size for both routines");

struct BatchItem {
  int32_t inst;  // instance
  int32_t r0;    // first local replica of the quad
};

// One instance: its packing and the arguments of that packing's routine.
struct BatchInst {
  int32_t bs4;   // 1: bit-sliced 4 x 4, 0: byte per replica
  int32_t part;  // bs4 with Ly = 2 mod 4 (two-row last word line of each plane)
  i8q::I8Args i8;
  bs4q::Bs4Args b4;
};

template <int NDIM>
__global__ void __launch_bounds__(kBatchBlock) k_sweep_batch(const BatchInst* inst, const BatchItem* items, int n_items,
                                                             unsigned int* counter) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t lut[2 * i8q::kLutSet];
  __shared__ uint32_t extra[i8q::kExtraWords];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = next;
    __syncthreads();
    if (it >= n_items) break;
    const BatchItem bi = items[it];
    const BatchInst& I = inst[bi.inst];
    if (I.bs4) {
      const bool pt = I.b4.rep_thr != nullptr;
      if (I.part) {
        if (pt)
          bs4q::bs4_quad<NDIM, true, false, true, true>(I.b4, bi.r0, lds, extra);
        else
          bs4q::bs4_quad<NDIM, true, false, false, true>(I.b4, bi.r0, lds, extra);
      } else if (pt) {
        bs4q::bs4_quad<NDIM, true, false, true>(I.b4, bi.r0, lds, extra);
      } else {
        bs4q::bs4_quad<NDIM, true, false, false>(I.b4, bi.r0, lds, extra);
      }
    } else {
      i8q::i8_quad<NDIM, false>(I.i8, bi.r0, lds, lut, extra);
    }
    __syncthreads();
  }
}

// Zeroes the queue counter on the stream (no memset node), so a replayed
// graph restarts the queue.
__global__ void k_reset_counter(unsigned int* counter) {
  if (threadIdx.x == 0) counter[0] = 0u;
}

}  // namespace

hipError_t build_batch(const ising_graph* const* graphs, const SweepLaunch* launches, const int* layouts, int n_inst,
                       BatchPlan* plan) {
  plan->ndim = graphs[0]->ndim;
  std::vector<BatchInst> inst((size_t)n_inst);
  std::vector<std::pair<int64_t, BatchItem>> items;
  size_t lds = 0;
  for (int k = 0; k < n_inst; ++k) {
    const ising_graph* g = graphs[k];
    const SweepLaunch& s = launches[k];
    const Lattice& L = g->lat;
    BatchInst& I = inst[(size_t)k];
    I.bs4 = layouts[k] == ISING_LAYOUT_BS4 ? 1 : 0;
    I.part = (I.bs4 && L.Ly % 4 != 0) ? 1 : 0;
    // threads that work on this instance's items: its requested block size
    // (the autotuner's pick, say) within the launch's block, else all of it
    const int want = s.block_threads > 0 && s.block_threads < kBatchBlock ? s.block_threads : kBatchBlock;
    const int block = I.bs4 ? sweep_bs4_block(L, want) : sweep_i8_block(L, want);
    if (block <= 0) return hipErrorInvalidValue;
    auto fill = [&](auto& a) {
      a.lat = L;
      a.wbits = g->d_wbits;
      a.spins = s.spins;
      a.thr = s.d_thr;
      a.rep_thr = s.rep_thr;
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
    };
    fill(I.i8);
    fill(I.b4);
    const size_t b = I.bs4 ? sweep_bs4_dyn_lds(L) : sweep_i8_dyn_lds(L);
    if (b > lds) lds = b;
    // relative VALU cost per attempt of the two routines (about 18 : 23)
    const int64_t cost = (int64_t)L.n * (s.t_end - s.t_begin) * (I.bs4 ? 18 : 23);
    for (int r0 = 0; r0 < s.n_replicas; r0 += 4) items.push_back({cost * std::min(4, s.n_replicas - r0), BatchItem{k, r0}});
  }
  // costliest first; ties in instance and replica order
  std::stable_sort(items.begin(), items.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  std::vector<BatchItem> order(items.size());
  for (size_t i = 0; i < items.size(); ++i) order[i] = items[i].second;
  plan->n_items = (int)order.size();
  plan->lds = lds;
  plan->block = kBatchBlock;
  const void* kernel = plan->ndim == 2 ? (const void*)k_sweep_batch<2> : (const void*)k_sweep_batch<3>;
  hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0, dev = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBatchBlock, lds);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  plan->grid = std::min(plan->n_items, per_cu * cus);
  e = hipMalloc(&plan->d_inst, sizeof(BatchInst) * (size_t)n_inst);
  if (e == hipSuccess) e = hipMalloc(&plan->d_items, sizeof(BatchItem) * order.size());
  if (e == hipSuccess) e = hipMalloc((void**)&plan->d_counter, sizeof(unsigned int));
  if (e == hipSuccess)
    e = hipMemcpy(plan->d_inst, inst.data(), sizeof(BatchInst) * (size_t)n_inst, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(plan->d_items, order.data(), sizeof(BatchItem) * order.size(), hipMemcpyHostToDevice);
  return e;
}

hipError_t run_batch(const BatchPlan& plan, hipStream_t stream) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, stream, plan.d_counter);
  if (plan.ndim == 2)
    hipLaunchKernelGGL(k_sweep_batch<2>, dim3(plan.grid), dim3(plan.block), plan.lds, stream,
                       (const BatchInst*)plan.d_inst, (const BatchItem*)plan.d_items, plan.n_items, plan.d_counter);
  else
    hipLaunchKernelGGL(k_sweep_batch<3>, dim3(plan.grid), dim3(plan.block), plan.lds, stream,
                       (const BatchInst*)plan.d_inst, (const BatchItem*)plan.d_items, plan.n_items, plan.d_counter);
  return hipGetLastError();
}

void free_batch(BatchPlan& plan) {
  (void)hipFree(plan.d_inst);
  (void)hipFree(plan.d_items);
  (void)hipFree(plan.d_counter);
  plan.d_inst = plan.d_items = nullptr;
  plan.d_counter = nullptr;
}

}  // namespace ising
