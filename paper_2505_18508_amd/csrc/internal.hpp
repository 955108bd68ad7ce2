// Internal declarations of the library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "lattice.hpp"

struct ThrCacheEntry {
  int32_t schedule, n_sweeps, kmax;
  double beta0, beta1;
  uint64_t table_hash;
  std::vector<double> table;  // the beta table of a table schedule (compared on a hit)
  std::vector<uint32_t> host; // source of the upload (kept: the copy is asynchronous)
  uint32_t* d_thr;            // device [n_sweeps][kmax]
  hipEvent_t ready;           // recorded after the upload, on the stream that made it
  hipStream_t made_on;
};

// Host source of an uncached table's asynchronous upload, released once its
// event has completed.
struct ThrUpload {
  std::vector<uint32_t> host;
  hipEvent_t done;
};

struct ising_graph {
  int32_t ndim;
  int32_t dims[3];
  ising::Lattice lat;
  int64_t n, n_edges, w_total;
  int32_t degree;
  int device;
  std::vector<int8_t> w_host;  // edge order
  int8_t* d_w = nullptr;       // device edge weights [n_edges]
  uint8_t* d_wbits = nullptr;  // device per-site weight sign bits, colour-split order [n]
  mutable std::mutex mu;
  mutable std::vector<ThrCacheEntry> thr_cache;
  mutable std::vector<ThrUpload> thr_uploads;
};

namespace ising {

// Record a message for ising_last_error() and return code.
int fail(int code, const char* fmt, ...);
int fail_hip(hipError_t e, const char* what);
// Metropolis threshold of an energy increase 4k at inverse temperature beta:
// accept iff u < min(2^32 - 1, floor(2^32 exp(-4 k beta))), u a Philox word.
uint32_t accept_threshold(double beta, int k);
// ISING_E_STATE unless the graph's device is the current one.
int check_device(const ising_graph* g);

// Work description of one sweep-kernel launch (device pointers).
struct SweepLaunch {
  const uint32_t* d_thr;  // full-schedule threshold table [S][kmax] (unused with rep_thr)
  const uint32_t* rep_thr;  // per-replica fixed thresholds [R][kmax] or null
  int8_t* spins;
  int64_t* cut;
  int64_t* energy;
  uint32_t* flips;
  unsigned long long* stats;
  uint64_t seed;
  int32_t n_replicas;
  int32_t replica_offset;
  int32_t t_begin, t_end;
  int32_t init;
  int32_t block_threads;
};

hipError_t launch_sweep_i8(const ising_graph* g, const SweepLaunch& s, hipStream_t stream);
hipError_t launch_sweep_bp32(const ising_graph* g, const SweepLaunch& s, hipStream_t stream);
hipError_t launch_sweep_bs4(const ising_graph* g, const SweepLaunch& s, hipStream_t stream);
// HBM-resident bit-packed sweeps; words: stream_words_bytes() of device
// memory, bad: one uint32 per 32-replica group.
// part: stream_part_bytes() of per-block flip and RNG counts (needed when s.flips or s.stats).
size_t stream_words_bytes(const Lattice& L, int n_replicas);
size_t stream_part_bytes(const Lattice& L, int n_replicas, bool flips, bool stats);
// cut_part: cut_part_bytes() of scratch for the cut's partial sums, or null
// (then allocated on the stream when needed).
hipError_t launch_sweep_stream(const ising_graph* g, const SweepLaunch& s, uint32_t* words, uint32_t* bad,
                               uint32_t* part, hipStream_t stream, int64_t* cut_part = nullptr);
// Bytes of partial sums launch_cut_energy passes between its two kernels (0:
// one block per replica, none needed).
size_t cut_part_bytes(const Lattice& L, int64_t n_replicas);
hipError_t launch_cut_energy(const ising_graph* g, const int8_t* spins, int64_t n_replicas, int64_t* cut,
                             int64_t* energy, hipStream_t stream, int64_t* part_scratch = nullptr);
hipError_t launch_philox_dump(uint64_t key, const uint32_t* ctr, int64_t m, uint32_t* out, hipStream_t stream);

// A prepared persistent launch over several instances (four-replica
// packings, chosen per instance: layouts[k] = ISING_LAYOUT_I8 or _BS4).
struct BatchPlan {
  int ndim = 2;
  void* d_inst = nullptr;     // per-instance packing and kernel arguments
  void* d_items = nullptr;    // (instance, quad) work items, costliest first
  unsigned int* d_counter = nullptr;
  int n_items = 0;
  size_t lds = 0;
  int grid = 0, block = 0;
};
hipError_t build_batch(const ising_graph* const* graphs, const SweepLaunch* launches, const int* layouts, int n_inst,
                       BatchPlan* plan);
hipError_t run_batch(const BatchPlan& plan, hipStream_t stream);
void free_batch(BatchPlan& plan);

// LDS bytes one block of each sweep kernel needs for a lattice.
size_t sweep_i8_lds_bytes(const Lattice& L);
size_t sweep_bp32_lds_bytes(const Lattice& L);
size_t sweep_bs4_lds_bytes(const Lattice& L);
// The dynamic (state) part of that for the four-replica kernels.
size_t sweep_i8_dyn_lds(const Lattice& L);
size_t sweep_bs4_dyn_lds(const Lattice& L);
// Block size a sweep kernel uses for a requested size (0 = default; 0
// returned when the kernel cannot take the lattice).
int sweep_i8_block(const Lattice& L, int requested);
int sweep_bp32_block(const Lattice& L, int requested);
int sweep_bs4_block(const Lattice& L, int requested);
// The bs4 block size a run of n_replicas takes when none is requested: the
// largest, or about 512 threads where four or more replica quads share a CU
// and two blocks fit its LDS.
int sweep_bs4_default_block(const Lattice& L, int n_replicas, int cus, size_t lds_per_cu);
// The 4 x 4 bit-sliced kernel needs Ly (the second-fastest axis) divisible by 4.
bool sweep_bs4_supported(const Lattice& L);

}  // namespace ising
