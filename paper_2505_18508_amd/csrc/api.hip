// C ABI of the library (declared in include/ising.h): argument checking,
// instance construction, schedules and acceptance thresholds, kernel
// selection.  All GPU work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ising.h"
#include "ising_checks.h"
#include "internal.hpp"
#include "philox.hpp"

using ising::Lattice;

using ising::fail;
using ising::fail_hip;

namespace {

struct DeviceInfo {
  int cus = 0;
  size_t lds_per_block = 0;
};

DeviceInfo device_info(int dev) {
  static std::mutex mu;
  static std::vector<DeviceInfo> cache;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1);
  if (cache[dev].cus == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      cache[dev].cus = prop.multiProcessorCount;
      cache[dev].lds_per_block = prop.sharedMemPerBlock;
    }
  }
  return cache[dev];
}

int check_dims(int32_t ndim, const int32_t* dims) {
  if (ndim != 2 && ndim != 3) return fail(ISING_E_TOPOLOGY, "ndim must be 2 or 3 (got %d)", ndim);
  if (!dims) return fail(ISING_E_ARG, "dims is NULL");
  int64_t n = 1;
  for (int d = 0; d < ndim; ++d) {
    if (dims[d] < 2 || (dims[d] & 1))
      return fail(ISING_E_TOPOLOGY, "dimension %d has length %d; every length must be even and >= 2", d, dims[d]);
    n *= dims[d];
    if (n * ndim >= ((int64_t)1 << 31)) return fail(ISING_E_UNSUPPORTED, "torus too large (n * ndim >= 2^31)");
  }
  return ISING_OK;
}

void generate_weights(int32_t ndim, int64_t n, uint64_t seed, int8_t* out) {
  const int64_t ne = ndim * n;
  for (int64_t blk = 0; blk * 4 < ne; ++blk) {
    const ising::u32x4 u = ising::philox_ref(seed, (uint32_t)blk, 0u, 0u, ising::kTagWeight);
    for (int k = 0; k < 4 && blk * 4 + k < ne; ++k) out[blk * 4 + k] = (u.v[k] >> 31) ? 1 : -1;
  }
}

// Per-site weight sign bits (direction order +x, -x, +y, -y, +z, -z; bit set:
// weight -1), in colour-split order.
std::vector<uint8_t> site_weight_bits(const Lattice& L, const std::vector<int8_t>& w) {
  std::vector<uint8_t> bits(L.n, 0);
  const int nd = L.ndim;
  for (int64_t z = 0; z < L.Lz; ++z)
    for (int64_t y = 0; y < L.Ly; ++y)
      for (int64_t x = 0; x < L.Lx; ++x) {
        auto idx = [&](int64_t xx, int64_t yy, int64_t zz) { return (zz * L.Ly + yy) * L.Lx + xx; };
        const int64_t i = idx(x, y, z);
        int8_t ws[6];
        ws[0] = w[nd * i + 0];
        ws[1] = w[nd * idx((x + L.Lx - 1) % L.Lx, y, z) + 0];
        ws[2] = w[nd * i + 1];
        ws[3] = w[nd * idx(x, (y + L.Ly - 1) % L.Ly, z) + 1];
        if (nd == 3) {
          ws[4] = w[nd * i + 2];
          ws[5] = w[nd * idx(x, y, (z + L.Lz - 1) % L.Lz) + 2];
        }
        uint8_t b = 0;
        for (int d = 0; d < 2 * nd; ++d) b |= (ws[d] < 0 ? 1 : 0) << d;
        int p;
        uint32_t h;
        ising::site_to_split(L, (uint32_t)i, p, h);
        bits[(size_t)p * L.half + h] = b;
      }
  return bits;
}

// struct_size of ising_run_params before replica_thresholds was appended
constexpr size_t kParamsSizeV1 = offsetof(ising_run_params, replica_thresholds);

// The per-replica thresholds of p, NULL for callers of the older struct.
const uint32_t* replica_thr(const ising_run_params* p) {
  return p->struct_size >= sizeof(ising_run_params) ? p->replica_thresholds : nullptr;
}

int check_params(const ising_run_params* p) {
  if (!p) return fail(ISING_E_ARG, "params is NULL");
  if (p->struct_size != sizeof(ising_run_params) && p->struct_size != kParamsSizeV1)
    return fail(ISING_E_ARG, "params.struct_size is %u, this library expects %zu (or %zu)", p->struct_size,
                sizeof(ising_run_params), kParamsSizeV1);
  if (p->n_sweeps < 1) return fail(ISING_E_ARG, "n_sweeps must be >= 1");
  switch (p->schedule) {
    case ISING_SCHED_LINEAR:
      if (!(p->beta0 >= 0.0) || !(p->beta1 >= 0.0) || !std::isfinite(p->beta0) || !std::isfinite(p->beta1))
        return fail(ISING_E_ARG, "linear schedule needs finite beta0, beta1 >= 0");
      break;
    case ISING_SCHED_GEOMETRIC:
      if (!(p->beta0 > 0.0) || !(p->beta1 > 0.0) || !std::isfinite(p->beta0) || !std::isfinite(p->beta1))
        return fail(ISING_E_ARG, "geometric schedule needs finite beta0, beta1 > 0");
      break;
    case ISING_SCHED_TABLE:
      if (!p->beta_table) return fail(ISING_E_ARG, "table schedule needs beta_table");
      for (int32_t t = 0; t < p->n_sweeps; ++t)
        if (!(p->beta_table[t] >= 0.0) || !std::isfinite(p->beta_table[t]))
          return fail(ISING_E_ARG, "beta_table[%d] is not a finite value >= 0", t);
      break;
    default:
      return fail(ISING_E_ARG, "unknown schedule %d", p->schedule);
  }
  return ISING_OK;
}

// Inverse temperature of sweep t and the acceptance thresholds of an energy
// increase of 4k, k = 1..kmax.  The schedule is a reading (the paper fixes the
// trial length in sweeps only); thresholds implement min(1, exp(-beta dE)) for
// a uniform 32-bit word: accept iff u < floor(2^32 exp(-4 k beta)).
double schedule_beta(const ising_run_params* p, int32_t t) {
  if (p->schedule == ISING_SCHED_TABLE) return p->beta_table[t];
  if (p->n_sweeps == 1) return p->beta0;
  const double frac = (double)t / (double)(p->n_sweeps - 1);
  if (p->schedule == ISING_SCHED_LINEAR) return p->beta0 + (p->beta1 - p->beta0) * frac;
  return p->beta0 * std::pow(p->beta1 / p->beta0, frac);
}

using ising::accept_threshold;

void fill_thresholds(const ising_run_params* p, int kmax, uint32_t* out) {
  for (int32_t t = 0; t < p->n_sweeps; ++t) {
    const double beta = schedule_beta(p, t);
    for (int k = 1; k <= kmax; ++k) out[(size_t)t * kmax + (k - 1)] = accept_threshold(beta, k);
  }
}

uint64_t fnv1a(const void* data, size_t bytes) {
  const unsigned char* c = (const unsigned char*)data;
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

constexpr size_t kMaxCachedTables = 64;

bool same_schedule(const ThrCacheEntry& e, const ising_run_params* p, int kmax, double b0, double b1, uint64_t th) {
  return e.schedule == p->schedule && e.n_sweeps == p->n_sweeps && e.kmax == kmax && e.beta0 == b0 &&
         e.beta1 == b1 && e.table_hash == th &&
         (p->schedule != ISING_SCHED_TABLE ||
          std::memcmp(e.table.data(), p->beta_table, sizeof(double) * p->n_sweeps) == 0);
}

// A cached table is usable on `stream` once its upload has completed; a
// stream other than the uploading one waits for that upload's event while it
// is still in flight (a batch plan, made synchronously, waits on the host).
// Called with the graph's lock held.
int use_cached(const ThrCacheEntry& e, hipStream_t stream, bool for_plan, uint32_t** out, bool* owned) {
  if (for_plan) {
    hipError_t err = hipEventSynchronize(e.ready);
    if (err != hipSuccess) return fail_hip(err, "threshold table upload");
  } else if (stream != e.made_on && hipEventQuery(e.ready) == hipErrorNotReady) {
    hipError_t err = hipStreamWaitEvent(stream, e.ready, 0);
    if (err != hipSuccess) return fail_hip(err, "threshold table wait");
  }
  *out = e.d_thr;
  *owned = false;
  return ISING_OK;
}

// Release the host sources of finished uncached uploads.  Lock held.
void reap_uploads(const ising_graph* g) {
  auto& v = g->thr_uploads;
  for (size_t i = 0; i < v.size();) {
    if (hipEventQuery(v[i].done) == hipErrorNotReady) {
      ++i;
      continue;
    }
    (void)hipEventDestroy(v[i].done);
    v[i] = std::move(v.back());
    v.pop_back();
  }
}

// Device threshold table of p's whole schedule, cached on the graph.  Cached
// tables are immutable and freed with the graph; beyond the cache size a
// stream-ordered allocation is made and released after the launch.  No path
// but a batch plan's (for_plan: synchronous, as batch creation is) waits for
// the device: uploads are asynchronous on `stream` from host copies that live
// until the copy has completed.
int threshold_table(const ising_graph* g, const ising_run_params* p, hipStream_t stream, uint32_t** out,
                    bool* owned, bool for_plan = false) {
  const int kmax = g->degree / 2;
  const uint64_t th = p->schedule == ISING_SCHED_TABLE ? fnv1a(p->beta_table, sizeof(double) * p->n_sweeps) : 0;
  const double b0 = p->schedule == ISING_SCHED_TABLE ? 0.0 : p->beta0;
  const double b1 = p->schedule == ISING_SCHED_TABLE ? 0.0 : p->beta1;
  {
    std::lock_guard<std::mutex> lock(g->mu);
    for (const ThrCacheEntry& e : g->thr_cache)
      if (same_schedule(e, p, kmax, b0, b1, th)) return use_cached(e, stream, for_plan, out, owned);
  }
  std::vector<uint32_t> host((size_t)p->n_sweeps * kmax);
  fill_thresholds(p, kmax, host.data());
  const size_t bytes = host.size() * sizeof(uint32_t);
  std::lock_guard<std::mutex> lock(g->mu);
  for (const ThrCacheEntry& e : g->thr_cache)  // another thread may have added it meanwhile
    if (same_schedule(e, p, kmax, b0, b1, th)) return use_cached(e, stream, for_plan, out, owned);
  reap_uploads(g);
  uint32_t* d = nullptr;
  if (for_plan) {  // kept by a batch plan and freed with it
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return fail(ISING_E_NOMEM, "threshold table (%zu bytes): %s", bytes, hipGetErrorString(e));
    e = hipMemcpy(d, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return fail_hip(e, "threshold table upload");
    }
    *out = d;
    *owned = true;
    return ISING_OK;
  }
  const bool cache = g->thr_cache.size() < kMaxCachedTables;
  hipError_t e = cache ? hipMalloc(&d, bytes) : hipMallocAsync((void**)&d, bytes, stream);
  if (e != hipSuccess) return fail(ISING_E_NOMEM, "threshold table (%zu bytes): %s", bytes, hipGetErrorString(e));
  hipEvent_t ev = nullptr;
  e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMemcpyAsync(d, host.data(), bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(ev, stream);
  if (e != hipSuccess) {
    // the copy may be in flight: wait for the stream before the host source goes
    (void)hipStreamSynchronize(stream);
    if (ev) (void)hipEventDestroy(ev);
    if (cache) (void)hipFree(d);
    else (void)hipFreeAsync(d, stream);
    return fail_hip(e, "threshold table upload");
  }
  if (cache) {
    std::vector<double> table;
    if (p->schedule == ISING_SCHED_TABLE) table.assign(p->beta_table, p->beta_table + p->n_sweeps);
    g->thr_cache.push_back(ThrCacheEntry{p->schedule, p->n_sweeps, kmax, b0, b1, th, std::move(table),
                                         std::move(host), d, ev, stream});
    *owned = false;
  } else {
    g->thr_uploads.push_back(ThrUpload{std::move(host), ev});
    *owned = true;
  }
  *out = d;
  return ISING_OK;
}

using ising::check_device;

}  // namespace

namespace ising {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int fail_hip(hipError_t e, const char* what) { return fail(ISING_E_HIP, "%s: %s", what, hipGetErrorString(e)); }

uint32_t accept_threshold(double beta, int k) {
  const double scaled = std::ldexp(std::exp(-(double)(4 * k) * beta), 32);
  return scaled >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)std::floor(scaled);
}

int check_device(const ising_graph* g) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (dev != g->device)
    return fail(ISING_E_STATE, "graph lives on device %d but device %d is current", g->device, dev);
  return ISING_OK;
}

// chains.hip (declared here, not in internal.hpp: only this file calls it)
hipError_t launch_compare_chains(int64_t n, const uint32_t* u, const uint32_t* sel2, const uint32_t* sel3,
                                 uint32_t T1, uint32_t T2, uint32_t T3, uint32_t* out, hipStream_t stream);
}  // namespace ising

extern "C" {

const char* ising_last_error(void) { return ising::g_last_error.c_str(); }

int ising_generate_weights(int32_t ndim, const int32_t* dims, uint64_t weight_seed, int8_t* host_out) {
  int rc = check_dims(ndim, dims);
  if (rc) return rc;
  if (!host_out) return fail(ISING_E_ARG, "host_out is NULL");
  const Lattice L = ising::make_lattice(ndim, dims);
  generate_weights(ndim, L.n, weight_seed, host_out);
  return ISING_OK;
}

int ising_create_graph(int32_t ndim, const int32_t* dims, uint64_t weight_seed, const int8_t* weights,
                       ising_graph** out) {
  if (!out) return fail(ISING_E_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_dims(ndim, dims);
  if (rc) return rc;
  ising_graph* g = new (std::nothrow) ising_graph();
  if (!g) return fail(ISING_E_NOMEM, "graph handle");
  g->ndim = ndim;
  for (int d = 0; d < 3; ++d) g->dims[d] = d < ndim ? dims[d] : 0;
  g->lat = ising::make_lattice(ndim, dims);
  g->n = g->lat.n;
  g->n_edges = (int64_t)ndim * g->n;
  g->degree = 2 * ndim;
  try {
    g->w_host.resize((size_t)g->n_edges);
  } catch (...) {
    delete g;
    return fail(ISING_E_NOMEM, "host weights");
  }
  if (weights) {
    for (int64_t e = 0; e < g->n_edges; ++e) {
      if (weights[e] != 1 && weights[e] != -1) {
        delete g;
        return fail(ISING_E_ARG, "weights[%lld] = %d; weights must be +1 or -1", (long long)e, (int)weights[e]);
      }
    }
    std::memcpy(g->w_host.data(), weights, (size_t)g->n_edges);
  } else {
    generate_weights(ndim, g->n, weight_seed, g->w_host.data());
  }
  g->w_total = 0;
  for (int8_t v : g->w_host) g->w_total += v;
  std::vector<uint8_t> bits = site_weight_bits(g->lat, g->w_host);

  hipError_t e = hipGetDevice(&g->device);
  if (e != hipSuccess) {
    delete g;
    return fail_hip(e, "hipGetDevice");
  }
  e = hipMalloc(&g->d_w, (size_t)g->n_edges);
  if (e == hipSuccess) e = hipMalloc(&g->d_wbits, (size_t)g->n);
  if (e != hipSuccess) {
    (void)hipFree(g->d_w);
    (void)hipFree(g->d_wbits);
    delete g;
    return fail(e == hipErrorOutOfMemory ? ISING_E_NOMEM : ISING_E_HIP, "graph device tables: %s",
                hipGetErrorString(e));
  }
  e = hipMemcpy(g->d_w, g->w_host.data(), (size_t)g->n_edges, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g->d_wbits, bits.data(), (size_t)g->n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(g->d_w);
    (void)hipFree(g->d_wbits);
    delete g;
    return fail_hip(e, "graph upload");
  }
  *out = g;
  return ISING_OK;
}

void ising_destroy_graph(ising_graph* g) {
  if (!g) return;
  (void)hipFree(g->d_w);
  (void)hipFree(g->d_wbits);
  for (ThrCacheEntry& e : g->thr_cache) {
    (void)hipFree(e.d_thr);  // waits for the device, uploads included
    (void)hipEventDestroy(e.ready);
  }
  for (ThrUpload& u : g->thr_uploads) {
    (void)hipEventSynchronize(u.done);
    (void)hipEventDestroy(u.done);
  }
  delete g;
}

int ising_graph_info(const ising_graph* g, int64_t* n_spins, int64_t* n_edges, int64_t* w_total, int32_t* degree) {
  if (!g) return fail(ISING_E_ARG, "graph is NULL");
  if (n_spins) *n_spins = g->n;
  if (n_edges) *n_edges = g->n_edges;
  if (w_total) *w_total = g->w_total;
  if (degree) *degree = g->degree;
  return ISING_OK;
}

int ising_graph_weights(const ising_graph* g, int8_t* host_out) {
  if (!g) return fail(ISING_E_ARG, "graph is NULL");
  if (!host_out) return fail(ISING_E_ARG, "host_out is NULL");
  std::memcpy(host_out, g->w_host.data(), (size_t)g->n_edges);
  return ISING_OK;
}

int ising_thresholds(const ising_run_params* p, int32_t degree, uint32_t* host_out) {
  int rc = check_params(p);
  if (rc) return rc;
  if (degree != 4 && degree != 6) return fail(ISING_E_ARG, "degree must be 4 or 6");
  if (!host_out) return fail(ISING_E_ARG, "host_out is NULL");
  fill_thresholds(p, degree / 2, host_out);
  return ISING_OK;
}

int ising_schedule_beta(const ising_run_params* p, int32_t t, double* beta_out) {
  int rc = check_params(p);
  if (rc) return rc;
  if (t < 0 || t >= p->n_sweeps) return fail(ISING_E_ARG, "sweep %d outside [0, %d)", t, p->n_sweeps);
  if (!beta_out) return fail(ISING_E_ARG, "beta_out is NULL");
  *beta_out = schedule_beta(p, t);
  return ISING_OK;
}

}  // extern "C"

namespace {

// Validation shared by single runs and batches; picks the layout.
int check_run(const ising_graph* g, const ising_run_params* p, const int8_t* spins_inout, int* layout_out) {
  if (!g) return fail(ISING_E_ARG, "graph is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (p->n_replicas < 1) return fail(ISING_E_ARG, "n_replicas must be >= 1");
  if (p->sweep_begin < 0 || p->sweep_end > p->n_sweeps || p->sweep_begin >= p->sweep_end)
    return fail(ISING_E_ARG, "window [%d, %d) is not inside [0, %d)", p->sweep_begin, p->sweep_end, p->n_sweeps);
  if (p->init_spins && p->sweep_begin != 0) return fail(ISING_E_ARG, "init_spins needs sweep_begin == 0");
  if (!spins_inout) return fail(ISING_E_ARG, "spins_inout is NULL");
  if (p->replica_offset < 0 || (int64_t)p->replica_offset + p->n_replicas > INT32_MAX)
    return fail(ISING_E_ARG, "replica_offset out of range");
  if (p->replica_offset % 4 != 0) return fail(ISING_E_ARG, "replica_offset must be a multiple of 4");
  rc = check_device(g);
  if (rc) return rc;
  const DeviceInfo dev = device_info(g->device);
  const bool i8_fits = ising::sweep_i8_block(g->lat, p->block_threads) > 0 &&
                       ising::sweep_i8_lds_bytes(g->lat) <= dev.lds_per_block;
  const bool bp_fits = ising::sweep_bp32_block(g->lat, p->block_threads) > 0 &&
                       ising::sweep_bp32_lds_bytes(g->lat) <= dev.lds_per_block;
  const bool bs4_fits = ising::sweep_bs4_block(g->lat, p->block_threads) > 0 &&
                        ising::sweep_bs4_lds_bytes(g->lat) <= dev.lds_per_block;
  int layout = p->layout;
  const bool per_replica = replica_thr(p) != nullptr;
  if (per_replica && layout == ISING_LAYOUT_AUTO) layout = bs4_fits ? ISING_LAYOUT_BS4 : ISING_LAYOUT_I8;
  if (per_replica && layout != ISING_LAYOUT_BS4 && layout != ISING_LAYOUT_I8)
    return fail(ISING_E_UNSUPPORTED, "per-replica thresholds need layout I8 or BS4");
  if (per_replica && p->stats_out)
    return fail(ISING_E_UNSUPPORTED, "RNG statistics are not collected with per-replica thresholds");
  if (layout == ISING_LAYOUT_AUTO) {
    // 32 replicas per block wins per attempt, but only fills the chip with at
    // least one group per compute unit; below that, four replicas per block,
    // bit-sliced over four sites where the lattice allows it
    const int64_t groups = ((int64_t)p->n_replicas + 31) / 32;
    if (bp_fits && (groups >= dev.cus || (!i8_fits && !bs4_fits)))
      layout = ISING_LAYOUT_BP32;
    else if (bs4_fits)
      layout = ISING_LAYOUT_BS4;
    else if (i8_fits)
      layout = ISING_LAYOUT_I8;
    else
      layout = ISING_LAYOUT_STREAM;
  }
  if (layout == ISING_LAYOUT_STREAM) {
    if (g->lat.hx < 1) return fail(ISING_E_UNSUPPORTED, "torus too small");
    *layout_out = layout;
    return ISING_OK;
  }
  if (layout != ISING_LAYOUT_I8 && layout != ISING_LAYOUT_BP32 && layout != ISING_LAYOUT_BS4)
    return fail(ISING_E_ARG, "unknown layout %d", p->layout);
  if (layout == ISING_LAYOUT_BS4 && !ising::sweep_bs4_supported(g->lat))
    return fail(ISING_E_UNSUPPORTED, "torus too small for layout %d", layout);
  if ((layout == ISING_LAYOUT_I8 && !i8_fits) || (layout == ISING_LAYOUT_BP32 && !bp_fits) ||
      (layout == ISING_LAYOUT_BS4 && !bs4_fits))
    return fail(ISING_E_UNSUPPORTED, "torus of %lld sites does not fit the on-chip sweep kernel of layout %d",
                (long long)g->n, layout);
  *layout_out = layout;
  return ISING_OK;
}

ising::SweepLaunch make_launch(const ising_run_params* p, const uint32_t* d_thr, int8_t* spins, int64_t* cut,
                               int64_t* energy, uint32_t* flips) {
  ising::SweepLaunch s;
  s.d_thr = d_thr;
  s.rep_thr = replica_thr(p);
  s.spins = spins;
  s.cut = cut;
  s.energy = energy;
  s.flips = flips;
  s.stats = (unsigned long long*)p->stats_out;
  s.seed = p->seed;
  s.n_replicas = p->n_replicas;
  s.replica_offset = p->replica_offset;
  s.t_begin = p->sweep_begin;
  s.t_end = p->sweep_end;
  s.init = p->init_spins ? 1 : 0;
  s.block_threads = p->block_threads;
  return s;
}

// The sweep launch of a checked run (layout resolved); the streamed layout
// takes its working state (words, input flags, counters) from the caller.
hipError_t dispatch_run(const ising_graph* g, const ising_run_params* p, int layout, ising::SweepLaunch& s,
                        uint32_t* words, uint32_t* bad, uint32_t* part, hipStream_t st, int64_t* cut_part = nullptr) {
  if (layout == ISING_LAYOUT_BS4 && s.block_threads == 0)
    s.block_threads = ising::sweep_bs4_default_block(g->lat, p->n_replicas, device_info(g->device).cus,
                                                     device_info(g->device).lds_per_block);
  if (layout == ISING_LAYOUT_STREAM) return ising::launch_sweep_stream(g, s, words, bad, part, st, cut_part);
  return layout == ISING_LAYOUT_BP32  ? ising::launch_sweep_bp32(g, s, st)
         : layout == ISING_LAYOUT_BS4 ? ising::launch_sweep_bs4(g, s, st)
                                      : ising::launch_sweep_i8(g, s, st);
}

// ---------------------------------------------------------------------------
// Scratch of ising_run_trials_noalloc: a fixed array in device memory (one
// copy per GPU, held until the process ends).  Host code never uses the
// array's name as an address: its device address comes from
// hipGetSymbolAddress, once per device with that device current.
constexpr size_t kScratchBytes = ISING_NOALLOC_SCRATCH_BYTES;
constexpr int kScratchDevices = 64;
constexpr int kFillWords = 960;  // words per fill launch, passed as kernel arguments

struct FillChunk {
  uint32_t n;
  uint32_t w[kFillWords];
};

__global__ void k_fill_words(uint32_t* dst, FillChunk c) {
  for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.w[i];
}

}  // namespace

static __device__ __align__(256) uint32_t scratch[kScratchBytes / sizeof(uint32_t)];

namespace {

std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kScratchDevices];

// Device address of the scratch array on device dev (the current device).
int scratch_on(int dev, uint32_t** out) {
  if (dev < 0 || dev >= kScratchDevices) return fail(ISING_E_UNSUPPORTED, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail_hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch_ptr[dev] = (uint32_t*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return ISING_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct ising_batch {
  ising::BatchPlan plan;
  std::vector<uint32_t*> owned_tables;
  int64_t attempts = 0;
  int device = 0;
};

extern "C" {

int ising_select_layout(const ising_graph* g, const ising_run_params* p, int32_t* layout_out) {
  if (!layout_out) return fail(ISING_E_ARG, "layout_out is NULL");
  int8_t placeholder = 0;  // validation only: no spins are read
  int layout = 0;
  const int rc = check_run(g, p, &placeholder, &layout);
  if (rc) return rc;
  *layout_out = layout;
  return ISING_OK;
}

int ising_run_trials(const ising_graph* g, const ising_run_params* p, int8_t* spins_inout, int64_t* cut_out,
                     int64_t* energy_out, uint32_t* flips_out, void* stream) {
  int layout = 0;
  int rc = check_run(g, p, spins_inout, &layout);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  uint32_t* d_thr = nullptr;
  bool owned = false;
  if (!replica_thr(p)) {  // per-replica thresholds replace the schedule's table
    rc = threshold_table(g, p, st, &d_thr, &owned);
    if (rc) return rc;
  }
  ising::SweepLaunch s = make_launch(p, d_thr, spins_inout, cut_out, energy_out, flips_out);
  hipError_t e;
  if (layout == ISING_LAYOUT_STREAM) {
    // stream-ordered working state: the words of every 32-replica group and their input flags
    const size_t wbytes = ising::stream_words_bytes(g->lat, p->n_replicas);
    const size_t groups = ((size_t)p->n_replicas + 31) / 32;
    const size_t pbytes = ising::stream_part_bytes(g->lat, p->n_replicas, s.flips != nullptr, s.stats != nullptr);
    uint32_t* words = nullptr;
    uint32_t* bad = nullptr;
    uint32_t* part = nullptr;
    e = hipMallocAsync((void**)&words, wbytes, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&bad, sizeof(uint32_t) * groups, st);
    if (e == hipSuccess && pbytes) e = hipMallocAsync((void**)&part, pbytes, st);
    if (e != hipSuccess) {
      if (words) (void)hipFreeAsync(words, st);
      if (bad) (void)hipFreeAsync(bad, st);
      if (owned) (void)hipFreeAsync(d_thr, st);
      return fail(ISING_E_NOMEM, "streamed state (%zu bytes): %s", wbytes, hipGetErrorString(e));
    }
    e = dispatch_run(g, p, layout, s, words, bad, part, st);
    (void)hipFreeAsync(words, st);
    (void)hipFreeAsync(bad, st);
    if (part) (void)hipFreeAsync(part, st);
  } else {
    e = dispatch_run(g, p, layout, s, nullptr, nullptr, nullptr, st);
  }
  if (owned) (void)hipFreeAsync(d_thr, st);
  if (e != hipSuccess) return fail_hip(e, "sweep kernel launch");
  return ISING_OK;
}

int ising_run_trials_noalloc(const ising_graph* g, const ising_run_params* p, int8_t* spins_inout, int64_t* cut_out,
                             int64_t* energy_out, uint32_t* flips_out, void* stream) {
  int layout = 0;
  int rc = check_run(g, p, spins_inout, &layout);
  if (rc) return rc;
  const int kmax = g->degree / 2;
  const bool per_replica = replica_thr(p) != nullptr;
  // scratch plan: the window's threshold rows, then (streamed layout) the
  // words of every 32-replica group, their input flags and counters
  const size_t rows = per_replica ? 0 : (size_t)(p->sweep_end - p->sweep_begin) * (size_t)kmax;
  const size_t off_words = round256(rows * sizeof(uint32_t));
  size_t off_bad = off_words, off_part = off_words, off_cut = off_words, total = off_words;
  if (layout == ISING_LAYOUT_STREAM) {
    const size_t groups = ((size_t)p->n_replicas + 31) / 32;
    off_bad = off_words + round256(ising::stream_words_bytes(g->lat, p->n_replicas));
    off_part = off_bad + round256(sizeof(uint32_t) * groups);
    off_cut = off_part + round256(ising::stream_part_bytes(g->lat, p->n_replicas, flips_out != nullptr,
                                                           p->stats_out != nullptr));
    total = off_cut + round256(cut_out || energy_out ? ising::cut_part_bytes(g->lat, p->n_replicas) : 0);
  }
  if (total > kScratchBytes)
    return fail(ISING_E_UNSUPPORTED, "this run needs %zu bytes of scratch; ising_run_trials_noalloc has %zu", total,
                kScratchBytes);
  uint32_t* base = nullptr;
  rc = scratch_on(g->device, &base);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t* d_thr = nullptr;
  if (!per_replica) {
    // rows t = sweep_begin .. sweep_end-1 of the table ising_thresholds gives,
    // carried by the fill launches' arguments: nothing on the host outlives the call
    FillChunk c;
    for (size_t i0 = 0; i0 < rows; i0 += kFillWords) {
      c.n = (uint32_t)(rows - i0 < (size_t)kFillWords ? rows - i0 : (size_t)kFillWords);
      for (uint32_t j = 0; j < c.n; ++j) {
        const size_t i = i0 + j;
        const int32_t t = p->sweep_begin + (int32_t)(i / (size_t)kmax);
        c.w[j] = ising::accept_threshold(schedule_beta(p, t), (int)(i % (size_t)kmax) + 1);
      }
      hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(256), 0, st, base + i0, c);
    }
    // the sweep kernels read row t at thr + t kmax, t in [sweep_begin, sweep_end)
    d_thr = (const uint32_t*)((uintptr_t)base - (uintptr_t)p->sweep_begin * (uintptr_t)kmax * sizeof(uint32_t));
  }
  ising::SweepLaunch s = make_launch(p, d_thr, spins_inout, cut_out, energy_out, flips_out);
  uint8_t* b8 = (uint8_t*)base;
  hipError_t e = dispatch_run(g, p, layout, s, (uint32_t*)(b8 + off_words), (uint32_t*)(b8 + off_bad),
                              (uint32_t*)(b8 + off_part), st, (int64_t*)(b8 + off_cut));
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(e, "sweep kernel launch");
  return ISING_OK;
}

int ising_batch_create(int32_t n_inst, const ising_graph* const* graphs, const ising_run_params* params,
                       int8_t* const* spins, int64_t* const* cut_out, int64_t* const* energy_out,
                       uint32_t* const* flips_out, ising_batch** out) {
  if (!out) return fail(ISING_E_ARG, "out is NULL");
  *out = nullptr;
  if (n_inst < 1 || !graphs || !params || !spins) return fail(ISING_E_ARG, "need n_inst >= 1 and graphs, params, spins");
  ising_batch* b = new (std::nothrow) ising_batch();
  if (!b) return fail(ISING_E_NOMEM, "batch handle");
  std::vector<ising::SweepLaunch> launches((size_t)n_inst);
  std::vector<int> layouts((size_t)n_inst);
  auto bail = [&](int code) {
    for (uint32_t* t : b->owned_tables) (void)hipFree(t);
    delete b;
    return code;
  };
  for (int k = 0; k < n_inst; ++k) {
    const ising_graph* g = graphs[k];
    const ising_run_params* p = &params[k];
    int layout = 0;
    int rc = check_run(g, p, spins[k], &layout);
    if (rc) return bail(rc);
    if (g->ndim != graphs[0]->ndim) return bail(fail(ISING_E_ARG, "instances of a batch must share ndim"));
    if (p->layout != ISING_LAYOUT_AUTO && p->layout != ISING_LAYOUT_I8 && p->layout != ISING_LAYOUT_BS4)
      return bail(fail(ISING_E_UNSUPPORTED, "batches use the four-replica layouts (i8, bs4)"));
    const size_t lds_max = device_info(g->device).lds_per_block;
    const bool bs4_ok = ising::sweep_bs4_block(g->lat, 0) > 0 && ising::sweep_bs4_lds_bytes(g->lat) <= lds_max;
    const bool i8_ok = ising::sweep_i8_block(g->lat, 0) > 0 && ising::sweep_i8_lds_bytes(g->lat) <= lds_max;
    int lay = p->layout == ISING_LAYOUT_AUTO ? (bs4_ok ? ISING_LAYOUT_BS4 : ISING_LAYOUT_I8) : p->layout;
    if ((lay == ISING_LAYOUT_BS4 && !bs4_ok) || (lay == ISING_LAYOUT_I8 && !i8_ok))
      return bail(fail(ISING_E_UNSUPPORTED, "instance %d does not fit the four-replica kernel of layout %d", k, lay));
    layouts[(size_t)k] = lay;
    if (p->stats_out) return bail(fail(ISING_E_UNSUPPORTED, "batches do not collect RNG statistics"));
    uint32_t* d_thr = nullptr;
    bool owned = false;
    if (!replica_thr(p)) {  // per-replica thresholds replace the schedule's table
      rc = threshold_table(g, p, nullptr, &d_thr, &owned, true);
      if (rc) return bail(rc);
      if (owned) b->owned_tables.push_back(d_thr);  // kept for the plan's lifetime
    }
    launches[(size_t)k] = make_launch(p, d_thr, spins[k], cut_out ? cut_out[k] : nullptr,
                                      energy_out ? energy_out[k] : nullptr, flips_out ? flips_out[k] : nullptr);
    b->attempts += (int64_t)p->n_replicas * g->n * (p->sweep_end - p->sweep_begin);
  }
  b->device = graphs[0]->device;
  hipError_t e = ising::build_batch(graphs, launches.data(), layouts.data(), n_inst, &b->plan);
  if (e != hipSuccess) {
    ising::free_batch(b->plan);
    return bail(fail_hip(e, "batch plan"));
  }
  *out = b;
  return ISING_OK;
}

int ising_batch_run(ising_batch* b, void* stream) {
  if (!b) return fail(ISING_E_ARG, "batch is NULL");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (dev != b->device) return fail(ISING_E_STATE, "batch lives on device %d but device %d is current", b->device, dev);
  e = ising::run_batch(b->plan, (hipStream_t)stream);
  return e == hipSuccess ? ISING_OK : fail_hip(e, "batch launch");
}

int ising_batch_info(const ising_batch* b, int64_t* n_items, int64_t* attempts, int32_t* grid, int32_t* block) {
  if (!b) return fail(ISING_E_ARG, "batch is NULL");
  if (n_items) *n_items = b->plan.n_items;
  if (attempts) *attempts = b->attempts;
  if (grid) *grid = b->plan.grid;
  if (block) *block = b->plan.block;
  return ISING_OK;
}

void ising_batch_destroy(ising_batch* b) {
  if (!b) return;
  ising::free_batch(b->plan);
  for (uint32_t* t : b->owned_tables) (void)hipFree(t);
  delete b;
}

int ising_eval_cut(const ising_graph* g, const int8_t* spins, int64_t n_replicas, int64_t* cut_out,
                   int64_t* energy_out, void* stream) {
  if (!g) return fail(ISING_E_ARG, "graph is NULL");
  if (n_replicas < 0 || n_replicas > INT32_MAX) return fail(ISING_E_ARG, "n_replicas out of range");
  if (n_replicas > 0 && !spins) return fail(ISING_E_ARG, "spins is NULL");
  int rc = check_device(g);
  if (rc) return rc;
  hipError_t e = ising::launch_cut_energy(g, spins, n_replicas, cut_out, energy_out, (hipStream_t)stream);
  if (e == hipErrorOutOfMemory) return fail(ISING_E_NOMEM, "cut scratch: %s", hipGetErrorString(e));
  if (e != hipSuccess) return fail_hip(e, "cut kernel launch");
  return ISING_OK;
}

int ising_philox_dump(uint64_t key, const uint32_t* ctr, int64_t m, uint32_t* out, void* stream) {
  if (m < 0 || m > ((int64_t)1 << 31)) return fail(ISING_E_ARG, "m out of range");
  if (m > 0 && (!ctr || !out)) return fail(ISING_E_ARG, "ctr or out is NULL");
  hipError_t e = ising::launch_philox_dump(key, ctr, m, out, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "philox kernel launch");
  return ISING_OK;
}

int ising_compare_chains(int64_t n, const uint32_t* u, const uint32_t* sel2, const uint32_t* sel3, uint32_t T1,
                         uint32_t T2, uint32_t T3, uint32_t* out, void* stream) {
  if (n < 0 || n > ((int64_t)1 << 31)) return fail(ISING_E_ARG, "n out of range");
  if (n > 0 && (!u || !sel2 || !sel3 || !out)) return fail(ISING_E_ARG, "u, sel2, sel3 or out is NULL");
  hipError_t e = ising::launch_compare_chains(n, u, sel2, sel3, T1, T2, T3, out, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "compare-chain kernel launch");
  return ISING_OK;
}

}  // extern "C"
