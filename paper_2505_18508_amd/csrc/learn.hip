// Learned culling: trajectory features, a 16-64-64-1 ReLU network (forward,
// mean-squared-error gradient, Adam), feature statistics, and rank-and-clone
// of replicas.  All fp32 network arithmetic; every reduction has a fixed
// order, so results are reproducible run to run.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ising.h"
#include "internal.hpp"
#include "philox.hpp"

namespace ising {
namespace {

constexpr int NF = ISING_N_FEATURES;  // 16
constexpr int NH = ISING_MLP_HIDDEN;  // 64
constexpr int P = ISING_MLP_PARAMS;   // 5313
constexpr int OFF_W1 = 0, OFF_B1 = NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH;
static_assert(OFF_B3 + 1 == P, "parameter layout");
constexpr uint32_t kTagMlp = 3u;

// ---------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------
struct FeatArgs {
  Lattice lat;
  const int8_t* w;  // edge weights, edge order
  const int8_t* spins;
  const int64_t* energy;
  const uint32_t* wflips;
  ising_track* track;
  float* feat;
  int32_t sweeps_done, window, n_sweeps, n_checkpoints;
  double beta;
};

constexpr int kFeatBlock = 256;

template <int NDIM>
__global__ void __launch_bounds__(kFeatBlock) k_features(FeatArgs a) {
  __shared__ uint32_t hist[8];
  const Lattice& L = a.lat;
  const int r = blockIdx.x;
  const int8_t* s = a.spins + (size_t)r * L.n;
  if (threadIdx.x < 8) hist[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t Lx = (uint32_t)L.Lx, Ly = (uint32_t)L.Ly, Lz = (uint32_t)L.Lz;
  const uint32_t plane = Lx * Ly;
  uint32_t cnt[7] = {0u, 0u, 0u, 0u, 0u, 0u, 0u};  // wave-uniform counts (lane 0 adds them)
  for (uint32_t base = 0; base < (uint32_t)L.n; base += kFeatBlock) {
    const uint32_t i = base + threadIdx.x;
    int bin = -1;
    if (i < (uint32_t)L.n) {
      const uint32_t line = fdiv(i, L.div_lx);
      const uint32_t x = i - line * Lx;
      const uint32_t z = NDIM == 2 ? 0u : fdiv(line, L.div_ly);
      const uint32_t y = line - z * Ly;
      const uint32_t xp = (x + 1u == Lx) ? i + 1u - Lx : i + 1u;
      const uint32_t xm = (x == 0u) ? i + Lx - 1u : i - 1u;
      const uint32_t yp = (y + 1u == Ly) ? i + Lx - plane : i + Lx;
      const uint32_t ym = (y == 0u) ? i + plane - Lx : i - Lx;
      int f = a.w[(size_t)NDIM * i + 0] * s[xp] + a.w[(size_t)NDIM * xm + 0] * s[xm] +
              a.w[(size_t)NDIM * i + 1] * s[yp] + a.w[(size_t)NDIM * ym + 1] * s[ym];
      if (NDIM == 3) {
        const uint32_t zp = (z + 1u == Lz) ? i - (Lz - 1u) * plane : i + plane;
        const uint32_t zm = (z == 0u) ? i + (Lz - 1u) * plane : i - plane;
        f += a.w[(size_t)NDIM * i + 2] * s[zp] + a.w[(size_t)NDIM * zm + 2] * s[zm];
      }
      bin = (s[i] * f + 6) / 2;  // s_i f_i in {-6, ..., 6}, even
    }
#pragma unroll
    for (int b = 0; b < 7; ++b) cnt[b] += (uint32_t)__popcll(__ballot(bin == b));
  }
  if ((threadIdx.x & 63) == 0)
    for (int b = 0; b < 7; ++b) atomicAdd(&hist[b], cnt[b]);
  __syncthreads();
  if (threadIdx.x != 0) return;

  const double E = (double)NDIM * (double)L.n;
  const double n = (double)L.n;
  const int64_t H = a.energy[r];
  ising_track t = a.track[r];
  const bool first = t.checkpoints == 0;
  const int64_t h_prev = first ? 0 : t.h_prev;
  const int64_t h_min_old = first ? INT64_MAX : t.h_min;
  const int32_t cp = t.checkpoints + 1;
  if (H < h_min_old) {
    t.h_min = H;
    t.last_improve = cp;
  } else {
    t.h_min = h_min_old;
  }
  t.flips_total += a.wflips[r];
  float* o = a.feat + (size_t)r * NF;
  o[0] = (float)((double)H / E);
  o[1] = (float)((double)t.h_min / E);
  o[2] = (float)((double)(H - h_prev) / E);
  o[3] = (float)((double)a.wflips[r] / (n * (double)a.window));
  o[4] = (float)((double)t.flips_total / (n * (double)a.sweeps_done));
  o[5] = (float)a.beta;
  o[6] = (float)((double)a.sweeps_done / (double)a.n_sweeps);
  for (int b = 0; b < 7; ++b) o[7 + b] = (float)((double)hist[b] / n);
  o[14] = (float)log(a.beta);
  o[15] = (float)((double)(cp - t.last_improve) / (double)a.n_checkpoints);
  t.h_prev = H;
  t.checkpoints = cp;
  a.track[r] = t;
}

// ---------------------------------------------------------------------------
// Network
// ---------------------------------------------------------------------------
__global__ void k_mlp_init(uint64_t seed, float* params) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  int fan_in = 0;
  if (i < OFF_B1) fan_in = NF;
  else if (i >= OFF_W2 && i < OFF_B2) fan_in = NH;
  else if (i >= OFF_W3 && i < OFF_B3) fan_in = NH;
  float v = 0.0f;
  if (fan_in) {
    const u32x4 u = philox_ref(seed, (uint32_t)i >> 2, 0u, 0u, kTagMlp);
    const float unit = (float)(u.v[i & 3] >> 8) * 0x1p-24f;  // [0, 1), exact
    v = sqrtf(6.0f / (float)fan_in) * (2.0f * unit - 1.0f);
  }
  params[i] = v;
}

__device__ __forceinline__ void load_params(float* sp, const float* params) {
  for (int k = threadIdx.x; k < P; k += blockDim.x) sp[k] = params[k];
}

// Row b of the batch: x row idx[b] (or b).  A row index outside [0, x_rows)
// reads nothing: z is zero and the caller makes that sample's outputs NaN.
__device__ __forceinline__ bool load_input(float* z, const float* x, int64_t x_rows, const int32_t* idx, int64_t b,
                                           const float* mean, const float* sd) {
  const int64_t row = idx ? (int64_t)idx[b] : b;
  if (row < 0 || row >= x_rows) {
#pragma unroll
    for (int k = 0; k < NF; ++k) z[k] = 0.0f;
    return false;
  }
  const float* xr = x + row * NF;
#pragma unroll
  for (int k = 0; k < NF; ++k) z[k] = mean ? (xr[k] - mean[k]) / sd[k] : xr[k];
  return true;
}

constexpr int kFwdBlock = 256;

__global__ void __launch_bounds__(kFwdBlock) k_mlp_forward(const float* params, const float* x, int64_t x_rows,
                                                          const int32_t* idx, const float* mean, const float* sd,
                                                          int64_t batch, float* y) {
  __shared__ float sp[P];
  load_params(sp, params);
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * kFwdBlock + threadIdx.x;
  if (b >= batch) return;
  float z[NF], h1[NH];
  if (!load_input(z, x, x_rows, idx, b, mean, sd)) {
    y[b] = __builtin_nanf("");
    return;
  }
  for (int j = 0; j < NH; ++j) {
    float acc = sp[OFF_B1 + j];
#pragma unroll
    for (int k = 0; k < NF; ++k) acc = fmaf(sp[OFF_W1 + j * NF + k], z[k], acc);
    h1[j] = fmaxf(acc, 0.0f);
  }
  float out = sp[OFF_B3];
  for (int j = 0; j < NH; ++j) {
    float acc = sp[OFF_B2 + j];
#pragma unroll
    for (int k = 0; k < NH; ++k) acc = fmaf(sp[OFF_W2 + j * NH + k], h1[k], acc);
    out = fmaf(sp[OFF_W3 + j], fmaxf(acc, 0.0f), out);
  }
  y[b] = out;
}

// Loss and gradient: one 64-thread block per 64 samples writes the chunk's
// gradient and squared-error sum to its workspace row; k_mlp_reduce adds the
// rows in block order.
constexpr int kGradChunk = 64;
constexpr int kRow = P + 1;  // gradient + loss per workspace row
constexpr int kPad = NH + 1;

__global__ void __launch_bounds__(kGradChunk) k_mlp_grad(const float* params, const float* x, int64_t x_rows,
                                                        const int32_t* idx, const float* mean, const float* sd,
                                                        const float* target, int64_t batch, float* ws) {
  extern __shared__ float sm[];
  float* sp = sm;                          // [P]
  float* zs = sp + P;                      // [64][NF]
  float* h1s = zs + kGradChunk * NF;       // [64][kPad]
  float* h2s = h1s + kGradChunk * kPad;    // [64][kPad]
  float* d2s = h2s + kGradChunk * kPad;    // [64][kPad]
  float* d1s = d2s + kGradChunk * kPad;    // [64][kPad]
  float* dys = d1s + kGradChunk * kPad;    // [64]
  float* les = dys + kGradChunk;           // [64]
  load_params(sp, params);
  __syncthreads();
  const int s = threadIdx.x;
  const int64_t b = (int64_t)blockIdx.x * kGradChunk + s;
  float* z = zs + s * NF;
  float* h1 = h1s + s * kPad;
  float* h2 = h2s + s * kPad;
  float* d2 = d2s + s * kPad;
  float* d1 = d1s + s * kPad;
  if (b < batch) {
    float zr[NF];
    const bool valid = load_input(zr, x, x_rows, idx, b, mean, sd);
#pragma unroll
    for (int k = 0; k < NF; ++k) z[k] = zr[k];
    for (int j = 0; j < NH; ++j) {
      float acc = sp[OFF_B1 + j];
#pragma unroll
      for (int k = 0; k < NF; ++k) acc = fmaf(sp[OFF_W1 + j * NF + k], zr[k], acc);
      h1[j] = fmaxf(acc, 0.0f);
    }
    float out = sp[OFF_B3];
    for (int j = 0; j < NH; ++j) {
      float acc = sp[OFF_B2 + j];
      for (int k = 0; k < NH; ++k) acc = fmaf(sp[OFF_W2 + j * NH + k], h1[k], acc);
      h2[j] = fmaxf(acc, 0.0f);
      out = fmaf(sp[OFF_W3 + j], h2[j], out);
    }
    // an out-of-range row makes the loss and the gradient NaN (target not read)
    const float t = valid ? (idx ? target[idx[b]] : target[b]) : 0.0f;
    const float err = valid ? out - t : __builtin_nanf("");
    const float dy = 2.0f * err / (float)batch;
    dys[s] = dy;
    les[s] = err * err;
    for (int j = 0; j < NH; ++j) d2[j] = h2[j] > 0.0f ? sp[OFF_W3 + j] * dy : 0.0f;
    for (int k = 0; k < NH; ++k) {
      float acc = 0.0f;
      for (int j = 0; j < NH; ++j) acc = fmaf(sp[OFF_W2 + j * NH + k], d2[j], acc);
      d1[k] = h1[k] > 0.0f ? acc : 0.0f;
    }
  } else {
    for (int k = 0; k < NF; ++k) z[k] = 0.0f;
    for (int j = 0; j < NH; ++j) h1[j] = h2[j] = d2[j] = d1[j] = 0.0f;
    dys[s] = 0.0f;
    les[s] = 0.0f;
  }
  __syncthreads();
  // parameter-parallel sums over the chunk's samples, in sample order
  float* row = ws + (size_t)blockIdx.x * kRow;
  const int j = threadIdx.x;  // hidden unit
  {
    float acc[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) acc[k] = 0.0f;
    float bsum = 0.0f;
    for (int q = 0; q < kGradChunk; ++q) {
      const float d = d1s[q * kPad + j];
      bsum += d;
#pragma unroll
      for (int k = 0; k < NF; ++k) acc[k] = fmaf(d, zs[q * NF + k], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) row[OFF_W1 + j * NF + k] = acc[k];
    row[OFF_B1 + j] = bsum;
  }
  for (int k0 = 0; k0 < NH; k0 += 16) {
    float acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0f;
    for (int q = 0; q < kGradChunk; ++q) {
      const float d = d2s[q * kPad + j];
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[k] = fmaf(d, h1s[q * kPad + k0 + k], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) row[OFF_W2 + j * NH + k0 + k] = acc[k];
  }
  float b2 = 0.0f, w3 = 0.0f;
  for (int q = 0; q < kGradChunk; ++q) {
    b2 += d2s[q * kPad + j];
    w3 = fmaf(dys[q], h2s[q * kPad + j], w3);
  }
  row[OFF_B2 + j] = b2;
  row[OFF_W3 + j] = w3;
  if (j == 0) {
    float b3 = 0.0f, l = 0.0f;
    for (int q = 0; q < kGradChunk; ++q) {
      b3 += dys[q];
      l += les[q];
    }
    row[OFF_B3] = b3;
    row[P] = l;
  }
}

__global__ void k_mlp_reduce(const float* ws, int nblocks, int64_t batch, float* grad, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > P) return;
  float acc = 0.0f;
  for (int k = 0; k < nblocks; ++k) acc += ws[(size_t)k * kRow + p];
  if (p < P) grad[p] = acc;
  else if (loss) *loss = acc / (float)batch;
}

size_t grad_lds_bytes() { return sizeof(float) * (P + kGradChunk * NF + 4 * kGradChunk * kPad + 2 * kGradChunk); }

__global__ void k_adam(float* params, const float* grad, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Column statistics of a [rows][16] table in two passes, as the per-group
// standardisation does: per-block partial sums (double) of x, one block adds
// them in block order into the mean; then per-block partial sums of
// (x - mean)^2, added in block order into the variance.
constexpr int kStatBlock = 256;
constexpr int kStatGrid = 256;

// PASS 0: part[b][c][0] = sum of x; PASS 1: part[b][c][1] = sum of (x - mu[c])^2.
template <int PASS>
__global__ void __launch_bounds__(kStatBlock) k_colstats_partial(const float* x, int64_t rows, const double* mu,
                                                                 double* part) {
  __shared__ double ssum[kStatBlock];
  const int col = threadIdx.x & (NF - 1), lane = threadIdx.x / NF;  // 16 row lanes per column
  const int64_t per = (rows + kStatGrid - 1) / kStatGrid;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < rows ? r0 + per : rows;
  const double m = PASS ? mu[col] : 0.0;
  double s = 0.0;
  for (int64_t r = r0 + lane; r < r1; r += kStatBlock / NF) {
    const double v = (double)x[r * NF + col] - m;
    s += PASS ? v * v : v;
  }
  ssum[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < NF) {
    double t = 0.0;
    for (int l = 0; l < kStatBlock / NF; ++l) t += ssum[l * NF + threadIdx.x];
    part[((size_t)blockIdx.x * NF + threadIdx.x) * 2 + PASS] = t;
  }
}

// One block per (group, column): mean, then the sum of squared deviations,
// each reduced in double by a fixed tree, then the standardised column.
constexpr int kStdBlock = 256;
__global__ void __launch_bounds__(kStdBlock) k_standardize(float* x, int64_t rows, int32_t cols) {
  __shared__ double red[kStdBlock];
  const int64_t g = blockIdx.x / (uint32_t)cols;
  const int32_t c = (int32_t)(blockIdx.x - g * cols);
  float* base = x + (size_t)g * (size_t)rows * (size_t)cols + c;
  const int tid = threadIdx.x;
  auto block_sum = [&](double v) {
    red[tid] = v;
    __syncthreads();
    for (int h = kStdBlock / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
  };
  double s = 0.0;
  for (int64_t r = tid; r < rows; r += kStdBlock) s += (double)base[(size_t)r * cols];
  const double mu = block_sum(s) / (double)rows;
  double q = 0.0;
  for (int64_t r = tid; r < rows; r += kStdBlock) {
    const double d = (double)base[(size_t)r * cols] - mu;
    q += d * d;
  }
  double sd = sqrt(block_sum(q) / (double)rows);
  if (sd < 1e-6) sd = 1e-6;
  for (int64_t r = tid; r < rows; r += kStdBlock)
    base[(size_t)r * cols] = (float)(((double)base[(size_t)r * cols] - mu) / sd);
}

__global__ void k_colstats_mean(const double* part, int64_t rows, double* mu) {
  const int c = threadIdx.x;
  if (c >= NF) return;
  double s = 0.0;
  for (int k = 0; k < kStatGrid; ++k) s += part[((size_t)k * NF + c) * 2 + 0];
  mu[c] = s / (double)rows;
}

__global__ void k_colstats_final(const double* part, int64_t rows, const double* mu, float* mean, float* sd) {
  const int c = threadIdx.x;
  if (c >= NF) return;
  double q = 0.0;
  for (int k = 0; k < kStatGrid; ++k) q += part[((size_t)k * NF + c) * 2 + 1];
  double sdv = sqrt(q / (double)rows);
  if (sdv < 1e-6) sdv = 1e-6;
  mean[c] = (float)mu[c];
  sd[c] = (float)sdv;
}

// ---------------------------------------------------------------------------
// Rank and clone
// ---------------------------------------------------------------------------
constexpr int kRankBlock = 1024;
constexpr int kRankMax = 16384;

__device__ __forceinline__ uint32_t descending_key(float f) {
  if (f != f) return 0xFFFFFFFFu;  // NaN last
  if (f == 0.0f) f = 0.0f;         // -0 and +0 tie
  const uint32_t b = __float_as_uint(f);
  const uint32_t ordered = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // increasing with f
  return ~ordered;  // higher score -> smaller key
}

__global__ void __launch_bounds__(kRankBlock) k_rank(const float* score, int n, int npad, int32_t* order) {
  extern __shared__ unsigned long long keys[];
  for (int i = threadIdx.x; i < npad; i += kRankBlock)
    keys[i] = i < n ? (((unsigned long long)descending_key(score[i]) << 32) | (unsigned)i) : ~0ull;
  __syncthreads();
  for (int k = 2; k <= npad; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < npad; i += kRankBlock) {
        const int l = i ^ j;
        if (l > i) {
          const unsigned long long a = keys[i], b = keys[l];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += kRankBlock) order[i] = (int32_t)(keys[i] & 0xFFFFFFFFu);
}

__global__ void k_clone(const int32_t* order, int n_rep, int64_t n, int8_t* spins, ising_track* track) {
  const int half = n_rep / 2;
  const int pair = blockIdx.y;
  if (pair >= half) return;
  const int src = order[pair], dst = order[n_rep - 1 - pair];
  const int8_t* s = spins + (size_t)src * n;
  int8_t* d = spins + (size_t)dst * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
  if (track && blockIdx.x == 0 && threadIdx.x == 0) track[dst] = track[src];
}

__global__ void k_final_cut_score(const float* gain, const float* feat, int64_t n, double w_over_e, float* score) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) score[i] = (float)(0.5 * (w_over_e - (double)feat[i * NF]) + (double)gain[i]);
}

__global__ void k_cut_labels(const int64_t* final_cut, const int64_t* now_cut, int64_t n, double scale, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)((double)(final_cut[i] - (now_cut ? now_cut[i] : 0)) * scale);
}

__global__ void k_energy_score(const int64_t* energy, int64_t n, float* score) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) score[i] = -(float)energy[i];
}

}  // namespace
}  // namespace ising

using ising::fail;
using ising::fail_hip;

extern "C" {

int ising_features(const ising_graph* g, const int8_t* spins, const int64_t* energy, const uint32_t* window_flips,
                   int64_t n_replicas, ising_track* track, int32_t sweeps_done, int32_t window, int32_t n_sweeps,
                   double beta, int32_t n_checkpoints, float* features, void* stream) {
  if (!g) return fail(ISING_E_ARG, "graph is NULL");
  if (n_replicas < 0 || n_replicas > INT32_MAX) return fail(ISING_E_ARG, "n_replicas out of range");
  if (n_replicas == 0) return ISING_OK;
  if (!spins || !energy || !window_flips || !track || !features) return fail(ISING_E_ARG, "NULL buffer");
  if (window < 1 || sweeps_done < window || n_sweeps < sweeps_done || n_checkpoints < 1)
    return fail(ISING_E_ARG, "need 1 <= window <= sweeps_done <= n_sweeps and n_checkpoints >= 1");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(ISING_E_ARG, "beta must be finite and > 0");
  const int rc = ising::check_device(g);  // the kernel reads the graph's device weights
  if (rc) return rc;
  ising::FeatArgs a;
  a.lat = g->lat;
  a.w = g->d_w;
  a.spins = spins;
  a.energy = energy;
  a.wflips = window_flips;
  a.track = track;
  a.feat = features;
  a.sweeps_done = sweeps_done;
  a.window = window;
  a.n_sweeps = n_sweeps;
  a.n_checkpoints = n_checkpoints;
  a.beta = beta;
  hipStream_t st = (hipStream_t)stream;
  if (g->ndim == 2)
    hipLaunchKernelGGL(ising::k_features<2>, dim3((unsigned)n_replicas), dim3(ising::kFeatBlock), 0, st, a);
  else
    hipLaunchKernelGGL(ising::k_features<3>, dim3((unsigned)n_replicas), dim3(ising::kFeatBlock), 0, st, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ISING_OK : fail_hip(e, "features kernel launch");
}

int ising_mlp_init(uint64_t seed, float* params, void* stream) {
  if (!params) return fail(ISING_E_ARG, "params is NULL");
  hipLaunchKernelGGL(ising::k_mlp_init, dim3((ISING_MLP_PARAMS + 255) / 256), dim3(256), 0, (hipStream_t)stream, seed,
                     params);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ISING_OK : fail_hip(e, "mlp init launch");
}

int ising_mlp_forward(const float* params, const float* x, int64_t x_rows, const int32_t* idx, const float* mean,
                      const float* std, int64_t batch, float* y, void* stream) {
  if (batch < 0 || batch > ((int64_t)1 << 31)) return fail(ISING_E_ARG, "batch out of range");
  if (x_rows < 0) return fail(ISING_E_ARG, "x_rows must be >= 0");
  if (!idx && batch > x_rows) return fail(ISING_E_ARG, "batch exceeds x_rows without idx");
  if (batch == 0) return ISING_OK;
  if (!params || !x || !y) return fail(ISING_E_ARG, "NULL buffer");
  if ((mean == nullptr) != (std == nullptr)) return fail(ISING_E_ARG, "mean and std must both be given or both NULL");
  const int64_t grid = (batch + ising::kFwdBlock - 1) / ising::kFwdBlock;
  hipLaunchKernelGGL(ising::k_mlp_forward, dim3((unsigned)grid), dim3(ising::kFwdBlock), 0, (hipStream_t)stream, params,
                     x, x_rows, idx, mean, std, batch, y);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ISING_OK : fail_hip(e, "mlp forward launch");
}

int64_t ising_mlp_workspace_floats(int64_t batch) {
  if (batch <= 0) return 0;
  return ((batch + ising::kGradChunk - 1) / ising::kGradChunk) * (int64_t)ising::kRow;
}

int ising_mlp_loss_grad(const float* params, const float* x, int64_t x_rows, const int32_t* idx, const float* mean,
                        const float* std, const float* target, int64_t batch, float* grad, float* loss, float* workspace,
                        void* stream) {
  if (batch < 1 || batch > ((int64_t)1 << 31)) return fail(ISING_E_ARG, "batch out of range");
  if (x_rows < 0) return fail(ISING_E_ARG, "x_rows must be >= 0");
  if (!idx && batch > x_rows) return fail(ISING_E_ARG, "batch exceeds x_rows without idx");
  if (!params || !x || !target || !grad || !workspace) return fail(ISING_E_ARG, "NULL buffer");
  if ((mean == nullptr) != (std == nullptr)) return fail(ISING_E_ARG, "mean and std must both be given or both NULL");
  hipStream_t st = (hipStream_t)stream;
  const int64_t nb = (batch + ising::kGradChunk - 1) / ising::kGradChunk;
  const size_t lds = ising::grad_lds_bytes();
  hipError_t e = hipFuncSetAttribute((const void*)ising::k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return fail_hip(e, "mlp grad attribute");
  hipLaunchKernelGGL(ising::k_mlp_grad, dim3((unsigned)nb), dim3(ising::kGradChunk), lds, st, params, x, x_rows, idx, mean,
                     std, target, batch, workspace);
  hipLaunchKernelGGL(ising::k_mlp_reduce, dim3((ISING_MLP_PARAMS + 1 + 255) / 256), dim3(256), 0, st, workspace, (int)nb,
                     batch, grad, loss);
  e = hipGetLastError();
  return e == hipSuccess ? ISING_OK : fail_hip(e, "mlp grad launch");
}

int ising_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, int32_t step, float lr, float beta1,
                    float beta2, float eps, void* stream) {
  if (n < 0 || n > INT32_MAX) return fail(ISING_E_ARG, "n out of range");
  if (n == 0) return ISING_OK;
  if (!params || !grad || !m || !v) return fail(ISING_E_ARG, "NULL buffer");
  if (step < 1) return fail(ISING_E_ARG, "step must be >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) || !(lr >= 0.0f))
    return fail(ISING_E_ARG, "need 0 <= beta1, beta2 < 1, eps > 0, lr >= 0");
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  hipLaunchKernelGGL(ising::k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, params, grad, m,
                     v, n, lr, beta1, beta2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ISING_OK : fail_hip(e, "adam launch");
}

int ising_feature_stats(const float* x, int64_t rows, float* mean, float* std, void* stream) {
  if (rows < 1) return fail(ISING_E_ARG, "rows must be >= 1");
  if (!x || !mean || !std) return fail(ISING_E_ARG, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  double* part = nullptr;
  const size_t n_part = (size_t)ising::kStatGrid * ISING_N_FEATURES * 2;
  const size_t bytes = sizeof(double) * (n_part + ISING_N_FEATURES);
  hipError_t e = hipMallocAsync((void**)&part, bytes, st);
  if (e != hipSuccess) return fail(ISING_E_NOMEM, "stats workspace: %s", hipGetErrorString(e));
  double* mu = part + n_part;
  hipLaunchKernelGGL(ising::k_colstats_partial<0>, dim3(ising::kStatGrid), dim3(ising::kStatBlock), 0, st, x, rows,
                     (const double*)nullptr, part);
  hipLaunchKernelGGL(ising::k_colstats_mean, dim3(1), dim3(64), 0, st, part, rows, mu);
  hipLaunchKernelGGL(ising::k_colstats_partial<1>, dim3(ising::kStatGrid), dim3(ising::kStatBlock), 0, st, x, rows,
                     (const double*)mu, part);
  hipLaunchKernelGGL(ising::k_colstats_final, dim3(1), dim3(64), 0, st, part, rows, (const double*)mu, mean, std);
  e = hipGetLastError();
  (void)hipFreeAsync(part, st);
  return e == hipSuccess ? ISING_OK : fail_hip(e, "feature stats launch");
}

int ising_standardize_groups(float* x, int64_t n_groups, int64_t rows, int32_t cols, void* stream) {
  if (n_groups < 0 || rows < 1 || cols < 1) return fail(ISING_E_ARG, "need n_groups >= 0, rows >= 1, cols >= 1");
  if (n_groups * (int64_t)cols > (int64_t)INT32_MAX) return fail(ISING_E_UNSUPPORTED, "too many groups x columns");
  if (n_groups == 0) return ISING_OK;
  if (!x) return fail(ISING_E_ARG, "NULL buffer");
  hipLaunchKernelGGL(ising::k_standardize, dim3((unsigned)(n_groups * cols)), dim3(ising::kStdBlock), 0,
                     (hipStream_t)stream, x, rows, cols);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ISING_OK : fail_hip(e, "standardize launch");
}

int ising_cull_clone(const float* score, int64_t n_replicas, int64_t n_spins, int8_t* spins, ising_track* track,
                     int32_t* order_out, void* stream) {
  if (n_replicas < 1 || n_replicas > ising::kRankMax)
    return fail(n_replicas > ising::kRankMax ? ISING_E_UNSUPPORTED : ISING_E_ARG, "n_replicas must be in [1, %d]",
                ising::kRankMax);
  if (n_spins < 1) return fail(ISING_E_ARG, "n_spins must be >= 1");
  if (!score || !spins) return fail(ISING_E_ARG, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  int npad = 1;
  while (npad < n_replicas) npad <<= 1;
  if (npad < 2) npad = 2;
  int32_t* order = order_out;
  if (!order) {
    hipError_t e = hipMallocAsync((void**)&order, sizeof(int32_t) * n_replicas, st);
    if (e != hipSuccess) return fail(ISING_E_NOMEM, "order buffer: %s", hipGetErrorString(e));
  }
  const size_t lds = sizeof(unsigned long long) * npad;
  hipError_t e = hipFuncSetAttribute((const void*)ising::k_rank, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(ising::k_rank, dim3(1), dim3(ising::kRankBlock), lds, st, score, (int)n_replicas, npad, order);
    const int half = (int)(n_replicas / 2);
    if (half > 0) {
      int64_t gx = (n_spins + 4095) / 4096;
      if (gx > 64) gx = 64;
      hipLaunchKernelGGL(ising::k_clone, dim3((unsigned)gx, (unsigned)half), dim3(256), 0, st, order, (int)n_replicas,
                         n_spins, spins, track);
    }
    e = hipGetLastError();
  }
  if (!order_out) (void)hipFreeAsync(order, st);
  return e == hipSuccess ? ISING_OK : fail_hip(e, "cull launch");
}

int ising_final_cut_score(const ising_graph* g, const float* gain, const float* features, int64_t n_replicas,
                          float* score, void* stream) {
  if (!g) return fail(ISING_E_ARG, "graph is NULL");
  if (n_replicas < 0 || n_replicas > INT32_MAX) return fail(ISING_E_ARG, "n_replicas out of range");
  if (n_replicas == 0) return ISING_OK;
  if (!gain || !features || !score) return fail(ISING_E_ARG, "NULL buffer");
  const double w_over_e = (double)g->w_total / (double)g->n_edges;
  hipLaunchKernelGGL(ising::k_final_cut_score, dim3((unsigned)((n_replicas + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, gain, features, n_replicas, w_over_e, score);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ISING_OK : fail_hip(e, "final cut score launch");
}

int ising_cut_labels(const int64_t* final_cut, const int64_t* now_cut, int64_t n_replicas, double scale, float* out,
                     void* stream) {
  if (n_replicas < 0 || n_replicas > INT32_MAX) return fail(ISING_E_ARG, "n_replicas out of range");
  if (!std::isfinite(scale)) return fail(ISING_E_ARG, "scale must be finite");
  if (n_replicas == 0) return ISING_OK;
  if (!final_cut || !out) return fail(ISING_E_ARG, "NULL buffer");
  hipLaunchKernelGGL(ising::k_cut_labels, dim3((unsigned)((n_replicas + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     final_cut, now_cut, n_replicas, scale, out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ISING_OK : fail_hip(e, "cut labels launch");
}

int ising_energy_score(const int64_t* energy, int64_t n_replicas, float* score, void* stream) {
  if (n_replicas < 0 || n_replicas > INT32_MAX) return fail(ISING_E_ARG, "n_replicas out of range");
  if (n_replicas == 0) return ISING_OK;
  if (!energy || !score) return fail(ISING_E_ARG, "NULL buffer");
  hipLaunchKernelGGL(ising::k_energy_score, dim3((unsigned)((n_replicas + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, energy, n_replicas, score);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ISING_OK : fail_hip(e, "energy score launch");
}

}  // extern "C"
