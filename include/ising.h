/*
 * ising.h -- C ABI of the MI355X (gfx950) library for replica-parallel
 * checkerboard Metropolis annealing on +/-1-weighted toroidal Ising /
 * Max-Cut instances.
 *
 * Problem (paper, Section II): maximise the cut of eq. (1),
 *     cut(x) = 1/2 sum_{i<j} w_ij (1 - x_i x_j),  x in {-1,+1}^n,
 * which is the same as minimising the Ising energy of eq. (2) with
 * J_ij = -w_ij and h_i = 0:  H(s) = sum_{i<j} w_ij s_i s_j = W_total - 2 cut(s),
 * every edge counted once.  Instances (Section I; Appendix A, Fig. 2) are
 * toroidal grids with nearest-neighbour couplings w_ij in {-1,+1}; the 3-D
 * cubic torus (six neighbours) is the same family with one more axis.
 * A trial (Section III) is a run of S sweeps whose state is read out at its
 * end; trial length in sweeps is its only parameter.  The paper withholds its
 * own update rule, so a sweep here is one checkerboard Metropolis pass:
 * every site of colour 0, then every site of colour 1, each proposing one
 * flip, accepted when the energy change dE <= 0 or when a Philox4x32-10 word
 * u < floor(2^32 exp(-beta_t dE)).
 *
 * Conventions shared by every entry point
 *  - Every function returns ISING_OK (0) or a negative ISING_E_* code; no C++
 *    exception crosses this boundary.  ising_last_error() gives a message for
 *    the last failing call on the calling thread.
 *  - Argument errors are reported synchronously.  GPU work is enqueued on the
 *    caller's HIP stream (`stream` is a hipStream_t; NULL = the null stream)
 *    and returns before it completes; a fault in it surfaces as ISING_E_HIP
 *    from a later call or from the caller's own synchronisation.
 *  - Spin buffers use the canonical layout: int8 [R][n], row-major per
 *    replica, value +1 or -1, site i = row-major index of its coordinates
 *    (2-D {rows, cols}: i = r*cols + c; 3-D {Lz, Ly, Lx}: i = (z*Ly + y)*Lx + x).
 *    Edge e = ndim*i + d joins site i to its +1 neighbour along the d-th
 *    fastest axis (2-D: d = 0 column, d = 1 row; 3-D: d = 0 x, 1 y, 2 z).
 *  - The caller owns every buffer it passes; the library never frees them.
 *    Device pointers must be device memory of the current HIP device.
 *  - Random numbers: Philox4x32-10 with key = seed (low word, high word) and
 *    counter (c0, c1, c2, c3); tags in c3: 0 Metropolis draw (c0 = site,
 *    c1 = sweep, c2 = replica >> 2, word replica & 3), 1 initial spin (c0 =
 *    site, c1 = 0, c2 = replica >> 2, word replica & 3, +1 iff top bit set),
 *    2 edge weight (c0 = edge >> 2, c1 = c2 = 0, word edge & 3, +1 iff top
 *    bit set).  Trajectories are therefore reproducible bit for bit and do
 *    not depend on launch shape or packing.
 */
#ifndef ISING_H
#define ISING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ISING_OK = 0,
  ISING_E_ARG = -1,          /* invalid argument (value, pointer or range)          */
  ISING_E_TOPOLOGY = -2,     /* torus shape not supported (odd or < 2 dimension)    */
  ISING_E_NOMEM = -3,        /* host or device allocation failed                    */
  ISING_E_HIP = -4,          /* HIP runtime error (includes errors of earlier work) */
  ISING_E_UNSUPPORTED = -5,  /* valid request the library cannot run (e.g. too large) */
  ISING_E_STATE = -6         /* object in the wrong state for the call              */
};

enum { ISING_SCHED_LINEAR = 0, ISING_SCHED_GEOMETRIC = 1, ISING_SCHED_TABLE = 2 };

/* Internal packing of the replicas; results do not depend on it. */
enum {
  ISING_LAYOUT_AUTO = 0,  /* library chooses by a fixed rule (ising_select_layout) */
  ISING_LAYOUT_I8 = 1,    /* 4 replicas per 32-bit word: spin + maintained field */
  ISING_LAYOUT_BP32 = 2,  /* 32 replicas per 32-bit word: one spin bit each      */
  ISING_LAYOUT_STREAM = 3, /* 32 replicas per word, state in HBM, one launch per */
                           /* colour half-sweep (lattices too large for LDS)     */
  ISING_LAYOUT_BS4 = 4     /* 4 replicas x 4 sites per 16-bit word, bit-sliced;  */
                           /* any even torus that fits a block's LDS             */
};

/* A cut or energy that could not be computed because the replica's spins
 * held a value other than +1 / -1. */
#define ISING_INVALID_VALUE INT64_MIN

typedef struct ising_graph ising_graph;

/*
 * Build a torus instance (paper, Section I and Appendix A: toroidal grid,
 * nearest-neighbour +/-1 couplings, periodic boundaries).
 *   ndim         2 or 3.
 *   dims         host int32[ndim]: 2-D {rows, cols}, 3-D {Lz, Ly, Lx}; every
 *                entry even and >= 2 (the checkerboard needs a bipartite
 *                torus), else ISING_E_TOPOLOGY.  A length of 2 gives two
 *                parallel edges between the same pair, each with its weight.
 *                n = product of dims must be < 2^31 / ndim.
 *   weight_seed  used when weights == NULL: w_e = +1 iff the top bit of word
 *                (e & 3) of Philox(weight_seed, (e >> 2, 0, 0, 2)) is set.
 *   weights      NULL, or host int8[ndim * n] of +1 / -1 in edge order
 *                (anything else: ISING_E_ARG).
 *   out          receives the handle (owns its host and device copies of the
 *                instance; created on the current HIP device).
 * Synchronous.
 */
int ising_create_graph(int32_t ndim, const int32_t* dims, uint64_t weight_seed,
                       const int8_t* weights, ising_graph** out);

/* Free a graph (NULL-safe).  Work that uses it must have completed. */
void ising_destroy_graph(ising_graph* g);

/* Sizes of an instance; any output pointer may be NULL.  w_total = sum of
 * all edge weights, so that energy = w_total - 2 cut (eq. (1), eq. (2)). */
int ising_graph_info(const ising_graph* g, int64_t* n_spins, int64_t* n_edges,
                     int64_t* w_total, int32_t* degree);

/* Copy the edge weights (edge order) to host int8[n_edges]. */
int ising_graph_weights(const ising_graph* g, int8_t* host_out);

/* Host-only: the weights ising_create_graph(ndim, dims, weight_seed, NULL)
 * would generate, into host int8[ndim * n].  Needs no GPU. */
int ising_generate_weights(int32_t ndim, const int32_t* dims, uint64_t weight_seed,
                           int8_t* host_out);

/* Parameters of a run of trials. */
typedef struct {
  uint32_t struct_size;      /* = sizeof(ising_run_params)                           */
  int32_t layout;            /* ISING_LAYOUT_*                                       */
  uint64_t seed;             /* Philox key of the run                                */
  int32_t n_replicas;        /* R >= 1: independent trials                           */
  int32_t n_sweeps;          /* S >= 1: trial length of the schedule (Section III)   */
  int32_t sweep_begin;       /* window [sweep_begin, sweep_end) of that schedule     */
  int32_t sweep_end;         /* 0 <= begin < end <= S                                */
  int32_t schedule;          /* ISING_SCHED_*                                        */
  int32_t init_spins;        /* 1: Philox initial state (needs begin == 0);          */
                             /* 0: start from spins_inout                            */
  double beta0, beta1;       /* linear: beta0 + (beta1-beta0)*(t/(S-1)), both >= 0;  */
                             /* geometric: beta0*(beta1/beta0)^(t/(S-1)), both > 0;  */
                             /* S == 1 gives beta0                                   */
  const double* beta_table;  /* host double[S], every entry >= 0, when TABLE         */
  int32_t block_threads;     /* 0: the library's rule; else threads per block (the   */
                             /* autotuner's pick, for instance)                      */
                             /* (rounded to the kernel's granularity)                */
  int32_t replica_offset;    /* global id of replica 0 of this call (Philox streams */
                             /* are keyed by global ids); a multiple of 4; normally 0 */
  uint64_t* stats_out;       /* device uint64[2] or NULL: the run adds the number of */
                             /* Philox4x32-10 blocks it evaluated to [0] and the     */
                             /* number of attempts that needed a uniform (dE > 0 and */
                             /* a nonzero threshold) to [1]                          */
  const uint32_t* replica_thresholds; /* device uint32 [R][degree/2] or NULL: replica */
                             /* r runs every sweep of the window at its own fixed    */
                             /* temperature, thresholds replica_thresholds[r][k-1]   */
                             /* for dE = 4k, instead of the schedule's (replica      */
                             /* exchange); layouts I8 and BS4 (AUTO picks one);      */
                             /* stats_out must then be NULL.                         */
                             /* Callers built against the struct without this field  */
                             /* pass the smaller struct_size and get NULL.           */
} ising_run_params;

/*
 * Run sweeps [sweep_begin, sweep_end) of the S-sweep schedule on R replicas.
 * Sweep t runs at beta_t; an energy change dE = 4k > 0 is accepted iff
 * u < T_k(t) = min(2^32 - 1, floor(2^32 exp(-4 k beta_t))) (the table
 * ising_thresholds returns), u = Philox word of (site, t, replica).
 *   spins_inout  device int8 [R][n], canonical layout: the window's initial
 *                state (ignored when init_spins) and, on completion, its
 *                final state.
 *   cut_out      device int64 [R] or NULL: eq. (1) cut of the final state.
 *   energy_out   device int64 [R] or NULL: eq. (2) energy of the final state.
 *                A replica whose input held a value other than +1/-1 gets
 *                ISING_INVALID_VALUE in both (its run takes values > 0 as
 *                +1 and all others as -1).
 *   flips_out    device uint32 [R] or NULL: accepted flips in the window
 *                (modulo 2^32).
 * Asynchronous on `stream`.
 */
int ising_run_trials(const ising_graph* g, const ising_run_params* p, int8_t* spins_inout,
                     int64_t* cut_out, int64_t* energy_out, uint32_t* flips_out, void* stream);

/*
 * ising_run_trials for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, layouts and results, bit for bit, but no allocation of
 * any kind.  The working memory is one fixed 16 MiB array per GPU inside the
 * library (ISING_NOALLOC_SCRATCH_BYTES), held until the process ends, which
 * takes the window's acceptance thresholds ((sweep_end - sweep_begin) *
 * degree/2 uint32) and, for the streamed layout, its HBM state (the words of
 * every 32-replica group, input flags, flip/RNG counters and, above 65,536
 * sites, the cut's partial sums).  A run needing more returns
 * ISING_E_UNSUPPORTED before anything is enqueued.  The thresholds are
 * carried into the array by small launches' arguments, so nothing on the
 * host outlives the call.  Every call on one GPU shares that GPU's array:
 * calls on one stream follow each other safely, calls that overlap on one GPU
 * (other streams, other threads) race and give undefined results.
 * Asynchronous on `stream`.
 */
#define ISING_NOALLOC_SCRATCH_BYTES (16u << 20)
int ising_run_trials_noalloc(const ising_graph* g, const ising_run_params* p, int8_t* spins_inout,
                             int64_t* cut_out, int64_t* energy_out, uint32_t* flips_out, void* stream);

/*
 * The ISING_LAYOUT_* that ising_run_trials would use for g and p (p->layout
 * AUTO resolved), into *layout_out.  Validates g and p as ising_run_trials
 * does (same error codes) and launches nothing; no spins buffer is needed.
 */
int ising_select_layout(const ising_graph* g, const ising_run_params* p, int32_t* layout_out);

/*
 * Exact cut (eq. (1)) and energy (eq. (2), J = -w, h = 0) of R states.
 *   spins        device int8 [n_replicas][n], canonical layout.
 *   cut_out, energy_out  device int64 [n_replicas]; either may be NULL.
 *   A replica holding a value other than +1 / -1 gets ISING_INVALID_VALUE.
 * Asynchronous on `stream`.  Lattices above 65,536 sites split each replica
 * into chunks whose sums pass through 24 bytes of stream-ordered scratch per
 * chunk and replica (allocated and freed on `stream`; ISING_E_NOMEM if that
 * fails).
 */
int ising_eval_cut(const ising_graph* g, const int8_t* spins, int64_t n_replicas,
                   int64_t* cut_out, int64_t* energy_out, void* stream);

/* Host-only: the acceptance thresholds T_k(t), k = 1..degree/2, of the whole
 * S-sweep schedule of p, into host uint32 [S][degree/2].  degree is 4 or 6. */
int ising_thresholds(const ising_run_params* p, int32_t degree, uint32_t* host_out);

/* Host-only: inverse temperature beta_t of sweep t of p's schedule (0 <= t < S). */
int ising_schedule_beta(const ising_run_params* p, int32_t t, double* beta_out);

/* Philox4x32-10 blocks on the GPU (the generator the kernels use), for
 * cross-checks: device uint32 ctr[m][4] in, device uint32 out[m][4] out.
 * Asynchronous on `stream`. */
int ising_philox_dump(uint64_t key, const uint32_t* ctr, int64_t m, uint32_t* out, void* stream);

/* ------------------------------------------------------------------------
 * Replica exchange (parallel tempering) on the same sweep kernels.  L ladders
 * of K inverse temperatures beta_0 <= ... <= beta_{K-1}; replica slot
 * r = l K + i starts at temperature i of ladder l.  Round q runs sweeps
 * [qE, (q+1)E) with every replica at its own temperature, then one exchange
 * pass over the adjacent pairs (k, k+1), k = q mod 2, q mod 2 + 2, ..., of
 * every ladder: the replicas at beta_k and beta_{k+1} swap temperatures with
 * probability min(1, exp((beta_k - beta_{k+1})(H_a - H_b))).  On an
 * even-degree torus H_a - H_b = 4m; m <= 0 or equal temperatures accept
 * without a draw, else accept iff u < min(2^32 - 1,
 * floor(2^32 exp(-(beta_{k+1} - beta_k) 4m))) (host-computed table),
 * u = word 0 of Philox(seed, (k, q, l, tag 4)).  Spins stay in their slots;
 * only temperature labels move.
 * ---------------------------------------------------------------------- */
typedef struct ising_pt ising_pt;

/*
 * Prepare replica exchange on g (synchronous; allocates device tables).
 *   n_temps K >= 2 and betas: host double [K], non-decreasing, >= 0;
 *   adjacent distinct temperatures at least 1e-4 apart (the exchange table
 *   of a pair has at most 65,536 entries).  n_ladders L >= 1; seed keys
 *   both the sweeps and the exchanges.  The graph must outlive the handle.
 */
int ising_pt_create(const ising_graph* g, int32_t n_temps, const double* betas, int32_t n_ladders, uint64_t seed,
                    ising_pt** out);

/*
 * Rounds [round_begin, round_begin + n_rounds) of sweeps_per_round sweeps
 * each, on device int8 spins [L K][n] (canonical layout, in/out; Philox
 * initial state when init_spins, which needs round_begin == 0).  cut_out /
 * energy_out: device int64 [L K] or NULL, the final states' eq. (1) / (2)
 * values.  Asynchronous on `stream`; the handle's labels advance with it.
 */
int ising_pt_run(ising_pt* pt, int8_t* spins, int32_t init_spins, int32_t round_begin, int32_t n_rounds,
                 int32_t sweeps_per_round, int64_t* cut_out, int64_t* energy_out, void* stream);

/*
 * Labels and counters: temp_index_out device int32 [L K] (temperature index
 * of every slot) or NULL, asynchronous on `stream`; accepted_out host
 * uint64 [K - 1] (exchanges accepted per pair since creation) or NULL,
 * synchronous.
 */
int ising_pt_state(const ising_pt* pt, int32_t* temp_index_out, uint64_t* accepted_out, void* stream);

void ising_pt_destroy(ising_pt* pt); /* NULL-safe */

/* ------------------------------------------------------------------------
 * Batches of uneven instances in one persistent launch.  Every (instance,
 * replica quad) pair is a work item; items are taken costliest first
 * (sites x sweeps) from a device queue by resident blocks until it is empty.
 * Each replica's trajectory is identical to the one ising_run_trials gives
 * for the same instance and parameters.
 * ---------------------------------------------------------------------- */
typedef struct ising_batch ising_batch;

/*
 * Prepare a batch (synchronous; allocates the plan's device tables).
 *   n_inst               >= 1 instances, all with the same ndim.
 *   graphs[k], params[k] instance k and its run (layout AUTO, I8 or BS4;
 *                        AUTO takes BS4 where the lattice allows it, else
 *                        I8; stats_out must be NULL; replica_thresholds
 *                        may be given, as for ising_run_trials;
 *                        block_threads > 0 limits the threads of the
 *                        1,024-thread launch block that work on this
 *                        instance's items, as it sizes a single run's
 *                        block, 0 = all of them).
 *   spins[k]             device int8 [R_k][n_k] (in/out, as ising_run_trials).
 *   cut_out, energy_out, flips_out  NULL, or arrays of n_inst device
 *                        pointers (entries may be NULL).
 * The graphs and buffers must outlive the batch.
 */
int ising_batch_create(int32_t n_inst, const ising_graph* const* graphs, const ising_run_params* params,
                       int8_t* const* spins, int64_t* const* cut_out, int64_t* const* energy_out,
                       uint32_t* const* flips_out, ising_batch** out);

/* Enqueue the whole batch on `stream`: a counter reset and one persistent
 * launch, with no allocation and no memset, so the call can be captured
 * into a HIP graph and replayed.  Runs on one stream at a time (the queue
 * counter is the plan's). */
int ising_batch_run(ising_batch* b, void* stream);

/* Work items, total spin-update attempts, grid and block of the launch. */
int ising_batch_info(const ising_batch* b, int64_t* n_items, int64_t* attempts, int32_t* grid, int32_t* block);

/* Free a batch plan (NULL-safe).  Work that uses it must have completed. */
void ising_batch_destroy(ising_batch* b);

/* ------------------------------------------------------------------------
 * Learned culling.  A small network reads per-replica trajectory features
 * at sweep checkpoints and predicts each replica's end-of-trial cut, so
 * that unpromising replicas are replaced by copies of promising ones.  (The
 * paper's trials are independent runs read out at their end, Section III;
 * culling is this library's extension of that campaign, and the plain
 * all-trials run remains the reference it is compared with by eq. (3).)
 * ---------------------------------------------------------------------- */

#define ISING_N_FEATURES 16
#define ISING_MLP_HIDDEN 64
/* parameters, in order: W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [64], b3 [1] */
#define ISING_MLP_PARAMS 5313

/* Per-replica trajectory record kept across checkpoints (device memory,
 * caller-owned, zero-filled before the first checkpoint of a trial). */
typedef struct {
  int64_t h_min;           /* lowest checkpoint energy so far                   */
  int64_t h_prev;          /* energy at the previous checkpoint                 */
  uint64_t flips_total;    /* accepted flips since the start of the trial       */
  int32_t checkpoints;     /* checkpoints recorded so far                       */
  int32_t last_improve;    /* checkpoint index at which h_min last decreased    */
} ising_track;

/*
 * Features of R replicas at a checkpoint after `sweeps_done` sweeps of an
 * S-sweep schedule, the last window having `window` sweeps.
 *   spins        device int8 [R][n], canonical layout (state at the checkpoint).
 *   energy       device int64 [R]: eq. (2) energy of that state (run output).
 *   window_flips device uint32 [R]: accepted flips of the last window.
 *   track        device ising_track [R], updated in place.
 *   beta         inverse temperature of the window's last sweep (> 0).
 *   n_checkpoints total checkpoints of the trial (>= 1).
 *   features     device float [R][16]:
 *     0 H/|E|, 1 min over checkpoints of H/|E|, 2 (H - H_prev)/|E| (H_prev = 0
 *     at the first checkpoint), 3 window flips/(n window), 4 total flips/(n
 *     sweeps_done), 5 beta, 6 sweeps_done/S, 7..13 fraction of sites with
 *     s_i f_i = -6, -4, -2, 0, 2, 4, 6 (f_i = sum_j w_ij s_j), 14 ln beta,
 *     15 (checkpoints since h_min last decreased) / n_checkpoints.
 * Asynchronous on `stream`.
 */
int ising_features(const ising_graph* g, const int8_t* spins, const int64_t* energy,
                   const uint32_t* window_flips, int64_t n_replicas, ising_track* track,
                   int32_t sweeps_done, int32_t window, int32_t n_sweeps, double beta,
                   int32_t n_checkpoints, float* features, void* stream);

/* Kaiming-uniform initial parameters from Philox (key = seed, counter
 * (index >> 2, 0, 0, 3), word index & 3): a weight of a layer with fan-in F
 * is sqrt(6/F) * (2 u - 1), u = (word >> 8) * 2^-24; biases 0.
 * params: device float [ISING_MLP_PARAMS].  Asynchronous. */
int ising_mlp_init(uint64_t seed, float* params, void* stream);

/* y[b] = W3 relu(W2 relu(W1 z_b + b1) + b2) + b3 with z_b = (x_b - mean) / std
 * (mean, std: device float[16], or both NULL for z = x).
 *   x       device float [x_rows][16]; sample b reads row idx[b] when idx !=
 *           NULL (device int32 [B]), else row b (then B <= x_rows, else
 *           ISING_E_ARG).  A sample whose idx[b] lies outside [0, x_rows)
 *           reads nothing and gets y[b] = NaN.
 *   y       device float [B].  Asynchronous. */
int ising_mlp_forward(const float* params, const float* x, int64_t x_rows, const int32_t* idx,
                      const float* mean, const float* std, int64_t batch, float* y, void* stream);

/* Floats of workspace ising_mlp_loss_grad needs for a batch. */
int64_t ising_mlp_workspace_floats(int64_t batch);

/* Mean squared error L = (1/B) sum_b (y_b - target_b)^2 of the forward pass
 * above and its gradient with respect to every parameter.
 *   x, x_rows, idx  as for ising_mlp_forward; a sample whose idx[b] lies
 *             outside [0, x_rows) reads neither x nor target and makes the
 *             loss and the gradient NaN.
 *   target    device float [B], or [x_rows] read at idx[b] when idx != NULL.
 *   grad      device float [ISING_MLP_PARAMS] (overwritten).
 *   loss      device float [1] (overwritten), or NULL.
 *   workspace device float [ising_mlp_workspace_floats(B)].
 * Summation order is fixed, so results are reproducible.  Asynchronous. */
int ising_mlp_loss_grad(const float* params, const float* x, int64_t x_rows, const int32_t* idx,
                        const float* mean, const float* std, const float* target, int64_t batch,
                        float* grad, float* loss, float* workspace, void* stream);

/* One Adam step (Kingma & Ba) on n parameters, step = 1, 2, ...:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).  0 <= n <= 2^31 - 1,
 * else ISING_E_ARG.  Asynchronous. */
int ising_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, int32_t step,
                    float lr, float beta1, float beta2, float eps, void* stream);

/* Column means and standard deviations (population, floored at 1e-6) of a
 * device float [rows][16] table, computed in double in two passes (the mean,
 * then the squared deviations from it) with a fixed summation order;
 * mean, std: device float [16].  Asynchronous. */
int ising_feature_stats(const float* x, int64_t rows, float* mean, float* std, void* stream);

/* In place, for every group g and column c of a device float
 * [n_groups][rows][cols] table: x = (x - mean) / std with the mean and
 * population standard deviation (floored at 1e-6) of column c over the rows
 * of group g, computed in double in a fixed order (two passes) and rounded
 * to float once.  A group is one population compared at one checkpoint (the
 * replicas of a run): what the whole group shares becomes 0, what remains
 * is each row's standing within it.  rows >= 1, cols >= 1.  Asynchronous. */
int ising_standardize_groups(float* x, int64_t n_groups, int64_t rows, int32_t cols, void* stream);

/*
 * Rank R replicas by score (higher first; ties: lower index first; NaN
 * last) and let the bottom floor(R/2) take copies of the top floor(R/2):
 * the j-th worst becomes a copy of the j-th best (spins and, when track is
 * not NULL, its ising_track).  Each replica keeps its index, hence its own
 * Philox stream, so copies diverge afterwards.
 *   score     device float [R];  spins device int8 [R][n] (in/out).
 *   order_out device int32 [R] or NULL: replica indices from best to worst.
 * R <= 16384.  Asynchronous.
 */
int ising_cull_clone(const float* score, int64_t n_replicas, int64_t n_spins, int8_t* spins,
                     ising_track* track, int32_t* order_out, void* stream);

/* The network is trained on the cut a replica still gains until the end of
 * its trial, gain = (final cut - cut now) / |E|; its ranking score is the
 * predicted final cut / |E| = cut now / |E| + gain, where
 * cut now / |E| = (W_total / |E| - features[r][0]) / 2 (eq. (1)-(2)).
 *   gain      device float [R] (network output);  features device float [R][16].
 *   score     device float [R] (may alias gain).  0 <= R <= 2^31 - 1, else
 * ISING_E_ARG.  Asynchronous. */
int ising_final_cut_score(const ising_graph* g, const float* gain, const float* features, int64_t n_replicas,
                          float* score, void* stream);

/* Training labels from end-of-trial cuts: out[r] = (final_cut[r] - now_cut[r])
 * * scale, computed in double and rounded to float once (now_cut NULL: 0).
 * With scale = 1/|E| and now_cut the cut at a checkpoint this is the cut a
 * replica still gains; without now_cut, its end-of-trial cut / |E|.
 *   final_cut, now_cut  device int64 [R];  out device float [R].
 * 0 <= R <= 2^31 - 1 and scale finite, else ISING_E_ARG.  Asynchronous. */
int ising_cut_labels(const int64_t* final_cut, const int64_t* now_cut, int64_t n_replicas, double scale,
                     float* out, void* stream);

/* score[r] = -energy[r] (the energy-ranked baseline of culling);
 * 0 <= n_replicas <= 2^31 - 1, else ISING_E_ARG.  Asynchronous. */
int ising_energy_score(const int64_t* energy, int64_t n_replicas, float* score, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* ising_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ISING_H */
