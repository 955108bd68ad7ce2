/*
 * CPU oracle for replica-parallel checkerboard Metropolis annealing on
 * +/-1-weighted toroidal Ising / Max-Cut instances.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product links, loads or calls
 * this code; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg do.  It is a plain, slow, single-threaded statement of what
 * the GPU library must compute, written independently of it (own Philox,
 * own torus construction, own threshold table, own cut/energy sum).
 *
 * Problem (paper, Section II): maximise the cut of eq. (1),
 *   cut(x) = 1/2 sum_{i<j} w_ij (1 - x_i x_j),  x in {-1,+1}^n,
 * equivalently minimise the Ising energy of eq. (2) with J_ij = -w_ij and
 * h_i = 0, i.e. H(s) = sum_{i<j} w_ij s_i s_j = W_total - 2 cut(s).
 * Instance family (Section I, Appendix A Fig. 2): toroidal square grid, four
 * nearest neighbours, periodic in both dimensions, w_ij in {-1,+1}.
 */
#ifndef ISING_ORACLE_H
#define ISING_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox counter tags (fourth counter word). */
enum { ORC_TAG_METROPOLIS = 0, ORC_TAG_INIT = 1, ORC_TAG_WEIGHT = 2, ORC_TAG_MLP = 3 };
enum { ORC_SCHED_LINEAR = 0, ORC_SCHED_GEOMETRIC = 1, ORC_SCHED_TABLE = 2 };

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 64-bit key = (lo, hi). */
void orc_philox4x32_10(uint64_t key, const uint32_t ctr[4], uint32_t out[4]);

/* Torus shape: ndim in {2, 3}; dims = {rows, cols} or {Lz, Ly, Lx}. */
int64_t orc_n_sites(int ndim, const int32_t* dims);
int64_t orc_n_edges(int ndim, const int32_t* dims);
/* Edge e = ndim*i + d joins site i to its +1 neighbour along axis d
 * (2-D: d=0 column, d=1 row; 3-D: d=0 x, d=1 y, d=2 z). */
void orc_torus_edges(int ndim, const int32_t* dims, int32_t* edge_a, int32_t* edge_b);
int orc_site_colour(int ndim, const int32_t* dims, int64_t i);

/* w_e = +1 iff the top bit of word (e & 3) of Philox(seed, (e>>2, 0, 0, TAG_WEIGHT)) is set. */
void orc_random_weights(uint64_t seed, int64_t n_edges, int8_t* w);

/* Inverse temperature of sweep t of an S-sweep schedule. */
double orc_beta(int schedule, double beta0, double beta1, const double* table, int32_t n_sweeps, int32_t t);
/* Acceptance threshold for an energy increase of 4k at inverse temperature beta. */
uint32_t orc_threshold(double beta, int k);

/* s_{r,i} = +1 iff the top bit of word (r & 3) of Philox(seed, (i, 0, r>>2, TAG_INIT)) is set. */
void orc_init_spins(uint64_t seed, int32_t replica_begin, int32_t n_replicas, int64_t n, int8_t* spins);

/* Exact cut and energy of each replica by a direct sum over the edge list. */
void orc_cut_energy(int64_t n, int64_t n_edges, const int32_t* edge_a, const int32_t* edge_b,
                    const int8_t* w, int32_t n_replicas, const int8_t* spins,
                    int64_t* cut, int64_t* energy);

/* Local fields f_i = sum over incident edges of w_e s_j, for one replica. */
void orc_fields(int ndim, const int32_t* dims, const int8_t* w, const int8_t* spins, int32_t* f);

/*
 * Run sweeps [begin, end) of an S-sweep schedule on replicas
 * replica_begin .. replica_begin + n_replicas - 1 (their Philox streams are
 * keyed by those global ids).  spins is [n_replicas][n] int8 +/-1, read
 * (unless init) and written; flips [n_replicas] receives accepted flips;
 * fields_out [n_replicas][n] (may be NULL) receives the maintained local
 * fields at the end of the window.  Returns 0, or -1 on bad arguments.
 */
int orc_run(int ndim, const int32_t* dims, const int8_t* w, uint64_t seed,
            int32_t replica_begin, int32_t n_replicas, int32_t n_sweeps,
            int32_t begin, int32_t end, int schedule, double beta0, double beta1,
            const double* table, int init, int8_t* spins, uint32_t* flips, int32_t* fields_out);

/*
 * As orc_run over sweeps [begin, end), but replica rr keeps its own fixed
 * temperature: every sweep uses its thresholds rep_thr[rr][k-1], k = 1..deg/2
 * (a replica-exchange round).  Returns 0, or -1 on bad arguments.
 */
int orc_run_fixed(int ndim, const int32_t* dims, const int8_t* w, uint64_t seed,
                  int32_t replica_begin, int32_t n_replicas, int32_t begin, int32_t end,
                  const uint32_t* rep_thr, int init, int8_t* spins, uint32_t* flips);

/* Largest cut over all 2^n states (n <= 30); best state written as bits. */
int64_t orc_maxcut_bruteforce(int64_t n, int64_t n_edges, const int32_t* edge_a,
                              const int32_t* edge_b, const int8_t* w, uint64_t* best_state);

#ifdef __cplusplus
}
#endif
#endif
