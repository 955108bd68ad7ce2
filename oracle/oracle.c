/*
 * CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain single-threaded C11.  Every function states the passage of the paper
 * it follows, or the reading taken where the paper is silent (the paper
 * withholds its own update rule, so the sweep is plain checkerboard
 * Metropolis annealing; the paper fixes only the objective, the instance
 * family and the notion of a sweep).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Philox4x32-10, from the definition in Salmon et al., "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64 products
 * of counter words 0 and 2 with fixed multipliers, the high halves xored with
 * the other two counter words and the round key, the key bumped by the two
 * Weyl constants between rounds.  Parity pinned against an independent
 * implementation (PyTorch's philox engine) in the tests.
 * ------------------------------------------------------------------------- */
void orc_philox4x32_10(uint64_t key, const uint32_t ctr[4], uint32_t out[4]) {
    const uint32_t mult_a = 0xD2511F53u, mult_b = 0xCD9E8D57u;
    const uint32_t weyl_a = 0x9E3779B9u, weyl_b = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = (uint32_t)(key & 0xffffffffu), k1 = (uint32_t)(key >> 32);
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl_a;
            k1 += weyl_b;
        }
        uint64_t p_a = (uint64_t)mult_a * (uint64_t)x0;
        uint64_t p_b = (uint64_t)mult_b * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p_b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p_b;
        uint32_t y2 = (uint32_t)(p_a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static uint32_t philox_word(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int word) {
    uint32_t ctr[4] = {c0, c1, c2, c3}, out[4];
    orc_philox4x32_10(key, ctr, out);
    return out[word];
}

/* ---------------------------------------------------------------------------
 * Torus (Section I; Appendix A Fig. 2: toroidal square grid, each variable
 * coupled to four nearest neighbours, periodic in both dimensions).  The
 * three-dimensional cubic torus (six neighbours) is the same construction
 * with one more axis.  Site numbering is row-major; a dimension of length 2
 * gives two parallel edges between the same pair (a multigraph), each with
 * its own weight.
 * ------------------------------------------------------------------------- */
int64_t orc_n_sites(int ndim, const int32_t* dims) {
    int64_t n = 1;
    for (int d = 0; d < ndim; ++d) n *= dims[d];
    return n;
}

int64_t orc_n_edges(int ndim, const int32_t* dims) { return (int64_t)ndim * orc_n_sites(ndim, dims); }

/* coordinates of site i: 2-D -> (row, col); 3-D -> (z, y, x) */
static void site_coords(int ndim, const int32_t* dims, int64_t i, int64_t* c) {
    for (int d = ndim - 1; d >= 0; --d) {
        c[d] = i % dims[d];
        i /= dims[d];
    }
}

static int64_t site_index(int ndim, const int32_t* dims, const int64_t* c) {
    int64_t i = 0;
    for (int d = 0; d < ndim; ++d) i = i * dims[d] + c[d];
    return i;
}

void orc_torus_edges(int ndim, const int32_t* dims, int32_t* edge_a, int32_t* edge_b) {
    int64_t n = orc_n_sites(ndim, dims);
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        site_coords(ndim, dims, i, c);
        for (int d = 0; d < ndim; ++d) {
            /* axis d of the edge order: the fastest-varying coordinate first */
            int axis = ndim - 1 - d;
            int64_t nb[3] = {c[0], c[1], c[2]};
            nb[axis] = (c[axis] + 1) % dims[axis];
            edge_a[ndim * i + d] = (int32_t)i;
            edge_b[ndim * i + d] = (int32_t)site_index(ndim, dims, nb);
        }
    }
}

/* Checkerboard colour: parity of the coordinate sum (even dims => bipartite). */
int orc_site_colour(int ndim, const int32_t* dims, int64_t i) {
    int64_t c[3];
    site_coords(ndim, dims, i, c);
    int64_t s = 0;
    for (int d = 0; d < ndim; ++d) s += c[d];
    return (int)(s & 1);
}

/* Random +/-1 weights (Section I says only "random"; reading: uniform +/-1
 * from the weight seed through Philox, tag WEIGHT, four edges per block). */
void orc_random_weights(uint64_t seed, int64_t n_edges, int8_t* w) {
    for (int64_t e = 0; e < n_edges; ++e) {
        uint32_t u = philox_word(seed, (uint32_t)(e >> 2), 0u, 0u, ORC_TAG_WEIGHT, (int)(e & 3));
        w[e] = (u >> 31) ? (int8_t)1 : (int8_t)-1;
    }
}

/* ---------------------------------------------------------------------------
 * Annealing schedule (the paper fixes only the trial length in sweeps,
 * Section III; the inverse-temperature ramp is a reading): sweep t of an
 * S-sweep schedule runs at
 *   linear:    beta0 + (beta1 - beta0) * (t / (S - 1))
 *   geometric: beta0 * (beta1 / beta0) ^ (t / (S - 1))
 *   table:     table[t]
 * with S = 1 giving beta0.
 * ------------------------------------------------------------------------- */
double orc_beta(int schedule, double beta0, double beta1, const double* table, int32_t n_sweeps, int32_t t) {
    if (schedule == ORC_SCHED_TABLE) return table[t];
    if (n_sweeps <= 1) return beta0;
    double frac = (double)t / (double)(n_sweeps - 1);
    if (schedule == ORC_SCHED_LINEAR) return beta0 + (beta1 - beta0) * frac;
    return beta0 * pow(beta1 / beta0, frac);
}

/* Metropolis acceptance min(1, exp(-beta * dE)) for dE = 4k > 0, as a 32-bit
 * threshold: accept iff a uniform 32-bit word u < floor(2^32 exp(-4 k beta)),
 * clamped to 2^32 - 1. */
uint32_t orc_threshold(double beta, int k) {
    double p = exp(-(double)(4 * k) * beta);
    double scaled = ldexp(p, 32);
    if (scaled >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)floor(scaled);
}

void orc_init_spins(uint64_t seed, int32_t replica_begin, int32_t n_replicas, int64_t n, int8_t* spins) {
    for (int32_t rr = 0; rr < n_replicas; ++rr) {
        uint32_t r = (uint32_t)(replica_begin + rr);
        for (int64_t i = 0; i < n; ++i) {
            uint32_t u = philox_word(seed, (uint32_t)i, 0u, r >> 2, ORC_TAG_INIT, (int)(r & 3));
            spins[(int64_t)rr * n + i] = (u >> 31) ? (int8_t)1 : (int8_t)-1;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Objective (Section II, eq. (1) and eq. (2) with J = -w, h = 0): each edge
 * counted once; cut = sum_e w_e [s_a != s_b], H = sum_e w_e s_a s_b.
 * ------------------------------------------------------------------------- */
void orc_cut_energy(int64_t n, int64_t n_edges, const int32_t* edge_a, const int32_t* edge_b,
                    const int8_t* w, int32_t n_replicas, const int8_t* spins,
                    int64_t* cut, int64_t* energy) {
    for (int32_t r = 0; r < n_replicas; ++r) {
        const int8_t* s = spins + (int64_t)r * n;
        int64_t c = 0, h = 0;
        for (int64_t e = 0; e < n_edges; ++e) {
            int sa = s[edge_a[e]], sb = s[edge_b[e]];
            if (sa != sb) c += w[e];
            h += (int64_t)w[e] * sa * sb;
        }
        cut[r] = c;
        energy[r] = h;
    }
}

/* adjacency of every site as (neighbour, weight) over its incident edges */
typedef struct {
    int64_t n;
    int deg;
    int32_t* nb;  /* [n][deg] */
    int8_t* wt;   /* [n][deg] */
} adjacency;

static int build_adjacency(int ndim, const int32_t* dims, const int8_t* w, adjacency* adj) {
    int64_t n = orc_n_sites(ndim, dims), ne = orc_n_edges(ndim, dims);
    int deg = 2 * ndim;
    int32_t* ea = (int32_t*)malloc(sizeof(int32_t) * (size_t)ne);
    int32_t* eb = (int32_t*)malloc(sizeof(int32_t) * (size_t)ne);
    int* fill = (int*)calloc((size_t)n, sizeof(int));
    adj->n = n;
    adj->deg = deg;
    adj->nb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n * deg));
    adj->wt = (int8_t*)malloc((size_t)(n * deg));
    if (!ea || !eb || !fill || !adj->nb || !adj->wt) {
        free(ea); free(eb); free(fill); free(adj->nb); free(adj->wt);
        return -1;
    }
    orc_torus_edges(ndim, dims, ea, eb);
    for (int64_t e = 0; e < ne; ++e) {
        int64_t a = ea[e], b = eb[e];
        adj->nb[a * deg + fill[a]] = (int32_t)b;
        adj->wt[a * deg + fill[a]] = w[e];
        fill[a]++;
        adj->nb[b * deg + fill[b]] = (int32_t)a;
        adj->wt[b * deg + fill[b]] = w[e];
        fill[b]++;
    }
    free(ea); free(eb); free(fill);
    return 0;
}

static void free_adjacency(adjacency* adj) {
    free(adj->nb);
    free(adj->wt);
}

void orc_fields(int ndim, const int32_t* dims, const int8_t* w, const int8_t* spins, int32_t* f) {
    adjacency adj;
    if (build_adjacency(ndim, dims, w, &adj) != 0) return;
    for (int64_t i = 0; i < adj.n; ++i) {
        int32_t acc = 0;
        for (int k = 0; k < adj.deg; ++k) acc += adj.wt[i * adj.deg + k] * spins[adj.nb[i * adj.deg + k]];
        f[i] = acc;
    }
    free_adjacency(&adj);
}

/* ---------------------------------------------------------------------------
 * Trials (Section III: a trial is a run of S sweeps whose solution is read
 * out at its end; the sweep is the fundamental step).  Reading of the sweep:
 * every site of colour 0, then every site of colour 1, each visited once; a
 * visit proposes flipping s_i, with energy change dE = -2 s_i f_i, and
 * accepts if dE <= 0 (no draw) or if u < threshold(beta_t, dE/4), where u is
 * word (r & 3) of Philox(seed, (i, t, r>>2, TAG_METROPOLIS)).  Accepted flips
 * update the maintained fields of the neighbours: f_j -= 2 w_ij s_i(old).
 * ------------------------------------------------------------------------- */
/* The sweeps of orc_run and orc_run_fixed: replica rr runs at the schedule's
 * beta_t, or, when rep_thr is given, with its own thresholds
 * rep_thr[rr][k-1] (k = 1..deg/2) at every sweep. */
static int run_core(int ndim, const int32_t* dims, const int8_t* w, uint64_t seed,
                    int32_t replica_begin, int32_t n_replicas, int32_t n_sweeps,
                    int32_t begin, int32_t end, int schedule, double beta0, double beta1,
                    const double* table, const uint32_t* rep_thr, int init, int8_t* spins,
                    uint32_t* flips, int32_t* fields_out) {
    if (ndim != 2 && ndim != 3) return -1;
    for (int d = 0; d < ndim; ++d)
        if (dims[d] < 2 || (dims[d] & 1)) return -1;
    if (n_replicas < 0 || replica_begin < 0 || n_sweeps <= 0 || begin < 0 || end > n_sweeps || begin > end) return -1;
    if (init && begin != 0) return -1;

    int64_t n = orc_n_sites(ndim, dims);
    adjacency adj;
    if (build_adjacency(ndim, dims, w, &adj) != 0) return -1;
    int deg = adj.deg;
    int* colour = (int*)malloc(sizeof(int) * (size_t)n);
    int32_t* f = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    uint32_t* thr = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(deg / 2 + 1));
    if (!colour || !f || !thr) {
        free(colour); free(f); free(thr); free_adjacency(&adj);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) colour[i] = orc_site_colour(ndim, dims, i);

    if (init) orc_init_spins(seed, replica_begin, n_replicas, n, spins);

    for (int32_t rr = 0; rr < n_replicas; ++rr) {
        uint32_t r = (uint32_t)(replica_begin + rr);
        int8_t* s = spins + (int64_t)rr * n;
        uint32_t nflip = 0;
        for (int64_t i = 0; i < n; ++i) {
            int32_t acc = 0;
            for (int k = 0; k < deg; ++k) acc += adj.wt[i * deg + k] * s[adj.nb[i * deg + k]];
            f[i] = acc;
        }
        for (int32_t t = begin; t < end; ++t) {
            if (rep_thr) {
                for (int k = 1; k <= deg / 2; ++k) thr[k] = rep_thr[(int64_t)rr * (deg / 2) + k - 1];
            } else {
                double beta = orc_beta(schedule, beta0, beta1, table, n_sweeps, t);
                for (int k = 1; k <= deg / 2; ++k) thr[k] = orc_threshold(beta, k);
            }
            for (int c = 0; c < 2; ++c) {
                for (int64_t i = 0; i < n; ++i) {
                    if (colour[i] != c) continue;
                    int dE = -2 * s[i] * f[i];
                    int accept;
                    if (dE <= 0) {
                        accept = 1;
                    } else {
                        uint32_t u = philox_word(seed, (uint32_t)i, (uint32_t)t, r >> 2, ORC_TAG_METROPOLIS, (int)(r & 3));
                        accept = u < thr[dE / 4];
                    }
                    if (accept) {
                        int old = s[i];
                        for (int k = 0; k < deg; ++k) f[adj.nb[i * deg + k]] -= 2 * adj.wt[i * deg + k] * old;
                        s[i] = (int8_t)(-old);
                        nflip++;
                    }
                }
            }
        }
        if (flips) flips[rr] = nflip;
        if (fields_out) memcpy(fields_out + (int64_t)rr * n, f, sizeof(int32_t) * (size_t)n);
    }
    free(colour); free(f); free(thr);
    free_adjacency(&adj);
    return 0;
}

int orc_run(int ndim, const int32_t* dims, const int8_t* w, uint64_t seed,
            int32_t replica_begin, int32_t n_replicas, int32_t n_sweeps,
            int32_t begin, int32_t end, int schedule, double beta0, double beta1,
            const double* table, int init, int8_t* spins, uint32_t* flips, int32_t* fields_out) {
    return run_core(ndim, dims, w, seed, replica_begin, n_replicas, n_sweeps, begin, end, schedule, beta0, beta1,
                    table, NULL, init, spins, flips, fields_out);
}

int orc_run_fixed(int ndim, const int32_t* dims, const int8_t* w, uint64_t seed,
                  int32_t replica_begin, int32_t n_replicas, int32_t begin, int32_t end,
                  const uint32_t* rep_thr, int init, int8_t* spins, uint32_t* flips) {
    if (!rep_thr) return -1;
    return run_core(ndim, dims, w, seed, replica_begin, n_replicas, end, begin, end, ORC_SCHED_LINEAR, 1.0, 1.0,
                    NULL, rep_thr, init, spins, flips, NULL);
}

/* Exhaustive maximum of eq. (1) over all 2^n states. */
int64_t orc_maxcut_bruteforce(int64_t n, int64_t n_edges, const int32_t* edge_a,
                              const int32_t* edge_b, const int8_t* w, uint64_t* best_state) {
    int64_t best = INT64_MIN;
    uint64_t arg = 0;
    for (uint64_t state = 0; state < ((uint64_t)1 << n); ++state) {
        int64_t c = 0;
        for (int64_t e = 0; e < n_edges; ++e) {
            int xa = (int)((state >> edge_a[e]) & 1), xb = (int)((state >> edge_b[e]) & 1);
            if (xa != xb) c += w[e];
        }
        if (c > best) {
            best = c;
            arg = state;
        }
    }
    if (best_state) *best_state = arg;
    return best;
}
