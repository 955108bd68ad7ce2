/* Runs every entry point of the C oracle on small tori, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py):
 * any out-of-bounds access, use of freed memory or undefined arithmetic
 * aborts the program.  It also checks identities the oracle must satisfy
 * (energy = W_total - 2 cut; maintained fields equal recomputed ones), and
 * prints "ok" at the end. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int fail(const char* what) {
  fprintf(stderr, "check failed: %s\n", what);
  return 1;
}

static int one_torus(int ndim, const int32_t* dims, int R, int S) {
  const int64_t n = orc_n_sites(ndim, dims), ne = orc_n_edges(ndim, dims);
  int8_t* w = malloc((size_t)ne);
  int32_t* ea = malloc(sizeof(int32_t) * (size_t)ne);
  int32_t* eb = malloc(sizeof(int32_t) * (size_t)ne);
  int8_t* s = malloc((size_t)(R * n));
  uint32_t* fl = malloc(sizeof(uint32_t) * (size_t)R);
  int32_t* fo = malloc(sizeof(int32_t) * (size_t)(R * n));
  int32_t* f = malloc(sizeof(int32_t) * (size_t)n);
  int64_t* cut = malloc(sizeof(int64_t) * (size_t)R);
  int64_t* en = malloc(sizeof(int64_t) * (size_t)R);
  uint32_t* thr = malloc(sizeof(uint32_t) * (size_t)(R * ndim));
  double* table = malloc(sizeof(double) * (size_t)S);
  int bad = 0;
  orc_random_weights(12345u, ne, w);
  orc_torus_edges(ndim, dims, ea, eb);
  int64_t wt = 0;
  for (int64_t e = 0; e < ne; ++e) wt += w[e];
  for (int i = 0; i < S; ++i) table[i] = 0.01 * i;
  for (int sched = 0; sched < 3; ++sched) {
    if (orc_run(ndim, dims, w, 0xDEADBEEFCAFEull, 8, R, S, 0, S, sched, 0.05, 4.0, table, 1, s, fl, fo)) return fail("run");
    orc_cut_energy(n, ne, ea, eb, w, R, s, cut, en);
    for (int r = 0; r < R; ++r) {
      if (en[r] != wt - 2 * cut[r]) bad |= fail("energy = W - 2 cut");
      orc_fields(ndim, dims, w, s + (size_t)r * n, f);
      if (memcmp(f, fo + (size_t)r * n, sizeof(int32_t) * (size_t)n)) bad |= fail("maintained fields");
    }
    /* resume from the state just computed, over a later window */
    if (orc_run(ndim, dims, w, 7u, 0, R, 2 * S, S, 2 * S, sched == 2 ? 0 : sched, 0.3, 2.0, NULL, 0, s, fl, NULL))
      return fail("resume");
  }
  for (int r = 0; r < R; ++r)
    for (int k = 0; k < ndim; ++k) thr[r * ndim + k] = orc_threshold(0.1 * (r + 1), k + 1);
  if (orc_run_fixed(ndim, dims, w, 99u, 4, R, 0, S, thr, 1, s, fl)) return fail("run_fixed");
  orc_init_spins(5u, 0, R, n, s);
  if (n <= 16) {
    uint64_t best = 0;
    const int64_t mc = orc_maxcut_bruteforce(n, ne, ea, eb, w, &best);
    int8_t* bs = malloc((size_t)n);
    for (int64_t i = 0; i < n; ++i) bs[i] = ((best >> i) & 1u) ? 1 : -1;
    int64_t c1, e1;
    orc_cut_energy(n, ne, ea, eb, w, 1, bs, &c1, &e1);
    if (c1 != mc) bad |= fail("brute-force state attains its cut");
    free(bs);
  }
  for (int64_t i = 0; i < n; ++i) (void)orc_site_colour(ndim, dims, i);
  free(w); free(ea); free(eb); free(s); free(fl); free(fo); free(f); free(cut); free(en); free(thr); free(table);
  return bad;
}

int main(void) {
  const int32_t d2[][2] = {{2, 2}, {2, 4}, {4, 6}, {6, 8}, {12, 10}, {2, 20}};
  const int32_t d3[][3] = {{2, 2, 2}, {2, 2, 4}, {4, 4, 6}, {6, 4, 8}};
  int bad = 0;
  for (size_t k = 0; k < sizeof d2 / sizeof d2[0]; ++k) bad |= one_torus(2, d2[k], 6, 40);
  for (size_t k = 0; k < sizeof d3 / sizeof d3[0]; ++k) bad |= one_torus(3, d3[k], 5, 30);
  uint32_t ctr[4] = {1u, 2u, 3u, 4u}, out[4];
  orc_philox4x32_10(~0ull, ctr, out);
  for (int k = 1; k <= 3; ++k) (void)orc_threshold(0.0, k), (void)orc_threshold(1e300, k), (void)orc_threshold(1e-300, k);
  for (int t = 0; t < 5; ++t) (void)orc_beta(1, 0.05, 4.0, NULL, 5, t), (void)orc_beta(0, 0.1, 3.0, NULL, 1, 0);
  if (bad) return 1;
  printf("ok\n");
  return 0;
}
