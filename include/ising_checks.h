/*
 * ising_checks.h -- cross-check entry points of the MI355X library: internal
 * building blocks run on caller-given data, so that tests can compare them
 * with plain host code.  Nothing here is needed to anneal.
 *
 * Error codes and ownership as in ising.h: every function returns 0
 * (ISING_OK) or a negative code; the caller owns every buffer.
 */
#ifndef ISING_CHECKS_H
#define ISING_CHECKS_H

#include <stdint.h>

#include "ising.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The threshold compare chains of the bit-sliced kernels, on n sets of 32
 * words.  Paper, Section III (with the acceptance reading of ising.h): a
 * replica at dE = 4k > 0 flips iff its uniform 32-bit word u is below the
 * threshold T_k, strictly.
 *
 *   u          device uint32 [n][32], the words of each set.
 *   sel2, sel3 device uint32 [n], disjoint level bits of each set: word j is
 *              compared with T3 where bit j of sel3 is set, else with T2
 *              where bit j of sel2 is set, else with T1.
 *   T1..T3     thresholds, the same for every set.
 *   out        device uint32 [n][8]; bit j of each result = (word j < its
 *              threshold), 0 above the words a result covers:
 *     [0] 32 words, two levels: T2 where sel2, else T1;
 *     [1] 32 words, three levels: T3 where sel3, T2 where sel2, else T1;
 *     [2] words 0..15, one level per replica: word 4 i + q against A[q];
 *     [3] [4] [5] 32 words against T1, T2, T3, in the form screened per
 *         wave of 64 sets (a set past the last repeats it);
 *     [6] words 0..15, two levels per replica: B[q] where sel2, else A[q];
 *     [7] words 0..15, three levels per replica: C[q] where sel3, B[q]
 *         where sel2, else A[q];
 *   with A = {T1, T2, T3, T1}, B = {T2, T1, T2, T3}, C = {T3, T3, T1, T2}.
 *
 * ISING_E_ARG for n < 0 or a NULL buffer with n > 0; ISING_E_HIP if the
 * launch fails.  Asynchronous on `stream` (NULL: the default stream). */
int ising_compare_chains(int64_t n, const uint32_t* u, const uint32_t* sel2, const uint32_t* sel3, uint32_t T1,
                         uint32_t T2, uint32_t T3, uint32_t* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ISING_CHECKS_H */
