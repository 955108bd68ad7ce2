/* Calls the product library's host-only entry points (no GPU needed) for a
 * build whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py): schedules and
 * thresholds of every kind, generated weights, and the argument checks of
 * the entry points that reject a call before touching a device.  Prints "ok"
 * at the end. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ising.h"

int main(void) {
  int bad = 0;
  const int32_t d2[2] = {100, 200}, d3[3] = {4, 6, 8}, odd[2] = {5, 4};
  int8_t* w = malloc(2 * 100 * 200);
  bad |= ising_generate_weights(2, d2, 81u, w) != ISING_OK;
  int8_t* w3 = malloc(3 * 4 * 6 * 8);
  bad |= ising_generate_weights(3, d3, ~0ull, w3) != ISING_OK;
  bad |= ising_generate_weights(2, odd, 1u, w) != ISING_E_TOPOLOGY;
  const int S = 2000;
  double* table = malloc(sizeof(double) * S);
  for (int t = 0; t < S; ++t) table[t] = 4.0 * t / S;
  uint32_t* thr = malloc(sizeof(uint32_t) * 3 * S);
  for (int sched = 0; sched < 3; ++sched) {
    ising_run_params p;
    memset(&p, 0, sizeof p);
    p.struct_size = sizeof p;
    p.n_replicas = 4;
    p.n_sweeps = S;
    p.sweep_end = S;
    p.schedule = sched;
    p.beta0 = 0.05;
    p.beta1 = 4.0;
    p.beta_table = table;
    bad |= ising_thresholds(&p, 4, thr) != ISING_OK;
    bad |= ising_thresholds(&p, 6, thr) != ISING_OK;
    double beta = 0.0;
    bad |= ising_schedule_beta(&p, S - 1, &beta) != ISING_OK;
    bad |= ising_schedule_beta(&p, S, &beta) != ISING_E_ARG;
    p.struct_size = 8;
    bad |= ising_thresholds(&p, 4, thr) != ISING_E_ARG;
  }
  /* rejected before any device work */
  bad |= ising_adam_step((float*)16, (const float*)16, (float*)16, (float*)16, (int64_t)1 << 31, 1, 1e-3f, 0.9f,
                         0.999f, 1e-8f, NULL) != ISING_E_ARG;
  bad |= ising_energy_score((const int64_t*)16, -1, (float*)16, NULL) != ISING_E_ARG;
  bad |= ising_cut_labels((const int64_t*)16, NULL, -1, 1.0, (float*)16, NULL) != ISING_E_ARG;
  bad |= ising_mlp_forward((const float*)16, (const float*)16, 8, NULL, NULL, NULL, 9, (float*)16, NULL) != ISING_E_ARG;
  bad |= ising_create_graph(2, odd, 1u, NULL, NULL) == ISING_OK;
  ising_destroy_graph(NULL);
  bad |= strlen(ising_last_error()) == 0;
  free(w);
  free(w3);
  free(table);
  free(thr);
  if (bad) {
    fprintf(stderr, "a host entry point returned an unexpected code\n");
    return 1;
  }
  printf("ok\n");
  return 0;
}
