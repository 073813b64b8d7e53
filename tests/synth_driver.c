/*
 * Test driver for the synthetic generator (synth/synth.c), built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_synth_sanitized.py.  It generates slices of the twelve-station
 * batched workload (stations of 1-8, 10, 12, 14 and 16 M rows, uniform
 * 200-of-4096 background, 50 sources x 5 copies keeping 160 bits, seeds
 * 1030 + s) from twelve host threads at once, each call running its own
 * OpenMP team, then generates every slice again from one thread and checks
 * that both runs wrote the same rows.  Exit status 0 on success.
 *
 * usage: synth_driver ROWS_PER_SLICE
 */
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint64_t n;
  uint32_t dim, nnz;
  uint64_t seed;
  uint32_t markov_keep, n_sources, rep_min, rep_max, plant_keep, jac_lo_milli, jac_hi_milli, noise_permille,
      noise_keep;
  uint64_t chain_len;
  uint32_t channel;
} synth_spec;

int synth_generate_range(const synth_spec *sp, uint64_t lo, uint64_t hi, uint16_t *out, int32_t *label);

enum { kStations = 12 };
static const uint64_t kMillions[kStations] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16};

typedef struct {
  synth_spec spec;
  uint64_t lo, hi;
  uint16_t *rows;
  int32_t *label;
  int rc;
} job_t;

static void *run(void *p) {
  job_t *j = (job_t *)p;
  j->rc = synth_generate_range(&j->spec, j->lo, j->hi, j->rows, j->label);
  return NULL;
}

int main(int argc, char **argv) {
  const uint64_t slice = argc > 1 ? strtoull(argv[1], NULL, 10) : 20000;
  job_t jobs[kStations], again[kStations];
  pthread_t th[kStations];
  for (int s = 0; s < kStations; ++s) {
    synth_spec sp;
    memset(&sp, 0, sizeof sp);
    sp.n = kMillions[s] * 1000000ull;
    sp.dim = 4096;
    sp.nnz = 200;
    sp.seed = 1030 + (uint64_t)s;
    sp.n_sources = 50;
    sp.rep_min = sp.rep_max = 5;
    sp.plant_keep = 160;
    /* a slice from the middle of the station: planted slots fall inside it
       only by chance, so the last slice also covers the station's end */
    const uint64_t lo = s == kStations - 1 ? sp.n - slice : (sp.n / 2) - slice / 2;
    for (int k = 0; k < 2; ++k) {
      job_t *j = k ? &again[s] : &jobs[s];
      j->spec = sp;
      j->lo = lo;
      j->hi = lo + slice;
      j->rows = (uint16_t *)malloc(slice * sp.nnz * sizeof(uint16_t));
      j->label = (int32_t *)malloc(slice * sizeof(int32_t));
      if (!j->rows || !j->label) {
        fprintf(stderr, "allocation failed\n");
        return 2;
      }
    }
  }
  for (int s = 0; s < kStations; ++s) pthread_create(&th[s], NULL, run, &jobs[s]);
  for (int s = 0; s < kStations; ++s) pthread_join(th[s], NULL);
  for (int s = 0; s < kStations; ++s) run(&again[s]);
  int bad = 0;
  for (int s = 0; s < kStations; ++s) {
    if (jobs[s].rc || again[s].rc) {
      fprintf(stderr, "station %d: generator returned %d / %d\n", s, jobs[s].rc, again[s].rc);
      bad = 1;
      continue;
    }
    if (memcmp(jobs[s].rows, again[s].rows, slice * 200 * sizeof(uint16_t)) ||
        memcmp(jobs[s].label, again[s].label, slice * sizeof(int32_t))) {
      fprintf(stderr, "station %d: concurrent and single-threaded rows differ\n", s);
      bad = 1;
    }
    free(jobs[s].rows);
    free(jobs[s].label);
    free(again[s].rows);
    free(again[s].label);
  }
  if (!bad) printf("synth_driver ok: %d stations x %llu rows\n", kStations, (unsigned long long)slice);
  return bad;
}
