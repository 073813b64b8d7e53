/*
 * Seeded synthetic fingerprint generator.
 *
 * This module produces the inputs that both the CPU oracle and the GPU path
 * consume.  It holds none of the search method's arithmetic: no hash
 * functions, no signatures, no buckets, no votes.  It only draws sparse
 * binary fingerprints (sorted uint16 index lists with a fixed number of set
 * bits per row, the structure the paper's fingerprinting stage yields: every
 * fingerprint carries the same number of non-zeros) with the temporal
 * structure of continuous seismic data:
 *
 *   - background rows that are either independent uniform k-subsets of [0,d)
 *     or a Markov chain in which each row keeps a fixed number of the
 *     previous row's bits (neighbouring fingerprints overlap strongly, the
 *     paper reports over 60 % overlap in one example, section 6.2);
 *   - rare repeating sources: a template set copied into random time slots,
 *     each copy keeping an exact number of template bits so that its Jaccard
 *     similarity to the template is known exactly;
 *   - (test-only) a repeating-noise source that fills a fraction of all slots
 *     with near-identical copies, to exercise the occurrence filter
 *     (section 6.5).
 *
 * Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).  Every random
 * decision is drawn from a stream keyed by (seed, purpose tag, index), so a
 * row's content depends only on the seed and its own position, never on
 * thread scheduling.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define TAG_BG 1ull      /* independent background row, indexed by row */
#define TAG_CHAIN 2ull   /* the Markov chain (one sequential stream)    */
#define TAG_SRC 3ull     /* per-source repeat count                     */
#define TAG_TPL 4ull     /* per-source template                         */
#define TAG_SLOT 5ull    /* slot assignment (one sequential stream)     */
#define TAG_COPY 6ull    /* per-slot copy content                       */
#define TAG_NOISE 7ull   /* noise template                              */

typedef struct {
  uint64_t n;             /* rows                                          */
  uint32_t dim;           /* d, 2..65536                                   */
  uint32_t nnz;           /* set bits per row                              */
  uint64_t seed;
  uint32_t markov_keep;   /* 0: independent rows; else bits kept from the previous row */
  uint32_t n_sources;     /* planted repeating sources                     */
  uint32_t rep_min;       /* copies per source ~ U{rep_min..rep_max}       */
  uint32_t rep_max;
  uint32_t plant_keep;    /* >0: each copy keeps exactly this many template bits */
  uint32_t jac_lo_milli;  /* plant_keep == 0: per-copy Jaccard ~ U[lo,hi]/1000 */
  uint32_t jac_hi_milli;
  uint32_t noise_permille;/* test-only: rows replaced by near-copies of one noise template */
  uint32_t noise_keep;    /* template bits each noise copy keeps           */
  uint64_t chain_len;     /* Markov only: 0 = one chain over all rows; else independent
                             chains of chain_len rows, chain c drawn from stream c    */
  uint32_t channel;       /* channel of a multi-channel station: the planted sources
                             (slots, repeat counts, templates) are shared by every
                             channel of a seed, while the background rows and the
                             content of each planted copy are drawn per channel;
                             channel 0 is the single-channel workload            */
} synth_spec;

typedef struct { uint64_t s; } rng_t;

static inline uint64_t sm64_next(rng_t *r) {
  uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* A stream keyed by (seed, tag, idx): the state is one splitmix64 output of a
 * combination of the three, so distinct keys give unrelated streams. */
static inline rng_t stream_for(uint64_t seed, uint64_t tag, uint64_t idx) {
  rng_t r;
  r.s = seed ^ (tag << 56) ^ (idx * 0xD6E8FEB86659FD93ull);
  r.s = sm64_next(&r);
  return r;
}

/* Seed of the per-channel streams (background rows, copy content). */
static inline uint64_t channel_seed(const synth_spec *sp) {
  return sp->channel ? sp->seed ^ ((uint64_t)sp->channel * 0xA24BAED4963EE407ull) : sp->seed;
}

/* Uniform integer in [0, n) by the multiply-shift map of a 32-bit draw. */
static inline uint32_t below(rng_t *r, uint32_t n) {
  return (uint32_t)(((sm64_next(r) >> 32) * (uint64_t)n) >> 32);
}

/* Uniform double in [0,1) from the top 53 bits. */
static inline double unit(rng_t *r) {
  return (double)(sm64_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

static inline int bm_test(const uint64_t *bm, uint32_t x) { return (bm[x >> 6] >> (x & 63)) & 1; }
static inline void bm_set(uint64_t *bm, uint32_t x) { bm[x >> 6] |= 1ull << (x & 63); }

/* Write the set bits of a bitmap in increasing order. */
static void bm_emit(const uint64_t *bm, uint32_t words, uint16_t *out) {
  uint32_t k = 0;
  for (uint32_t w = 0; w < words; ++w) {
    uint64_t v = bm[w];
    while (v) {
      int b = __builtin_ctzll(v);
      out[k++] = (uint16_t)(w * 64 + b);
      v &= v - 1;
    }
  }
}

/* Floyd's algorithm: a uniform k-subset of [0, d) into the bitmap. */
static void floyd(rng_t *r, uint32_t d, uint32_t k, uint64_t *bm) {
  for (uint32_t j = d - k; j < d; ++j) {
    uint32_t t = below(r, j + 1);
    if (bm_test(bm, t)) bm_set(bm, j); else bm_set(bm, t);
  }
}

/* Draw `cnt` new elements uniformly from [0,d) minus the `excl` bitmap,
 * setting them in both `excl` and `out`. */
static void draw_outside(rng_t *r, uint32_t d, uint32_t cnt, uint64_t *excl, uint64_t *out) {
  for (uint32_t c = 0; c < cnt; ++c) {
    uint32_t x;
    do { x = below(r, d); } while (bm_test(excl, x));
    bm_set(excl, x);
    bm_set(out, x);
  }
}

/* Keep exactly `keep` of the `k` elements of `src` (partial Fisher-Yates on a
 * scratch copy), setting the kept ones in `out`. */
static void keep_subset(rng_t *r, const uint16_t *src, uint32_t k, uint32_t keep, uint16_t *scratch,
                        uint64_t *out) {
  memcpy(scratch, src, k * sizeof(uint16_t));
  for (uint32_t q = 0; q < keep; ++q) {
    uint32_t pick = q + below(r, k - q);
    uint16_t t = scratch[q]; scratch[q] = scratch[pick]; scratch[pick] = t;
    bm_set(out, scratch[q]);
  }
}

/* Copy of a template keeping `keep` template bits; the rest are drawn from
 * outside the template, so |copy ∩ template| = keep exactly. */
static int make_copy(rng_t *r, uint32_t d, uint32_t k, const uint16_t *tpl, uint32_t keep, uint16_t *out) {
  uint32_t words = (d + 63) / 64;
  uint64_t *excl = (uint64_t *)calloc(words, 8);
  uint64_t *cur = (uint64_t *)calloc(words, 8);
  uint16_t *scratch = (uint16_t *)malloc(k * sizeof(uint16_t));
  if (!excl || !cur || !scratch) {
    free(excl); free(cur); free(scratch);
    return 1;
  }
  for (uint32_t q = 0; q < k; ++q) bm_set(excl, tpl[q]);
  keep_subset(r, tpl, k, keep, scratch, cur);
  draw_outside(r, d, k - keep, excl, cur);
  bm_emit(cur, words, out);
  free(excl); free(cur); free(scratch);
  return 0;
}

static int uniform_row(rng_t *r, uint32_t d, uint32_t k, uint16_t *out) {
  uint32_t words = (d + 63) / 64;
  uint64_t *bm = (uint64_t *)calloc(words, 8);
  if (!bm) return 1;
  floyd(r, d, k, bm);
  bm_emit(bm, words, out);
  free(bm);
  return 0;
}

int synth_check(const synth_spec *sp) {
  if (!sp || sp->dim < 2 || sp->dim > 65536 || sp->nnz == 0 || sp->nnz > sp->dim) return 1;
  if (sp->markov_keep > sp->nnz) return 1;
  if (sp->markov_keep && (sp->dim - sp->nnz) < (sp->nnz - sp->markov_keep)) return 1;
  if (sp->n_sources && (sp->rep_min == 0 || sp->rep_max < sp->rep_min)) return 1;
  if (sp->plant_keep > sp->nnz) return 1;
  if (sp->noise_keep > sp->nnz) return 1;
  if (sp->jac_hi_milli > 1000 || sp->jac_lo_milli > sp->jac_hi_milli) return 1;
  if ((sp->n_sources || sp->noise_permille) && sp->dim - sp->nnz < sp->nnz)
    return 1; /* copies need room outside the template */
  return 0;
}

/* Number of planted rows (sources and noise) the spec asks for. */
uint64_t synth_planted_count(const synth_spec *sp) {
  uint64_t tot = 0;
  for (uint32_t s = 0; s < sp->n_sources; ++s) {
    rng_t r = stream_for(sp->seed, TAG_SRC, s);
    tot += sp->rep_min + below(&r, sp->rep_max - sp->rep_min + 1);
  }
  tot += sp->n * (uint64_t)sp->noise_permille / 1000;
  return tot;
}

/* Fill rows [lo, hi) of the data set described by `sp` into out[(hi-lo)][nnz]
 * and, when `label` is non-NULL, label[(hi-lo)] with -1 (background), the
 * source id (planted copy) or -2 (noise copy).  Returns 0 on success, 1 for
 * an invalid spec or range, 2 when the planted rows exceed half the slots,
 * 3 when a host allocation fails. */
int synth_generate_range(const synth_spec *sp, uint64_t lo, uint64_t hi, uint16_t *out, int32_t *label) {
  if (synth_check(sp) || lo > hi || hi > sp->n || (!out && hi > lo)) return 1;
  const uint32_t d = sp->dim, k = sp->nnz, words = (d + 63) / 64;
  const uint64_t cnt = hi - lo;
  int oom = 0; /* set by any thread whose allocation failed */

  /* 1. background */
  if (sp->markov_keep == 0) {
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < (int64_t)cnt; ++q) {
      rng_t r = stream_for(channel_seed(sp), TAG_BG, lo + (uint64_t)q);
      if (uniform_row(&r, d, k, out + (uint64_t)q * k)) {
#pragma omp atomic write
        oom = 1;
      }
    }
  } else {
    /* chains: one over all rows, or independent chains of chain_len rows
       (those that meet [lo, hi) are walked in parallel from their start) */
    const uint64_t clen = sp->chain_len ? sp->chain_len : sp->n;
    const int64_t c0 = (int64_t)(lo / clen), c1 = (int64_t)((hi - 1) / clen) + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = c0; c < c1; ++c) {
      rng_t r = stream_for(channel_seed(sp), TAG_CHAIN, (uint64_t)c);
      uint16_t *prev = (uint16_t *)malloc(k * sizeof(uint16_t));
      uint16_t *cur = (uint16_t *)malloc(k * sizeof(uint16_t));
      uint16_t *scratch = (uint16_t *)malloc(k * sizeof(uint16_t));
      uint64_t *excl = (uint64_t *)calloc(words, 8);
      uint64_t *bm = (uint64_t *)calloc(words, 8);
      const uint64_t start = (uint64_t)c * clen;
      const uint64_t stop = start + clen < hi ? start + clen : hi;
      if (!prev || !cur || !scratch || !excl || !bm || uniform_row(&r, d, k, prev)) {
        free(prev); free(cur); free(scratch); free(excl); free(bm);
#pragma omp atomic write
        oom = 1;
        continue;
      }
      for (uint64_t i = start; i < stop; ++i) {
        if (i > start) {
          memset(excl, 0, words * 8);
          memset(bm, 0, words * 8);
          for (uint32_t q = 0; q < k; ++q) bm_set(excl, prev[q]);
          keep_subset(&r, prev, k, sp->markov_keep, scratch, bm);
          draw_outside(&r, d, k - sp->markov_keep, excl, bm);
          bm_emit(bm, words, cur);
          uint16_t *t = prev; prev = cur; cur = t;
        }
        if (i >= lo) memcpy(out + (i - lo) * k, prev, k * sizeof(uint16_t));
      }
      free(prev); free(cur); free(scratch); free(excl); free(bm);
    }
  }
  if (oom) return 3;
  if (label)
    for (uint64_t q = 0; q < cnt; ++q) label[q] = -1;

  /* 2. slots for planted copies: one sequential stream over (source, copy) in
   *    order, then the noise copies; every slot is distinct. */
  uint64_t total = synth_planted_count(sp);
  if (total == 0) return 0;
  if (total > sp->n / 2) return 2;
  uint64_t nwords = (sp->n + 63) / 64;
  uint64_t *used = (uint64_t *)calloc(nwords, 8);
  uint64_t *slot = (uint64_t *)malloc(total * 8);
  int32_t *who = (int32_t *)malloc(total * 4);
  uint32_t *keep = (uint32_t *)malloc(total * 4);
  uint16_t *tpl = (uint16_t *)malloc(((uint64_t)sp->n_sources + 1) * k * sizeof(uint16_t));
  if (!used || !slot || !who || !keep || !tpl) {
    free(used); free(slot); free(who); free(keep); free(tpl);
    return 3;
  }
  rng_t rs = stream_for(sp->seed, TAG_SLOT, 0);
  uint64_t m = 0;
  for (uint32_t s = 0; s < sp->n_sources; ++s) {
    rng_t rr = stream_for(sp->seed, TAG_SRC, s);
    uint32_t reps = sp->rep_min + below(&rr, sp->rep_max - sp->rep_min + 1);
    for (uint32_t c = 0; c < reps; ++c) {
      uint64_t x;
      do { x = ((sm64_next(&rs) >> 11) * (unsigned __int128)sp->n) >> 53; } while ((used[x >> 6] >> (x & 63)) & 1);
      used[x >> 6] |= 1ull << (x & 63);
      slot[m] = x; who[m] = (int32_t)s;
      if (sp->plant_keep) {
        keep[m] = sp->plant_keep;
      } else {
        double J = (sp->jac_lo_milli + (sp->jac_hi_milli - sp->jac_lo_milli) * unit(&rs)) / 1000.0;
        double mm = 2.0 * k * J / (1.0 + J) + 0.5;
        uint32_t mk = (uint32_t)mm;
        keep[m] = mk > k ? k : mk;
      }
      ++m;
    }
  }
  uint64_t nnoise = sp->n * (uint64_t)sp->noise_permille / 1000;
  for (uint64_t c = 0; c < nnoise; ++c) {
    uint64_t x;
    do { x = ((sm64_next(&rs) >> 11) * (unsigned __int128)sp->n) >> 53; } while ((used[x >> 6] >> (x & 63)) & 1);
    used[x >> 6] |= 1ull << (x & 63);
    slot[m] = x; who[m] = -2; keep[m] = sp->noise_keep; ++m;
  }

  /* 3. copy content, keyed by slot */
  for (uint32_t s = 0; s < sp->n_sources; ++s) {
    rng_t rt = stream_for(sp->seed, TAG_TPL, s);
    oom |= uniform_row(&rt, d, k, tpl + (uint64_t)s * k);
  }
  {
    rng_t rt = stream_for(sp->seed, TAG_NOISE, 0);
    oom |= uniform_row(&rt, d, k, tpl + (uint64_t)sp->n_sources * k);
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < (int64_t)m; ++q) {
    uint64_t x = slot[q];
    if (x < lo || x >= hi) continue;
    rng_t rc = stream_for(channel_seed(sp), TAG_COPY, x);
    const uint16_t *t = tpl + (uint64_t)(who[q] >= 0 ? (uint32_t)who[q] : sp->n_sources) * k;
    if (make_copy(&rc, d, k, t, keep[q], out + (x - lo) * k)) {
#pragma omp atomic write
      oom = 1;
    }
    if (label) label[x - lo] = who[q];
  }
  free(used); free(slot); free(who); free(keep); free(tpl);
  return oom ? 3 : 0;
}

int synth_generate(const synth_spec *sp, uint16_t *out, int32_t *label) {
  return synth_generate_range(sp, 0, sp ? sp->n : 0, out, label);
}

/* ---------------------------------------------------------------------------
 * Synthetic continuous waveforms (input of the fingerprint extraction).
 *
 * One channel of ground motion sampled at a fixed rate: Gaussian background
 * noise, plus repeating sources whose waveform (a template: a P wave packet
 * followed by a larger, slower S wave packet, each a decaying sinusoid) is
 * added at random times with random amplitudes.  Sample k of the noise is
 * drawn from a stream keyed by (seed, k), so any range of samples can be
 * generated on its own; the events are drawn from streams keyed by the seed
 * and the source index.  Events never overlap one another.
 * ------------------------------------------------------------------------- */
#define TAG_WNOISE 8ull  /* background sample k                        */
#define TAG_WSRC 9ull    /* source s: repeat count and template shape    */
#define TAG_WSLOT 10ull  /* event start times (one sequential stream)    */
#define TAG_WAMP 11ull   /* event e: amplitude                           */

typedef struct {
  uint64_t n;            /* samples                                    */
  uint64_t seed;
  uint32_t n_sources;    /* repeating sources                          */
  uint32_t rep_min, rep_max;
  uint32_t event_len;    /* samples per event                          */
  float noise_std;       /* background standard deviation              */
  float amp_lo, amp_hi;  /* event amplitude ~ U[amp_lo, amp_hi]        */
  uint32_t reserved;
} synth_wave_spec;

typedef struct {
  float p_at, s_at, p_f, s_f, p_tau, s_tau, p_amp, s_amp;  /* samples, cycles per sample, samples */
} wave_tpl;

static void wave_template(uint64_t seed, uint32_t s, wave_tpl *t, uint32_t len) {
  rng_t r = stream_for(seed, TAG_WSRC, s);
  (void)sm64_next(&r); /* the repeat count's draw */
  t->p_at = (float)(0.10 + 0.05 * unit(&r)) * (float)len;
  t->s_at = t->p_at + (float)(0.20 + 0.15 * unit(&r)) * (float)len;
  t->p_f = (float)((5.0 + 7.0 * unit(&r)) / 100.0);  /* 5-12 Hz at 100 Hz */
  t->s_f = (float)((2.0 + 6.0 * unit(&r)) / 100.0);  /* 2-8 Hz */
  t->p_tau = (float)(0.03 + 0.05 * unit(&r)) * (float)len;
  t->s_tau = (float)(0.06 + 0.10 * unit(&r)) * (float)len;
  t->p_amp = (float)(0.5 + 0.5 * unit(&r));
  t->s_amp = (float)(1.0 + 1.0 * unit(&r));
}

static float wave_template_at(const wave_tpl *t, uint32_t q) {
  double v = 0.0;
  const double x = (double)q;
  if (x >= t->p_at) v += t->p_amp * exp(-(x - t->p_at) / t->p_tau) * sin(6.283185307179586 * t->p_f * (x - t->p_at));
  if (x >= t->s_at) v += t->s_amp * exp(-(x - t->s_at) / t->s_tau) * sin(6.283185307179586 * t->s_f * (x - t->s_at));
  return (float)v;
}

static uint32_t wave_repeats(const synth_wave_spec *sp, uint32_t s) {
  rng_t r = stream_for(sp->seed, TAG_WSRC, s);
  return sp->rep_min + below(&r, sp->rep_max - sp->rep_min + 1);
}

/* Number of events the spec places (sum of the sources' repeat counts). */
uint64_t synth_wave_events(const synth_wave_spec *sp) {
  uint64_t e = 0;
  for (uint32_t s = 0; s < sp->n_sources; ++s) e += wave_repeats(sp, s);
  return e;
}

/* Samples [lo, hi) into out[hi - lo]; when start/source are non-NULL they
 * receive every event's first sample and source (synth_wave_events entries,
 * ordered by source then repeat).  Returns 0, 1 for an invalid spec or range,
 * 2 when the events do not fit without overlap, 3 when an allocation fails. */
int synth_waveform_range(const synth_wave_spec *sp, uint64_t lo, uint64_t hi, float *out, uint64_t *start,
                         uint32_t *source) {
  if (!sp || lo > hi || hi > sp->n || (!out && hi > lo) || sp->event_len == 0 || sp->rep_min == 0 ||
      sp->rep_max < sp->rep_min || sp->amp_hi < sp->amp_lo)
    return 1;
  const uint64_t ne = synth_wave_events(sp);
  const uint64_t slots = sp->n / sp->event_len; /* events start on distinct multiples of event_len */
  if (ne > slots / 2) return 2;
  /* 1. background */
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < (int64_t)(hi - lo); ++q) {
    rng_t r = stream_for(sp->seed, TAG_WNOISE, lo + (uint64_t)q);
    const double u1 = (double)((sm64_next(&r) >> 11) + 1) * (1.0 / 9007199254740993.0);
    const double u2 = unit(&r);
    out[q] = (float)(sp->noise_std * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
  }
  /* 2. events: distinct slots drawn in order, one per event */
  uint64_t *slot = (uint64_t *)malloc((ne ? ne : 1) * sizeof(uint64_t));
  uint8_t *used = (uint8_t *)calloc(slots ? slots : 1, 1);
  wave_tpl *tpl = (wave_tpl *)malloc((sp->n_sources ? sp->n_sources : 1) * sizeof(wave_tpl));
  if (!slot || !used || !tpl) { free(slot); free(used); free(tpl); return 3; }
  rng_t rs = stream_for(sp->seed, TAG_WSLOT, 0);
  for (uint64_t e = 0; e < ne; ++e) {
    uint64_t x;
    do { x = ((sm64_next(&rs) >> 11) % slots); } while (used[x]);
    used[x] = 1;
    slot[e] = x * sp->event_len;
  }
  for (uint32_t s = 0; s < sp->n_sources; ++s) wave_template(sp->seed, s, &tpl[s], sp->event_len);
  uint64_t e = 0;
  for (uint32_t s = 0; s < sp->n_sources; ++s) {
    const uint32_t reps = wave_repeats(sp, s);
    for (uint32_t c = 0; c < reps; ++c, ++e) {
      const uint64_t t0 = slot[e];
      if (start) start[e] = t0;
      if (source) source[e] = s;
      if (t0 + sp->event_len <= lo || t0 >= hi) continue;
      rng_t ra = stream_for(sp->seed, TAG_WAMP, e);
      const float amp = (float)(sp->amp_lo + (sp->amp_hi - sp->amp_lo) * unit(&ra));
      const uint64_t a = t0 > lo ? t0 : lo, b = t0 + sp->event_len < hi ? t0 + sp->event_len : hi;
      for (uint64_t k = a; k < b; ++k) out[k - lo] += amp * wave_template_at(&tpl[s], (uint32_t)(k - t0));
    }
  }
  free(slot); free(used); free(tpl);
  return 0;
}
