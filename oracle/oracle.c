/*
 * CPU ORACLE — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised implementation of what the LSH
 * similarity search of Rong et al., "Locality-Sensitive Hashing for
 * Earthquake Detection: A Case Study of Scaling Data-Driven Science"
 * (VLDB 2018), computes.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may call it; the product library never links it, and it
 * shares no code (kernels, headers, helpers, tables) with the GPU path.
 *
 * Every function names the passage of the paper it follows.  Where the paper
 * is silent or ambiguous the reading taken is stated next to the code:
 *
 *   - hash family: the paper draws its hash mappings from murmurhash
 *     (Appendix D, Algorithm 1); here every function is the universal hash
 *     h_f(x) = (a_f * x + b_f) mod (2^31 - 1) over the 0-based element index x;
 *   - (a_f, b_f) come from a splitmix64 stream: a = 1 + next() mod (p - 1),
 *     b = next() mod p, drawn in function order;
 *   - function-to-table layout: MinHash table u row s uses function u*r + s;
 *     Min-Max table u uses functions u*r/2 + q, row 2q is the min and row
 *     2q+1 the max of that function (section 6.2, Algorithm 1);
 *   - band key (the paper's unspecified hash_combine): the r element indices
 *     attaining the r signature values, packed b = ceil(log2 d) bits each,
 *     row s at bit b*s; when b*r > 64 a chained 64-bit mix of the indices;
 *   - votes(i, j) = number of tables in which i and j share a bucket
 *     (section 6.1 "Search"; section 7.2 triplets); output when
 *     votes >= min_votes ("at least m", section 6.3);
 *   - self-match exclusion (section 7.1): pairs with j - i < min_lag dropped;
 *   - occurrence filter (section 6.5), static reading: a fingerprint is
 *     excluded when some table puts it in a bucket holding more than
 *     occ_num/occ_den of all N fingerprints, i.e. size * occ_den > N * occ_num,
 *     bucket sizes taken before any exclusion; an excluded fingerprint takes
 *     part in no pair of any table.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_P 2147483647ull /* 2^31 - 1 */

enum { ORC_MINHASH = 0, ORC_MINMAX = 1 };

/* ---------------------------------------------------------------------- */
/* Hash parameters                                                         */
/* ---------------------------------------------------------------------- */

/* splitmix64 (Steele, Lea & Flood, OOPSLA 2014): the published generator. */
static uint64_t orc_splitmix64(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* The first `count` outputs of splitmix64 seeded with `seed`. */
void orc_splitmix64_stream(uint64_t seed, uint32_t count, uint64_t *out) {
  uint64_t s = seed;
  for (uint32_t k = 0; k < count; ++k) out[k] = orc_splitmix64(&s);
}

/* Hash mappings (the role of single_hash in Appendix D, Algorithm 1): one
 * (a, b) pair per hash function, in function order. */
void orc_make_hash(uint64_t seed, uint32_t n_funcs, uint32_t *a, uint32_t *b) {
  uint64_t s = seed;
  for (uint32_t f = 0; f < n_funcs; ++f) {
    a[f] = (uint32_t)(1 + orc_splitmix64(&s) % (ORC_P - 1));
    b[f] = (uint32_t)(orc_splitmix64(&s) % ORC_P);
  }
}

/* h_f(x) = (a x + b) mod p, computed directly in 64-bit integers. */
uint32_t orc_hash(uint32_t a, uint32_t b, uint32_t x) {
  return (uint32_t)(((uint64_t)a * x + b) % ORC_P);
}

/* ---------------------------------------------------------------------- */
/* Signatures and band keys (section 6.1 "Hash signature generation",       */
/* section 6.2 Min-Max, Appendix D Algorithm 1)                             */
/* ---------------------------------------------------------------------- */

uint32_t orc_key_bits(uint32_t dim) {
  uint32_t b = 0;
  while ((1ull << b) < dim) ++b;
  return b;
}

/* murmur3's 64-bit finaliser, used only by the chained band key for b*r > 64. */
static uint64_t orc_fmix64(uint64_t k) {
  k ^= k >> 33; k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

/* Band key from the r element indices that attain the r signature values. */
uint64_t orc_band_key(const uint32_t *argx, uint32_t r, uint32_t dim) {
  uint32_t b = orc_key_bits(dim);
  uint64_t k = 0;
  if ((uint64_t)b * r <= 64) {
    for (uint32_t s = 0; s < r; ++s) k |= (uint64_t)argx[s] << (b * s);
  } else {
    for (uint32_t s = 0; s < r; ++s) k = orc_fmix64(k + argx[s] + 1);
  }
  return k;
}

/* orc_band_key applied to n tuples of r indices each (row-major argx[n][r]). */
void orc_band_keys(uint64_t n, const uint32_t *argx, uint32_t r, uint32_t dim, uint64_t *keys) {
  for (uint64_t i = 0; i < n; ++i) keys[i] = orc_band_key(argx + i * r, r, dim);
}

/* Signature of one fingerprint for one table: the r values (MinHash: the
 * min over the set of r functions; Min-Max: min and max of r/2 functions)
 * and the element index attaining each of them. */
static void orc_table_sig(const uint32_t *a, const uint32_t *b, uint32_t scheme, uint32_t r, uint32_t u,
                          const uint16_t *set, uint32_t len, uint32_t *val, uint32_t *argx) {
  for (uint32_t s = 0; s < r; ++s) {
    uint32_t f, want_max;
    if (scheme == ORC_MINHASH) { f = u * r + s; want_max = 0; }
    else { f = u * (r / 2) + s / 2; want_max = s & 1; }
    uint32_t best = 0, bx = 0;
    for (uint32_t q = 0; q < len; ++q) {
      uint32_t h = orc_hash(a[f], b[f], set[q]);
      if (q == 0 || (want_max ? h > best : h < best)) { best = h; bx = set[q]; }
    }
    val[s] = best;
    argx[s] = bx;
  }
}

/* Returns 0, or 1 for invalid arguments / input (empty row, index >= dim,
 * indices not strictly increasing). */
static int orc_check_rows(uint32_t dim, uint64_t n, const uint64_t *offsets, uint32_t nnz, const uint16_t *ind) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t lo = offsets ? offsets[i] : i * nnz, hi = offsets ? offsets[i + 1] : (i + 1) * nnz;
    if (hi <= lo) return 1;
    for (uint64_t q = lo; q < hi; ++q) {
      if (ind[q] >= dim) return 1;
      if (q > lo && ind[q] <= ind[q - 1]) return 1;
    }
  }
  return 0;
}

static int orc_check_hash(uint32_t dim, uint32_t t, uint32_t r, uint32_t scheme) {
  if (dim < 2 || dim > 65536 || t == 0 || r == 0) return 1;
  if (scheme != ORC_MINHASH && scheme != ORC_MINMAX) return 1;
  if (scheme == ORC_MINMAX && (r & 1)) return 1;
  return 0;
}

/* keys[u][i] for u in [0, t) (table-major); sigs (optional) [i][u][r]. */
int orc_signatures(uint32_t dim, uint32_t t, uint32_t r, uint32_t scheme, const uint32_t *a, const uint32_t *b,
                   uint64_t n, const uint64_t *offsets, uint32_t nnz, const uint16_t *ind, uint64_t *keys,
                   uint32_t *sigs) {
  if (orc_check_hash(dim, t, r, scheme) || orc_check_rows(dim, n, offsets, nnz, ind)) return 1;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t ii = 0; ii < (int64_t)n; ++ii) {
    uint64_t i = (uint64_t)ii;
    uint64_t lo = offsets ? offsets[i] : i * nnz, hi = offsets ? offsets[i + 1] : (i + 1) * nnz;
    uint32_t val[64], argx[64];
    for (uint32_t u = 0; u < t; ++u) {
      orc_table_sig(a, b, scheme, r, u, ind + lo, (uint32_t)(hi - lo), val, argx);
      keys[(uint64_t)u * n + i] = orc_band_key(argx, r, dim);
      if (sigs)
        for (uint32_t s = 0; s < r; ++s) sigs[(i * t + u) * r + s] = val[s];
    }
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Hash tables, occurrence filter, candidate pairs and votes                */
/* (section 6.1 "Hash table construction" and "Search"; section 6.5;        */
/*  section 7.1 self-matches; section 7.2 triplet output)                   */
/* ---------------------------------------------------------------------- */

typedef struct {
  uint64_t n_out, e_raw, e_voted, n_distinct, n_flagged, max_bucket;
} orc_stats;

typedef struct { uint64_t key; uint64_t id; } orc_kv;

static int cmp_kv(const void *x, const void *y) {
  const orc_kv *p = (const orc_kv *)x, *q = (const orc_kv *)y;
  if (p->key != q->key) return p->key < q->key ? -1 : 1;
  if (p->id != q->id) return p->id < q->id ? -1 : 1;
  return 0;
}

static int cmp_u64(const void *x, const void *y) {
  uint64_t p = *(const uint64_t *)x, q = *(const uint64_t *)y;
  return p < q ? -1 : (p > q ? 1 : 0);
}

/* Search from precomputed band keys (table-major, keys[u*n + i]).
 * On success *out_pairs holds n_out triplets as (i, j, votes) packed into
 * three arrays allocated with malloc (caller frees with orc_free). */
int orc_search_keys(uint32_t t, uint64_t n, const uint64_t *keys, uint32_t min_lag, uint32_t min_votes,
                    uint32_t occ_num, uint32_t occ_den, uint32_t **out_i, uint32_t **out_j, uint8_t **out_v,
                    orc_stats *st, uint8_t *flags_out) {
  memset(st, 0, sizeof(*st));
  *out_i = NULL; *out_j = NULL; *out_v = NULL;
  if (t == 0 || t > 255 || min_votes == 0 || n >= (1ull << 31)) return 1;

  /* Hash tables: for each table, fingerprints grouped by band key.  Sorting
   * (key, id) pairs places each bucket's members next to each other with
   * ids ascending. */
  orc_kv **tab = (orc_kv **)malloc(t * sizeof(orc_kv *));
  for (uint32_t u = 0; u < t; ++u) {
    tab[u] = (orc_kv *)malloc((n ? n : 1) * sizeof(orc_kv));
    for (uint64_t i = 0; i < n; ++i) { tab[u][i].key = keys[(uint64_t)u * n + i]; tab[u][i].id = i; }
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int u = 0; u < (int)t; ++u) qsort(tab[u], n, sizeof(orc_kv), cmp_kv);

  /* Bucket sizes, raw candidate count and the occurrence filter. */
  uint8_t *flag = (uint8_t *)calloc(n ? n : 1, 1);
  for (uint32_t u = 0; u < t; ++u) {
    uint64_t s = 0;
    while (s < n) {
      uint64_t e = s + 1;
      while (e < n && tab[u][e].key == tab[u][s].key) ++e;
      uint64_t size = e - s;
      st->e_raw += size * (size - 1) / 2;
      if (size > st->max_bucket) st->max_bucket = size;
      if (occ_den && (unsigned __int128)size * occ_den > (unsigned __int128)n * occ_num)
        for (uint64_t q = s; q < e; ++q) flag[tab[u][q].id] = 1;
      s = e;
    }
  }
  for (uint64_t i = 0; i < n; ++i) st->n_flagged += flag[i];

  /* Candidate pairs: every pair of distinct, unflagged members of a bucket
   * with j - i >= min_lag, once per table in which they share a bucket. */
  uint64_t cap = 1024, cnt = 0;
  uint64_t *pairs = (uint64_t *)malloc(cap * sizeof(uint64_t));
  for (uint32_t u = 0; u < t; ++u) {
    uint64_t s = 0;
    while (s < n) {
      uint64_t e = s + 1;
      while (e < n && tab[u][e].key == tab[u][s].key) ++e;
      for (uint64_t x = s; x < e; ++x)
        for (uint64_t y = x + 1; y < e; ++y) {
          uint64_t i = tab[u][x].id, j = tab[u][y].id;
          if (j - i < min_lag || flag[i] || flag[j]) continue;
          if (cnt == cap) { cap *= 2; pairs = (uint64_t *)realloc(pairs, cap * sizeof(uint64_t)); }
          pairs[cnt++] = (i << 32) | j;
        }
      s = e;
    }
  }
  for (uint32_t u = 0; u < t; ++u) free(tab[u]);
  free(tab);

  /* Votes: the number of tables that emitted a pair is the number of
   * tables in which its two fingerprints share a bucket. */
  qsort(pairs, cnt, sizeof(uint64_t), cmp_u64);
  st->e_voted = cnt;
  uint64_t outcap = 16, nout = 0;
  uint32_t *oi = (uint32_t *)malloc(outcap * 4), *oj = (uint32_t *)malloc(outcap * 4);
  uint8_t *ov = (uint8_t *)malloc(outcap);
  uint64_t s = 0;
  while (s < cnt) {
    uint64_t e = s + 1;
    while (e < cnt && pairs[e] == pairs[s]) ++e;
    st->n_distinct += 1;
    uint64_t votes = e - s;
    if (votes >= min_votes) {
      if (nout == outcap) {
        outcap *= 2;
        oi = (uint32_t *)realloc(oi, outcap * 4); oj = (uint32_t *)realloc(oj, outcap * 4);
        ov = (uint8_t *)realloc(ov, outcap);
      }
      oi[nout] = (uint32_t)(pairs[s] >> 32); oj[nout] = (uint32_t)pairs[s]; ov[nout] = (uint8_t)votes;
      ++nout;
    }
    s = e;
  }
  free(pairs);
  st->n_out = nout;
  if (flags_out) memcpy(flags_out, flag, n);
  free(flag);
  *out_i = oi; *out_j = oj; *out_v = ov;
  return 0;
}

/* Full search: signatures for all t tables, then orc_search_keys. */
int orc_search(uint32_t dim, uint32_t t, uint32_t r, uint32_t scheme, const uint32_t *a, const uint32_t *b,
               uint64_t n, const uint64_t *offsets, uint32_t nnz, const uint16_t *ind, uint32_t min_lag,
               uint32_t min_votes, uint32_t occ_num, uint32_t occ_den, uint32_t **out_i, uint32_t **out_j,
               uint8_t **out_v, orc_stats *st) {
  uint64_t *keys = (uint64_t *)malloc((n ? n : 1) * (uint64_t)t * sizeof(uint64_t));
  int rc = orc_signatures(dim, t, r, scheme, a, b, n, offsets, nnz, ind, keys, NULL);
  if (rc == 0)
    rc = orc_search_keys(t, n, keys, min_lag, min_votes, occ_num, occ_den, out_i, out_j, out_v, st, NULL);
  free(keys);
  return rc;
}

/* votes(i, j) straight from the definition: the number of tables whose band
 * keys of i and j are equal. */
uint32_t orc_pair_votes(uint32_t t, uint64_t n, const uint64_t *keys, uint64_t i, uint64_t j) {
  uint32_t v = 0;
  for (uint32_t u = 0; u < t; ++u) v += keys[(uint64_t)u * n + i] == keys[(uint64_t)u * n + j];
  return v;
}

void orc_free(void *p) { free(p); }

/* Threads the OpenMP loops of the oracle use. */
int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
