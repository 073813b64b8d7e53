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

/* One hash table (section 6.1 "Hash table construction"): the n fingerprints
 * as (band key, id) sorted by key, then id, so that each bucket's members
 * are adjacent with ids ascending. */
static void orc_table_sort(uint64_t n, const uint64_t *keys_u, orc_kv *tab) {
  for (uint64_t i = 0; i < n; ++i) { tab[i].key = keys_u[i]; tab[i].id = i; }
  qsort(tab, n, sizeof(orc_kv), cmp_kv);
}

/* Bucket sizes of one sorted table: adds C(size, 2) of every bucket to
 * *e_raw, raises *max_bucket to the largest size, and (occurrence filter,
 * section 6.5) sets flag[id] for every member of a bucket whose size
 * exceeds occ_num/occ_den of the n fingerprints (occ_den == 0: no filter). */
static void orc_table_buckets(uint64_t n, const orc_kv *tab, uint32_t occ_num, uint32_t occ_den, uint8_t *flag,
                              uint64_t *e_raw, uint64_t *max_bucket) {
  uint64_t s = 0;
  while (s < n) {
    uint64_t e = s + 1;
    while (e < n && tab[e].key == tab[s].key) ++e;
    uint64_t size = e - s;
    *e_raw += size * (size - 1) / 2;
    if (size > *max_bucket) *max_bucket = size;
    if (occ_den && (unsigned __int128)size * occ_den > (unsigned __int128)n * occ_num)
      for (uint64_t q = s; q < e; ++q) flag[tab[q].id] = 1;
    s = e;
  }
}

/* A growable list of pairs packed as i << 32 | j. */
typedef struct { uint64_t *p; uint64_t cnt, cap; int oom; } orc_pairs;

static void orc_pairs_push(orc_pairs *v, uint64_t x) {
  if (v->oom) return;
  if (v->cnt == v->cap) {
    uint64_t nc = v->cap ? 2 * v->cap : 1024;
    uint64_t *np = (uint64_t *)realloc(v->p, nc * sizeof(uint64_t));
    if (!np) { v->oom = 1; return; }
    v->p = np;
    v->cap = nc;
  }
  v->p[v->cnt++] = x;
}

/* Candidate pairs of one sorted table (section 6.1 "Search"; self-matches,
 * section 7.1): every pair of members i < j of a bucket with j - i >= min_lag,
 * neither member flagged (flag may be NULL: no exclusion), and i in
 * [i_lo, i_hi), appended to *out. */
static void orc_table_pairs(uint64_t n, const orc_kv *tab, const uint8_t *flag, uint32_t min_lag, uint64_t i_lo,
                            uint64_t i_hi, orc_pairs *out) {
  uint64_t s = 0;
  while (s < n) {
    uint64_t e = s + 1;
    while (e < n && tab[e].key == tab[s].key) ++e;
    for (uint64_t x = s; x < e; ++x) {
      uint64_t i = tab[x].id;
      if (i < i_lo || i >= i_hi || (flag && flag[i])) continue;
      for (uint64_t y = x + 1; y < e; ++y) {
        uint64_t j = tab[y].id;
        if (j - i < min_lag || (flag && flag[j])) continue;
        orc_pairs_push(out, (i << 32) | j);
      }
    }
    s = e;
  }
}

/* Output arrays that grow as pairs are appended. */
typedef struct { uint32_t *i, *j; uint8_t *v; uint64_t cnt, cap; int oom; } orc_out;

static void orc_out_push(orc_out *o, uint32_t i, uint32_t j, uint8_t v) {
  if (o->oom) return;
  if (o->cnt == o->cap) {
    uint64_t nc = o->cap ? 2 * o->cap : 16;
    uint32_t *ni = (uint32_t *)realloc(o->i, nc * 4);
    if (ni) o->i = ni;
    uint32_t *nj = (uint32_t *)realloc(o->j, nc * 4);
    if (nj) o->j = nj;
    uint8_t *nv = (uint8_t *)realloc(o->v, nc);
    if (nv) o->v = nv;
    if (!ni || !nj || !nv) { o->oom = 1; return; }
    o->cap = nc;
  }
  o->i[o->cnt] = i; o->j[o->cnt] = j; o->v[o->cnt] = v;
  ++o->cnt;
}

/* Votes (section 6.1 "Search"; section 7.2 triplets): every table that
 * found a pair emitted it once, so after sorting the emitted pairs a pair
 * that appears k times shares a bucket in k tables.  Pairs with a flagged
 * member (flag may be NULL) are dropped; every other pair adds k to e_voted
 * and one to n_distinct, and is appended to the output when k >= min_votes
 * ("at least m", section 6.3).  Sorts pairs[] in place. */
static void orc_votes(uint64_t *pairs, uint64_t cnt, const uint8_t *flag, uint32_t min_votes, orc_out *out,
                      orc_stats *st) {
  qsort(pairs, cnt, sizeof(uint64_t), cmp_u64);
  uint64_t s = 0;
  while (s < cnt) {
    uint64_t e = s + 1;
    while (e < cnt && pairs[e] == pairs[s]) ++e;
    uint32_t i = (uint32_t)(pairs[s] >> 32), j = (uint32_t)pairs[s];
    if (!flag || (!flag[i] && !flag[j])) {
      uint64_t votes = e - s;
      st->e_voted += votes;
      st->n_distinct += 1;
      if (votes >= min_votes) orc_out_push(out, i, j, (uint8_t)votes);
    }
    s = e;
  }
}

/* Search from precomputed band keys (table-major, keys[u*n + i]).
 * The pairs are counted in n_parts vote partitions, consecutive ranges of
 * the smaller id i (a pair belongs to the partition of its i), one after
 * another; each partition's output is sorted by (i, j), so their
 * concatenation is the output of the whole search, and the counters add up
 * (partitioning only bounds memory, as in section 6.4).
 * On success the output triplets (i, j, votes) are in three arrays
 * allocated with malloc (caller frees with orc_free). */
int orc_search_keys(uint32_t t, uint64_t n, const uint64_t *keys, uint32_t min_lag, uint32_t min_votes,
                    uint32_t occ_num, uint32_t occ_den, uint32_t n_parts, uint32_t **out_i, uint32_t **out_j,
                    uint8_t **out_v, orc_stats *st, uint8_t *flags_out) {
  memset(st, 0, sizeof(*st));
  *out_i = NULL; *out_j = NULL; *out_v = NULL;
  if (t == 0 || t > 255 || min_votes == 0 || n >= (1ull << 31) || n_parts == 0) return 1;

  /* The t hash tables. */
  orc_kv **tab = (orc_kv **)calloc(t, sizeof(orc_kv *));
  uint8_t *flag = (uint8_t *)calloc(n ? n : 1, 1);
  int oom = !tab || !flag;
  for (uint32_t u = 0; u < t && !oom; ++u) oom = !(tab[u] = (orc_kv *)malloc((n ? n : 1) * sizeof(orc_kv)));
  if (oom) {
    if (tab) for (uint32_t u = 0; u < t; ++u) free(tab[u]);
    free(tab); free(flag);
    return 2;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int u = 0; u < (int)t; ++u) orc_table_sort(n, keys + (uint64_t)u * n, tab[u]);

  /* Bucket sizes, raw candidate count and the occurrence filter (sizes
   * before any exclusion, flags from every table before any pair). */
  for (uint32_t u = 0; u < t; ++u) orc_table_buckets(n, tab[u], occ_num, occ_den, flag, &st->e_raw, &st->max_bucket);
  for (uint64_t i = 0; i < n; ++i) st->n_flagged += flag[i];

  /* Pairs and votes, one vote partition at a time. */
  orc_out out = {0};
  for (uint32_t p = 0; p < n_parts && !oom; ++p) {
    const uint64_t lo = n * p / n_parts, hi = n * (p + 1) / n_parts;
    orc_pairs pairs = {0};
    for (uint32_t u = 0; u < t; ++u) orc_table_pairs(n, tab[u], flag, min_lag, lo, hi, &pairs);
    oom = pairs.oom;
    if (!oom) orc_votes(pairs.p, pairs.cnt, NULL, min_votes, &out, st);
    oom |= out.oom;
    free(pairs.p);
  }
  for (uint32_t u = 0; u < t; ++u) free(tab[u]);
  free(tab);
  if (flags_out) memcpy(flags_out, flag, n);
  free(flag);
  if (oom) {
    free(out.i); free(out.j); free(out.v);
    return 2;
  }
  st->n_out = out.cnt;
  *out_i = out.i; *out_j = out.j; *out_v = out.v;
  return 0;
}

/* One table of a search whose tables are taken one at a time (for inputs
 * whose keys do not fit in memory at once): sorts the table's keys
 * keys_u[n], adds its buckets to *e_raw / *max_bucket and ORs its
 * occurrence-filter exclusions into flag[n] (orc_table_buckets), and appends
 * its candidate pairs with i in any of the n_ranges ranges
 * [ranges[2k], ranges[2k+1]) to *pairs / *cnt (a malloc'ed array the caller
 * passes back on the next call and frees with orc_free), without exclusion:
 * the exclusions are final only after every table, and orc_count_votes drops
 * the pairs they hit.  Returns 0, or 2 when memory runs out. */
int orc_table_scan(uint64_t n, const uint64_t *keys_u, uint32_t occ_num, uint32_t occ_den, uint8_t *flag,
                   uint64_t *e_raw, uint64_t *max_bucket, uint32_t min_lag, uint32_t n_ranges,
                   const uint64_t *ranges, uint64_t **pairs, uint64_t *cnt) {
  orc_kv *tab = (orc_kv *)malloc((n ? n : 1) * sizeof(orc_kv));
  if (!tab) return 2;
  orc_table_sort(n, keys_u, tab);
  orc_table_buckets(n, tab, occ_num, occ_den, flag, e_raw, max_bucket);
  orc_pairs v = {*pairs, *cnt, *cnt, 0};
  for (uint32_t k = 0; k < n_ranges; ++k) orc_table_pairs(n, tab, NULL, min_lag, ranges[2 * k], ranges[2 * k + 1], &v);
  free(tab);
  *pairs = v.p;
  *cnt = v.cnt;
  return v.oom ? 2 : 0;
}

/* Votes of the pairs collected by orc_table_scan over every table: drops the
 * pairs with an excluded member (flag[n], may be NULL), counts the rest
 * (orc_votes) and returns the output triplets as orc_search_keys does, with
 * st->e_voted and st->n_distinct of these pairs.  Sorts pairs[] in place. */
int orc_count_votes(uint64_t *pairs, uint64_t cnt, const uint8_t *flag, uint32_t min_votes, uint32_t **out_i,
                    uint32_t **out_j, uint8_t **out_v, orc_stats *st) {
  memset(st, 0, sizeof(*st));
  orc_out out = {0};
  orc_votes(pairs, cnt, flag, min_votes, &out, st);
  if (out.oom) {
    free(out.i); free(out.j); free(out.v);
    return 2;
  }
  st->n_out = out.cnt;
  *out_i = out.i; *out_j = out.j; *out_v = out.v;
  return 0;
}

/* Full search: signatures for all t tables, then orc_search_keys. */
int orc_search(uint32_t dim, uint32_t t, uint32_t r, uint32_t scheme, const uint32_t *a, const uint32_t *b,
               uint64_t n, const uint64_t *offsets, uint32_t nnz, const uint16_t *ind, uint32_t min_lag,
               uint32_t min_votes, uint32_t occ_num, uint32_t occ_den, uint32_t **out_i, uint32_t **out_j,
               uint8_t **out_v, orc_stats *st) {
  uint64_t *keys = (uint64_t *)malloc((n ? n : 1) * (uint64_t)t * sizeof(uint64_t));
  if (!keys) return 2;
  int rc = orc_signatures(dim, t, r, scheme, a, b, n, offsets, nnz, ind, keys, NULL);
  if (rc == 0)
    rc = orc_search_keys(t, n, keys, min_lag, min_votes, occ_num, occ_den, 1, out_i, out_j, out_v, st, NULL);
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

/* Sets the number of threads later OpenMP loops of the oracle use (timing
 * only; results do not depend on it). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
