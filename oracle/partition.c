/*
 * CPU ORACLE — TEST INFRASTRUCTURE ONLY (section 6.4 and 6.5 forms).
 *
 * Plain, slow implementations, from band keys, of two forms of the search
 * that Rong et al. (VLDB 2018) describe besides the plain one:
 *
 *   - query-only hashing (section 6.4, "Partition"): only the query items
 *     are hashed into the t tables; every dataset item is then looked up in
 *     each table, and a query and an item share a vote for every table in
 *     which the item falls in the query's bucket.  The result is every
 *     (query, item) pair with at least min_votes votes, which is what a
 *     search over tables holding the whole dataset would report for the
 *     queries;
 *   - the partitioned search with the dynamic occurrence filter (section
 *     6.4 "Partition", section 6.5 "Removing correlated noise"): the
 *     fingerprints are split into n_parts consecutive partitions taken one
 *     after another; while partition p is searched, a fingerprint of p whose
 *     near-neighbour candidates outnumber occ_num/occ_den of the partition's
 *     fingerprints is excluded together with those candidates from the rest
 *     of the search; partition p reports the pairs whose smaller id lies in
 *     it.
 *
 * Readings where the paper is silent: a fingerprint's near-neighbour
 * candidates are the distinct other fingerprints that share a bucket with
 * it in at least one table, lie at least min_lag away (self-matches of
 * adjacent windows are no candidates, section 7.1) and are not excluded
 * yet; the candidate counts of a partition are all taken before any of its
 * exclusions (so the result does not depend on the order within a
 * partition); "its neighbours" are those candidates; exclusions only affect
 * later output (pairs already reported stay); the threshold compares
 * count * occ_den > partition size * occ_num in exact integers; occ_den = 0
 * turns the filter off, and then every partition count gives the plain
 * search's output.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t key; uint64_t id; } orc_kv2;

static int cmp_kv2(const void *x, const void *y) {
  const orc_kv2 *p = (const orc_kv2 *)x, *q = (const orc_kv2 *)y;
  if (p->key != q->key) return p->key < q->key ? -1 : 1;
  if (p->id != q->id) return p->id < q->id ? -1 : 1;
  return 0;
}

static int cmp_u64b(const void *x, const void *y) {
  uint64_t p = *(const uint64_t *)x, q = *(const uint64_t *)y;
  return p < q ? -1 : (p > q ? 1 : 0);
}

/* First position in tab[0, n) whose key is >= key (tab sorted by key). */
static uint64_t lower_key(const orc_kv2 *tab, uint64_t n, uint64_t key) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    if (tab[mid].key < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

typedef struct { uint64_t *p; uint64_t cnt, cap; int oom; } orc_vec;

static void vec_push(orc_vec *v, uint64_t x) {
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

typedef struct { uint32_t *a, *b; uint8_t *v; uint64_t cnt, cap; int oom; } orc_trip_out;

static void trip_push(orc_trip_out *o, uint32_t a, uint32_t b, uint8_t v) {
  if (o->oom) return;
  if (o->cnt == o->cap) {
    uint64_t nc = o->cap ? 2 * o->cap : 16;
    uint32_t *na = (uint32_t *)realloc(o->a, nc * 4);
    if (na) o->a = na;
    uint32_t *nb = (uint32_t *)realloc(o->b, nc * 4);
    if (nb) o->b = nb;
    uint8_t *nv = (uint8_t *)realloc(o->v, nc);
    if (nv) o->v = nv;
    if (!na || !nb || !nv) { o->oom = 1; return; }
    o->cap = nc;
  }
  o->a[o->cnt] = a; o->b[o->cnt] = b; o->v[o->cnt] = v;
  ++o->cnt;
}

/* Query-only hashing (section 6.4).  qkeys[u * nq + q] and dkeys[u * nd + x]
 * are the band keys of the queries and of the dataset items (table-major).
 * On success the pairs (q, x) with at least min_votes votes, ordered by
 * (q, x), are returned in three malloc'ed arrays with their vote counts
 * (freed with orc_free); *n_cand is the number of (table, query, item)
 * matches.  Returns 0, 1 for invalid arguments, 2 when memory runs out. */
int orc_query_keys(uint32_t t, uint64_t nq, const uint64_t *qkeys, uint64_t nd, const uint64_t *dkeys,
                   uint32_t min_votes, uint32_t **out_q, uint32_t **out_x, uint8_t **out_v, uint64_t *n_out,
                   uint64_t *n_cand) {
  *out_q = NULL; *out_x = NULL; *out_v = NULL; *n_out = 0; *n_cand = 0;
  if (t == 0 || t > 255 || min_votes == 0 || nq >= (1ull << 32) || nd >= (1ull << 32)) return 1;
  /* 1. the t tables of the queries only */
  orc_kv2 *tab = (orc_kv2 *)malloc((nq ? nq : 1) * (uint64_t)t * sizeof(orc_kv2));
  if (!tab) return 2;
  for (uint32_t u = 0; u < t; ++u) {
    orc_kv2 *tu = tab + (uint64_t)u * nq;
    for (uint64_t q = 0; q < nq; ++q) { tu[q].key = qkeys[(uint64_t)u * nq + q]; tu[q].id = q; }
    qsort(tu, nq, sizeof(orc_kv2), cmp_kv2);
  }
  /* 2. every dataset item looked up in every table: one match per query of
   *    the item's bucket */
  orc_vec m = {0};
  for (uint64_t x = 0; x < nd && !m.oom; ++x)
    for (uint32_t u = 0; u < t; ++u) {
      const orc_kv2 *tu = tab + (uint64_t)u * nq;
      const uint64_t k = dkeys[(uint64_t)u * nd + x];
      for (uint64_t s = lower_key(tu, nq, k); s < nq && tu[s].key == k; ++s) vec_push(&m, (tu[s].id << 32) | x);
    }
  free(tab);
  if (m.oom) { free(m.p); return 2; }
  *n_cand = m.cnt;
  /* 3. votes: a (query, item) pair matched in k tables appears k times */
  qsort(m.p, m.cnt, sizeof(uint64_t), cmp_u64b);
  orc_trip_out o = {0};
  for (uint64_t s = 0; s < m.cnt;) {
    uint64_t e = s + 1;
    while (e < m.cnt && m.p[e] == m.p[s]) ++e;
    if (e - s >= min_votes) trip_push(&o, (uint32_t)(m.p[s] >> 32), (uint32_t)m.p[s], (uint8_t)(e - s));
    s = e;
  }
  free(m.p);
  if (o.oom) { free(o.a); free(o.b); free(o.v); return 2; }
  *out_q = o.a; *out_x = o.b; *out_v = o.v; *n_out = o.cnt;
  return 0;
}

typedef struct {
  uint64_t n_out, e_raw, e_voted, n_distinct, n_flagged, max_bucket;
} orc_pstats;

/* Partitioned search with the dynamic occurrence filter (sections 6.4,
 * 6.5), from table-major band keys keys[u * n + i].  On success the output
 * triplets (i, j, votes), ordered by (i, j), are returned in malloc'ed
 * arrays; excluded[n] (optional) receives the final exclusions.  Counters:
 * e_raw and max_bucket of all tables (bucket sizes do not depend on the
 * filter), e_voted and n_distinct over the pairs each partition could report
 * (smaller id in the partition, lag kept, both not excluded), n_flagged the
 * excluded fingerprints at the end.  Returns 0, 1 for invalid arguments, 2
 * when memory runs out. */
int orc_search_partitioned_keys(uint32_t t, uint64_t n, const uint64_t *keys, uint32_t min_lag, uint32_t min_votes,
                                uint32_t occ_num, uint32_t occ_den, uint32_t n_parts, uint32_t **out_i,
                                uint32_t **out_j, uint8_t **out_v, orc_pstats *st, uint8_t *excluded_out) {
  memset(st, 0, sizeof *st);
  *out_i = NULL; *out_j = NULL; *out_v = NULL;
  if (t == 0 || t > 255 || min_votes == 0 || n >= (1ull << 31) || n_parts == 0) return 1;
  /* the t hash tables (section 6.1) and where each fingerprint sits in them */
  orc_kv2 *tab = (orc_kv2 *)malloc((n ? n : 1) * (uint64_t)t * sizeof(orc_kv2));
  uint64_t *at = (uint64_t *)malloc((n ? n : 1) * (uint64_t)t * sizeof(uint64_t)); /* position of i in table u */
  uint8_t *ex = (uint8_t *)calloc(n ? n : 1, 1);
  uint64_t *cand_cnt = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
  if (!tab || !at || !ex || !cand_cnt) { free(tab); free(at); free(ex); free(cand_cnt); return 2; }
  for (uint32_t u = 0; u < t; ++u) {
    orc_kv2 *tu = tab + (uint64_t)u * n;
    for (uint64_t i = 0; i < n; ++i) { tu[i].key = keys[(uint64_t)u * n + i]; tu[i].id = i; }
    qsort(tu, n, sizeof(orc_kv2), cmp_kv2);
    for (uint64_t s = 0; s < n; ++s) at[(uint64_t)u * n + tu[s].id] = s;
    for (uint64_t s = 0; s < n;) {
      uint64_t e = s + 1;
      while (e < n && tu[e].key == tu[s].key) ++e;
      st->e_raw += (e - s) * (e - s - 1) / 2;
      if (e - s > st->max_bucket) st->max_bucket = e - s;
      s = e;
    }
  }
  int oom = 0;
  orc_trip_out o = {0};
  orc_vec cand = {0};
  for (uint32_t p = 0; p < n_parts && !oom; ++p) {
    const uint64_t lo = n * p / n_parts, hi = n * (p + 1) / n_parts;
    /* candidates of every fingerprint of the partition, with the
     * exclusions as they stand at the partition's start */
    uint64_t *cstart = (uint64_t *)malloc((hi - lo + 1) * sizeof(uint64_t));
    if (!cstart) { oom = 1; break; }
    cand.cnt = 0;
    for (uint64_t i = lo; i < hi && !cand.oom; ++i) {
      cstart[i - lo] = cand.cnt;
      if (ex[i]) continue;
      const uint64_t first = cand.cnt;
      for (uint32_t u = 0; u < t; ++u) {
        const orc_kv2 *tu = tab + (uint64_t)u * n;
        const uint64_t pos = at[(uint64_t)u * n + i];
        uint64_t s = pos;
        while (s > 0 && tu[s - 1].key == tu[pos].key) --s;
        for (; s < n && tu[s].key == tu[pos].key; ++s) {
          const uint64_t j = tu[s].id;
          const uint64_t lag = j > i ? j - i : i - j;
          if (j != i && lag >= min_lag && !ex[j]) vec_push(&cand, j);
        }
      }
      if (cand.oom) break;
      qsort(cand.p + first, cand.cnt - first, sizeof(uint64_t), cmp_u64b);
      uint64_t m = first;
      for (uint64_t q = first; q < cand.cnt; ++q)
        if (q == first || cand.p[q] != cand.p[q - 1]) cand.p[m++] = cand.p[q];
      cand.cnt = m;
      cand_cnt[i] = m - first;
    }
    cstart[hi - lo] = cand.cnt;
    if (cand.oom) { free(cstart); oom = 1; break; }
    /* the partition's exclusions: its over-threshold fingerprints and their
     * candidates */
    if (occ_den) {
      for (uint64_t i = lo; i < hi; ++i) {
        if (ex[i] == 1) continue;
        if ((unsigned __int128)cand_cnt[i] * occ_den <= (unsigned __int128)(hi - lo) * occ_num) continue;
        ex[i] = 2; /* excluded in this partition; its candidates follow below */
      }
      for (uint64_t i = lo; i < hi; ++i) {
        if (ex[i] != 2) continue;
        for (uint64_t q = cstart[i - lo]; q < cstart[i - lo + 1]; ++q)
          if (!ex[cand.p[q]]) ex[cand.p[q]] = 3;
      }
      for (uint64_t i = 0; i < n; ++i) if (ex[i]) ex[i] = 1;
    }
    free(cstart);
    /* the partition's output: pairs (i, j), i in the partition, j > i */
    for (uint64_t i = lo; i < hi && !oom; ++i) {
      if (ex[i]) continue;
      cand.cnt = 0;
      for (uint32_t u = 0; u < t; ++u) {
        const orc_kv2 *tu = tab + (uint64_t)u * n;
        const uint64_t pos = at[(uint64_t)u * n + i];
        for (uint64_t s = pos + 1; s < n && tu[s].key == tu[pos].key; ++s) {
          const uint64_t j = tu[s].id;  /* ids ascend within a bucket: every later member is larger */
          if (j - i >= min_lag && !ex[j]) vec_push(&cand, j);
        }
      }
      if (cand.oom) { oom = 1; break; }
      qsort(cand.p, cand.cnt, sizeof(uint64_t), cmp_u64b);
      for (uint64_t s = 0; s < cand.cnt;) {
        uint64_t e = s + 1;
        while (e < cand.cnt && cand.p[e] == cand.p[s]) ++e;
        st->e_voted += e - s;
        st->n_distinct += 1;
        if (e - s >= min_votes) trip_push(&o, (uint32_t)i, (uint32_t)cand.p[s], (uint8_t)(e - s));
        s = e;
      }
    }
  }
  for (uint64_t i = 0; i < n; ++i) st->n_flagged += ex[i] != 0;
  if (excluded_out) memcpy(excluded_out, ex, n);
  free(tab); free(at); free(ex); free(cand_cnt); free(cand.p);
  if (oom || o.oom) { free(o.a); free(o.b); free(o.v); return 2; }
  st->n_out = o.cnt;
  *out_i = o.a; *out_j = o.b; *out_v = o.v;
  return 0;
}
