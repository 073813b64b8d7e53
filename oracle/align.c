/*
 * CPU ORACLE — TEST INFRASTRUCTURE ONLY (spatiotemporal alignment).
 *
 * Plain, slow implementations of the first two reductions that section 7 of
 * Rong et al. (VLDB 2018) applies to the similarity-search output, written
 * from the paper's description in its own order of steps:
 *
 *   - channel level (section 7.1 "Channel Level", section 7.2 "Channel"):
 *     the triplet lists (dt, idx1, sim) of the channels of one station are
 *     each sorted by (dt, idx1), merged, and consecutive rows with the same
 *     (dt, idx1) are reduced by summing sim; rows whose sum is below the
 *     threshold are dropped;
 *   - station level (section 7.1 "Station Level", section 7.2 "Station"):
 *     on the combined, (dt, idx1)-ordered entries, a linear pass finds along
 *     each diagonal dt the sequences whose consecutive idx1 differ by at most
 *     the gap; sequences on adjacent diagonals dt and dt + 1 whose idx1 spans
 *     come within the gap of each other are merged (transitively) into one
 *     cluster; every cluster is summarised (bounding box, entry count, summed
 *     similarity, its strongest entry) and small or wide clusters are pruned.
 *
 * Readings where the paper is silent: a triplet comes from a search output
 * pair (i, j, votes) with i < j as dt = j - i, idx1 = i, sim = votes; the
 * combined threshold keeps sums >= min_sim; "gap" is the difference of
 * consecutive idx1 values (a run continues while it is <= max_gap); a
 * cluster's width is dt_max - dt_min + 1 and "relatively narrow" means
 * width <= max_width; a cluster is kept when it also holds at least
 * min_entries entries and a summed similarity of at least min_sum; the
 * strongest entry is the largest sim, ties going to the smallest (dt, idx1);
 * clusters are listed in the order of their first entry in (dt, idx1) order.
 *
 * Only the tests and the benchmark's CPU-baseline leg call these functions.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint32_t dt, idx1, sim; } orc_trip;

static int cmp_trip(const void *x, const void *y) {
  const orc_trip *p = (const orc_trip *)x, *q = (const orc_trip *)y;
  if (p->dt != q->dt) return p->dt < q->dt ? -1 : 1;
  if (p->idx1 != q->idx1) return p->idx1 < q->idx1 ? -1 : 1;
  return 0;
}

/* (dt, idx1) of a before b: negative, equal: 0, after: positive. */
static int order_trip(const orc_trip *a, const orc_trip *b) { return cmp_trip(a, b); }

/* Channel-level sort-merge-reduce (section 7.2 "Channel").  Channel c holds
 * counts[c] search-output pairs (i[c][k], j[c][k], votes[c][k]) with
 * i < j.  On success the combined entries with summed sim >= min_sim,
 * ordered by (dt, idx1), are returned in three malloc'ed arrays (freed with
 * orc_free).  Returns 0, 1 for a pair with j <= i, 2 when memory runs out. */
int orc_channel_merge(uint32_t n_ch, const uint64_t *counts, const uint32_t *const *pi, const uint32_t *const *pj,
                      const uint8_t *const *pv, uint32_t min_sim, uint32_t **out_dt, uint32_t **out_idx1,
                      uint32_t **out_sim, uint64_t *n_out) {
  *out_dt = NULL; *out_idx1 = NULL; *out_sim = NULL; *n_out = 0;
  uint64_t total = 0;
  for (uint32_t c = 0; c < n_ch; ++c) total += counts[c];
  orc_trip **lists = (orc_trip **)calloc(n_ch ? n_ch : 1, sizeof(orc_trip *));
  uint64_t *head = (uint64_t *)calloc(n_ch ? n_ch : 1, sizeof(uint64_t));
  uint32_t *odt = (uint32_t *)malloc((total ? total : 1) * 4);
  uint32_t *oid = (uint32_t *)malloc((total ? total : 1) * 4);
  uint32_t *osm = (uint32_t *)malloc((total ? total : 1) * 4);
  int rc = (!lists || !head || !odt || !oid || !osm) ? 2 : 0;

  /* 1. sort phase: every channel's triplets by (dt, idx1) */
  for (uint32_t c = 0; c < n_ch && rc == 0; ++c) {
    lists[c] = (orc_trip *)malloc((counts[c] ? counts[c] : 1) * sizeof(orc_trip));
    if (!lists[c]) { rc = 2; break; }
    for (uint64_t k = 0; k < counts[c]; ++k) {
      if (pj[c][k] <= pi[c][k]) { rc = 1; break; }
      lists[c][k].dt = pj[c][k] - pi[c][k];
      lists[c][k].idx1 = pi[c][k];
      lists[c][k].sim = pv[c][k];
    }
    if (rc == 0) qsort(lists[c], counts[c], sizeof(orc_trip), cmp_trip);
  }

  /* 2. merge phase: repeatedly take the smallest head among the channels
   *    (the lowest channel on a tie), so equal (dt, idx1) rows end up next
   *    to each other; 3. reduce phase on the fly: a row equal to the
   *    previous one adds its sim, a new row closes the previous one. */
  uint64_t m = 0;
  int open = 0;
  orc_trip cur = {0, 0, 0};
  while (rc == 0) {
    int best = -1;
    for (uint32_t c = 0; c < n_ch; ++c) {
      if (head[c] == counts[c]) continue;
      if (best < 0 || order_trip(&lists[c][head[c]], &lists[best][head[best]]) < 0) best = (int)c;
    }
    if (best < 0) break;
    const orc_trip t = lists[best][head[best]++];
    if (open && t.dt == cur.dt && t.idx1 == cur.idx1) {
      cur.sim += t.sim;
      continue;
    }
    if (open && cur.sim >= min_sim) { odt[m] = cur.dt; oid[m] = cur.idx1; osm[m] = cur.sim; ++m; }
    cur = t;
    open = 1;
  }
  if (rc == 0 && open && cur.sim >= min_sim) { odt[m] = cur.dt; oid[m] = cur.idx1; osm[m] = cur.sim; ++m; }

  if (lists)
    for (uint32_t c = 0; c < n_ch; ++c) free(lists[c]);
  free(lists);
  free(head);
  if (rc != 0) {
    free(odt); free(oid); free(osm);
    return rc;
  }
  *out_dt = odt; *out_idx1 = oid; *out_sim = osm; *n_out = m;
  return 0;
}

typedef struct {
  uint32_t dt_min, dt_max, idx1_min, idx1_max;
  uint32_t n_entries, peak_sim, peak_dt, peak_idx1;
  uint64_t sim_sum;
} orc_cluster;

typedef struct { uint64_t first, last; uint32_t dt, lo, hi; } orc_run;

static uint64_t uf_find(uint64_t *parent, uint64_t x) {
  while (parent[x] != x) x = parent[x];
  return x;
}

static void uf_union(uint64_t *parent, uint64_t a, uint64_t b) {
  a = uf_find(parent, a);
  b = uf_find(parent, b);
  if (a == b) return;
  if (a < b) parent[b] = a; else parent[a] = b;  /* the smaller index is the root */
}

/* Station-level clustering (section 7.2 "Station").  The n entries
 * (dt[k], idx1[k], sim[k]) must be ordered by (dt, idx1) without repeats (the
 * channel merge's output).  On success the kept clusters, in the order of
 * their first entry, are returned in a malloc'ed array (freed with orc_free).
 * Returns 0, 1 for entries out of order, 2 when memory runs out. */
int orc_station_clusters(uint64_t n, const uint32_t *dt, const uint32_t *idx1, const uint32_t *sim, uint32_t max_gap,
                         uint32_t max_width, uint32_t min_entries, uint64_t min_sum, orc_cluster **out,
                         uint64_t *n_out) {
  *out = NULL;
  *n_out = 0;
  for (uint64_t k = 1; k < n; ++k)
    if (dt[k] < dt[k - 1] || (dt[k] == dt[k - 1] && idx1[k] <= idx1[k - 1])) return 1;

  /* 1. linear pass: runs along each diagonal */
  orc_run *run = (orc_run *)malloc((n ? n : 1) * sizeof(orc_run));
  if (!run) return 2;
  uint64_t nr = 0;
  for (uint64_t k = 0; k < n; ++k) {
    if (nr > 0 && run[nr - 1].dt == dt[k] && idx1[k] - run[nr - 1].hi <= max_gap) {
      run[nr - 1].last = k;
      run[nr - 1].hi = idx1[k];
    } else {
      run[nr].first = run[nr].last = k;
      run[nr].dt = dt[k];
      run[nr].lo = run[nr].hi = idx1[k];
      ++nr;
    }
  }

  /* 2. merge runs of adjacent diagonals whose spans come within the gap:
   *    run a against every run b of diagonal dt(a) + 1, those runs taken in
   *    order of their start until a start lies beyond hi(a) + gap */
  uint64_t *parent = (uint64_t *)malloc((nr ? nr : 1) * sizeof(uint64_t));
  uint64_t *next = (uint64_t *)malloc((nr ? nr : 1) * sizeof(uint64_t)); /* first run of a later diagonal */
  if (!parent || !next) { free(run); free(parent); free(next); return 2; }
  for (uint64_t r = 0; r < nr; ++r) parent[r] = r;
  for (uint64_t r = nr, ns = nr; r-- > 0;) {
    if (r + 1 < nr && run[r + 1].dt != run[r].dt) ns = r + 1;
    next[r] = ns;
  }
  for (uint64_t a = 0; a < nr; ++a)
    for (uint64_t b = next[a]; b < nr && run[b].dt == (uint64_t)run[a].dt + 1; ++b) {
      const uint64_t alo = run[a].lo, ahi = run[a].hi, blo = run[b].lo, bhi = run[b].hi;
      if (blo > ahi + max_gap) break;
      if (alo <= bhi + max_gap) uf_union(parent, a, b);
    }
  free(next);

  /* 3. one summary per cluster, kept at its root (its first run) */
  orc_cluster *sum = (orc_cluster *)calloc(nr ? nr : 1, sizeof(orc_cluster));
  if (!sum) { free(run); free(parent); return 2; }
  for (uint64_t r = 0; r < nr; ++r) {
    orc_cluster *s = &sum[uf_find(parent, r)];
    for (uint64_t k = run[r].first; k <= run[r].last; ++k) {
      if (s->n_entries == 0) {
        s->dt_min = s->dt_max = dt[k];
        s->idx1_min = s->idx1_max = idx1[k];
      }
      if (dt[k] < s->dt_min) s->dt_min = dt[k];
      if (dt[k] > s->dt_max) s->dt_max = dt[k];
      if (idx1[k] < s->idx1_min) s->idx1_min = idx1[k];
      if (idx1[k] > s->idx1_max) s->idx1_max = idx1[k];
      /* strongest entry: larger sim, or equal sim and earlier (dt, idx1) */
      if (s->n_entries == 0 || sim[k] > s->peak_sim ||
          (sim[k] == s->peak_sim && (dt[k] < s->peak_dt || (dt[k] == s->peak_dt && idx1[k] < s->peak_idx1)))) {
        s->peak_sim = sim[k];
        s->peak_dt = dt[k];
        s->peak_idx1 = idx1[k];
      }
      s->n_entries += 1;
      s->sim_sum += sim[k];
    }
  }

  /* 4. prune small and wide clusters; roots in run order are the clusters
   *    in the order of their first entry */
  orc_cluster *o = (orc_cluster *)malloc((nr ? nr : 1) * sizeof(orc_cluster));
  if (!o) { free(run); free(parent); free(sum); return 2; }
  uint64_t m = 0;
  for (uint64_t r = 0; r < nr; ++r) {
    if (parent[r] != r) continue;
    const orc_cluster *s = &sum[r];
    if (s->dt_max - s->dt_min + 1 > max_width || s->n_entries < min_entries || s->sim_sum < min_sum) continue;
    o[m++] = *s;
  }
  free(run);
  free(parent);
  free(sum);
  *out = o;
  *n_out = m;
  return 0;
}
