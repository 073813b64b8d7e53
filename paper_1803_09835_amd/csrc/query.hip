// Query-only hashing (section 6.4, "Partition"): only the queries are hashed
// into the t tables; every dataset item is looked up in each table, and a
// (query, item) pair gets one vote per table in which the item falls in the
// query's bucket.  The result is what a search over tables holding the whole
// dataset would report for the queries, without building the dataset's
// tables.
//
// GPU form: the queries' band keys are sorted per table by LSD radix passes
// (all tables in one launch per digit).  The dataset's keys are computed a
// group of tables at a time (bounded memory) by the signature kernel, and a
// probe kernel takes one table per workgroup and a block of items: the
// table's sorted query keys are staged in LDS (when they fit), every item's
// key is bisected there, and each match (query, item) is appended with one
// atomic per wavefront.  The matches are then sorted by (query, item) and
// counted run by run; runs of at least min_votes are the output.
#include <string.h>

#include <algorithm>

#include "host.hpp"

using namespace fl;

namespace {

constexpr int kQT = 256;
constexpr uint32_t kLdsKeys = 8192;  // query keys per table staged in LDS (64 KB)

struct QueryCtrl {
  int err;
  unsigned int pad;
  unsigned long long matches;  // appended (may exceed the record capacity)
  unsigned long long out;      // pairs kept
};

// Keys of queries [0, nq) in table-major order, ids 0..nq-1 per table.
__global__ __launch_bounds__(kQT) void k_query_ids(uint32_t* ids, uint64_t nq, uint32_t t) {
  const uint64_t total = nq * t;
  for (uint64_t e = (uint64_t)blockIdx.x * kQT + threadIdx.x; e < total; e += (uint64_t)gridDim.x * kQT)
    ids[e] = (uint32_t)(e % nq);
}

// First position in keys[0, n) whose key is >= k.
__device__ __forceinline__ uint32_t lower_bound_u64(const uint64_t* keys, uint32_t n, uint64_t k) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (keys[mid] < k) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Workgroup (blockIdx.y = table u of the group, blockIdx.x = block of
// items): every item's key in table u is bisected among the table's sorted
// query keys; its matches (q << 32 | x) go to rec[] at offsets reserved
// once per wavefront.  matches counts every match, also those beyond cap.
__global__ __launch_bounds__(kQT) void k_query_probe(const uint64_t* qk, const uint32_t* qid, uint32_t nq,
                                                     const uint64_t* dk, uint64_t nd, uint64_t* rec, uint64_t cap,
                                                     unsigned long long* matches) {
  __shared__ uint64_t sk[kLdsKeys];
  const uint32_t u = blockIdx.y;
  const uint64_t* K = qk + (uint64_t)u * nq;
  const uint32_t* I = qid + (uint64_t)u * nq;
  const uint64_t* D = dk + (uint64_t)u * nd;
  const bool lds = nq <= kLdsKeys;
  if (lds) {
    for (uint32_t q = threadIdx.x; q < nq; q += kQT) sk[q] = K[q];
    __syncthreads();
  }
  const uint64_t* S = lds ? sk : K;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * kQT;
  const uint64_t rounds = (nd + stride - 1) / stride;
  for (uint64_t rd = 0; rd < rounds; ++rd) {
    const uint64_t x = rd * stride + (uint64_t)blockIdx.x * kQT + threadIdx.x;
    uint32_t lo = 0, cnt = 0;
    if (x < nd) {
      const uint64_t k = D[x];
      lo = lower_bound_u64(S, nq, k);
      uint32_t e = lo;
      while (e < nq && S[e] == k) ++e;
      cnt = e - lo;
    }
    // one reservation per wavefront
    uint32_t incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, 64);
      if (lane >= (uint32_t)o) incl += y;
    }
    const uint32_t tot = __shfl(incl, 63, 64);
    if (tot == 0) continue;
    unsigned long long base = 0;
    if (lane == 63) base = atomicAdd(matches, (unsigned long long)tot);
    base = __shfl(base, 63, 64);
    const uint64_t at = base + incl - cnt;
    for (uint32_t m = 0; m < cnt; ++m)
      if (at + m < cap) rec[at + m] = ((uint64_t)I[lo + m] << 32) | x;
  }
}

// keep[e] = 1 at the first record of each run of equal records whose length
// reaches min_votes (the length, at most 255, in len[e]).
__global__ __launch_bounds__(kQT) void k_query_runs(const uint64_t* rec, uint64_t m, uint32_t min_votes,
                                                    uint64_t* keep, uint32_t* len) {
  for (uint64_t e = (uint64_t)blockIdx.x * kQT + threadIdx.x; e < m; e += (uint64_t)gridDim.x * kQT) {
    const uint64_t k = rec[e];
    uint64_t flag = 0;
    if (e == 0 || rec[e - 1] != k) {
      uint64_t q = e + 1;
      while (q < m && rec[q] == k) ++q;
      len[e] = (uint32_t)(q - e);
      flag = q - e >= min_votes;
    }
    keep[e] = flag;
  }
}

__global__ __launch_bounds__(kQT) void k_query_emit(const uint64_t* rec, const uint32_t* len, const uint64_t* pos,
                                                    uint64_t m, uint64_t total, uint32_t* oq, uint32_t* ox,
                                                    uint8_t* ov) {
  for (uint64_t e = (uint64_t)blockIdx.x * kQT + threadIdx.x; e < m; e += (uint64_t)gridDim.x * kQT) {
    const uint64_t p = pos[e];
    const uint64_t nxt = e + 1 < m ? pos[e + 1] : total;
    if (nxt == p) continue;
    const uint64_t k = rec[e];
    oq[p] = (uint32_t)(k >> 32);
    ox[p] = (uint32_t)k;
    ov[p] = (uint8_t)len[e];
  }
}

unsigned grid_q(uint64_t n) {
  const uint64_t b = (n + kQT - 1) / kQT;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 8u * device_cus()));
}

}  // namespace

extern "C" int fast_lsh_query(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* queries,
                              const fast_lsh_fps* dataset, uint32_t min_votes, uint32_t* oq, uint32_t* ox,
                              uint8_t* ov, uint64_t capacity, fast_lsh_stats* stats) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  RC(fl_check_hash(h));
  RC(fl_check_fps(queries));
  RC(fl_check_fps(dataset));
  if (min_votes < 1) return fl_fail(FAST_LSH_E_INVALID, "min_votes must be >= 1");
  if (queries->n >= (1ull << 32) || dataset->n >= (1ull << 32))
    return fl_fail(FAST_LSH_E_INVALID, "queries and dataset must each hold fewer than 2^32 fingerprints");
  fast_lsh_stats local;
  memset(&local, 0, sizeof local);
  HIPCK(hipSetDevice(c->device));
  const uint64_t nq = queries->n, nd = dataset->n;
  const uint32_t t = h->num_tables;
  if (nq == 0 || nd == 0) {
    if (stats) *stats = local;
    return FAST_LSH_OK;
  }
  hipStream_t s = c->stream;
  uint32_t* dh;
  RC(fl_upload_hash(c, h, &dh));
  QueryCtrl* ctl;
  RC(ws<QueryCtrl>(c, "q_ctrl", 1, &ctl));
  fill_u8(reinterpret_cast<uint8_t*>(ctl), sizeof(QueryCtrl), 0, s);

  // 1. the queries' tables: band keys, sorted per table with their ids
  uint64_t *qk0, *qk1;
  uint32_t *qi0, *qi1, *qhist, *qsums;
  RC(ws<uint64_t>(c, "q_k0", nq * t, &qk0));
  RC(ws<uint64_t>(c, "q_k1", nq * t, &qk1));
  RC(ws<uint32_t>(c, "q_i0", nq * t, &qi0));
  RC(ws<uint32_t>(c, "q_i1", nq * t, &qi1));
  const uint32_t qnt = radix_tiles(nq, 0);
  RC(ws<uint32_t>(c, "q_hist", (uint64_t)256 * qnt * t, &qhist));
  RC(ws<uint32_t>(c, "q_sums", scan_sums_elems((uint64_t)256 * qnt, t), &qsums));
  {
    int cap;
    bool vec;
    RC(fl_row_capacity(c, queries, &cap, &vec));
    SigArgs a = fl_sig_args(h, queries, dh, &ctl->err);
    a.table_begin = 0;
    a.table_count = t;
    a.vec_load = vec;
    a.keys = qk0;
    prof_begin(c, FAST_LSH_STAGE_SIGNATURES);
    launch_sig(cap, h->scheme == FAST_LSH_MINMAX, a, s);
    prof_end(c);
    LAUNCHCK();
  }
  const uint32_t kb = fl_key_bits(h->dim) * h->band_rows;
  const uint32_t key_bits = kb > 64 ? 64 : kb;  // chained keys use all 64 bits
  prof_begin(c, FAST_LSH_STAGE_GROUP);
  hipLaunchKernelGGL(k_query_ids, dim3(grid_q(nq * t)), dim3(kQT), 0, s, qi0, nq, t);
  for (uint32_t sh = 0; sh < key_bits; sh += 8) {
    radix_pass(qk0, qi0, qk1, qi1, nq, t, sh, qhist, qsums, 0, s);
    std::swap(qk0, qk1);
    std::swap(qi0, qi1);
  }
  prof_end(c);
  LAUNCHCK();

  // 2. the dataset a group of tables at a time: keys, then probes
  const uint64_t group_bytes = 8ull << 30;  // dataset keys held at once
  const uint32_t g = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(t, group_bytes / (8 * nd)));
  uint64_t* dk;
  RC(ws<uint64_t>(c, "q_dk", (uint64_t)g * nd, &dk));
  int dcap;
  bool dvec;
  RC(fl_row_capacity(c, dataset, &dcap, &dvec));
  uint64_t rec_cap = std::max<uint64_t>(1u << 20, 4 * (nq + nd));
  uint64_t* rec = nullptr;
  QueryCtrl hc;
  for (int attempt = 0; attempt < 2; ++attempt) {
    RC(ws<uint64_t>(c, "q_rec", rec_cap, &rec));
    fill_u64(reinterpret_cast<uint64_t*>(&ctl->matches), 1, 0, s);
    for (uint32_t tb = 0; tb < t; tb += g) {
      const uint32_t tc = std::min(g, t - tb);
      SigArgs a = fl_sig_args(h, dataset, dh, &ctl->err);
      a.table_begin = tb;
      a.table_count = tc;
      a.vec_load = dvec;
      a.keys = dk;
      prof_begin(c, FAST_LSH_STAGE_SIGNATURES);
      launch_sig(dcap, h->scheme == FAST_LSH_MINMAX, a, s);
      prof_end(c);
      LAUNCHCK();
      const uint32_t blocks = (uint32_t)std::min<uint64_t>((nd + kQT - 1) / kQT,
                                                           std::max<uint64_t>(1, 8ull * device_cus() / tc));
      prof_begin(c, FAST_LSH_STAGE_PAIRS);
      hipLaunchKernelGGL(k_query_probe, dim3(blocks, tc), dim3(kQT), 0, s, qk0 + (uint64_t)tb * nq,
                         qi0 + (uint64_t)tb * nq, (uint32_t)nq, dk, nd, rec, rec_cap, &ctl->matches);
      prof_end(c);
      LAUNCHCK();
    }
    RC(d2h(c, &hc, ctl));
    if (hc.err) return fl_fail(FAST_LSH_E_INVALID, "a fingerprint is empty or holds an index >= dim (%u)", h->dim);
    if (hc.matches <= rec_cap) break;
    rec_cap = hc.matches + 1024;  // every match counted: one more pass with room for all
  }
  const uint64_t m = hc.matches;

  // 3. votes: sort the matches by (query, item), count each run
  uint64_t n_out = 0;
  if (m) {
    uint64_t *r1, *keep, *ksum;
    uint32_t *v0, *v1, *len, *hist, *sums;
    RC(ws<uint64_t>(c, "q_rec1", m, &r1));
    RC(ws<uint32_t>(c, "q_v0", m, &v0));
    RC(ws<uint32_t>(c, "q_v1", m, &v1));
    const uint32_t nt = radix_tiles(m, 0);
    RC(ws<uint32_t>(c, "q_rhist", (uint64_t)256 * nt, &hist));
    RC(ws<uint32_t>(c, "q_rsums", scan_sums_elems((uint64_t)256 * nt, 1), &sums));
    const uint32_t xb = fl_key_bits((uint32_t)std::max<uint64_t>(nd, 2));
    const uint32_t qb = fl_key_bits((uint32_t)std::max<uint64_t>(nq, 2));
    uint64_t* r0 = rec;
    prof_begin(c, FAST_LSH_STAGE_OUTPUT);
    bool first = true;
    for (uint32_t base : {0u, 32u})
      for (uint32_t sh = 0; sh < (base ? qb : xb); sh += 8) {
        radix_pass(r0, first ? nullptr : v0, r1, v1, m, 1, base + sh, hist, sums, 0, s);
        first = false;
        std::swap(r0, r1);
        std::swap(v0, v1);
      }
    RC(ws<uint64_t>(c, "q_keep", m, &keep));
    RC(ws<uint32_t>(c, "q_len", m, &len));
    RC(ws<uint64_t>(c, "q_ksum", scan_sums_elems(m, 1) + 1, &ksum));
    hipLaunchKernelGGL(k_query_runs, dim3(grid_q(m)), dim3(kQT), 0, s, r0, m, min_votes, keep, len);
    scan_u64(keep, m, 1, ksum, reinterpret_cast<uint64_t*>(&ctl->out), s);
    prof_end(c);
    LAUNCHCK();
    RC(d2h(c, &hc, ctl));
    n_out = hc.out;
    if (n_out <= capacity && n_out) {
      if (!oq || !ox || !ov) return fl_fail(FAST_LSH_E_INVALID, "output pointer is NULL");
      prof_begin(c, FAST_LSH_STAGE_OUTPUT);
      hipLaunchKernelGGL(k_query_emit, dim3(grid_q(m)), dim3(kQT), 0, s, r0, len, keep, m, n_out, oq, ox, ov);
      prof_end(c);
      LAUNCHCK();
    }
  }
  HIPCK(hipStreamSynchronize(s));
  prof_collect(c);
  local.n_out = n_out;
  local.e_raw = m;
  local.e_voted = m;
  local.n_distinct = ~0ull;
  if (stats) *stats = local;
  if (n_out > capacity)
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)n_out,
                   (unsigned long long)capacity);
  return FAST_LSH_OK;
}
