// Host orchestration of the similarity search over a set of stations
// (section 6.1 "Search"; occurrence filter, section 6.5; self-match lag,
// section 7.1), and its public entry points.
//
// One search runs every kernel once over all stations together: the
// stations' fingerprints get consecutive global ids, their mixed keys carry
// the station id in the top four bits (above a 60-bit bijective mix of the
// band key) so that no bucket ever holds two stations and each station's
// buckets are contiguous in every sorted table, and the occurrence filter
// and the counters are kept per station.  A single station is the case
// S = 1 (untagged, 64-bit mix).
//
// The part of the search whose launch shapes depend only on the input
// shapes (signatures, grouping, buckets, big bins, exclusion counts and the
// small-bucket pair kernel) is enqueued by enqueue_prefix, either directly
// or into a captured HIP graph.  The rest depends on counts the device
// produces (large buckets, output size) and is launched after one read-back.
#include <string.h>

#include <algorithm>
#include <vector>

#include "host.hpp"

using namespace fl;

namespace {

struct Plan {
  uint32_t t, G, TG, row_dw, row_pitch, need;
};

// Occurrence filter (section 6.5): the largest bucket of a station of ns
// fingerprints within the threshold, size * den <= ns * num, i.e.
// floor(ns * num / den); all ones when no filter is set.
uint64_t occ_bound(uint64_t ns, const fast_lsh_filter* flt) {
  if (!flt->occ_den) return ~0ull;
  return (uint64_t)(((unsigned __int128)ns * flt->occ_num) / flt->occ_den);
}

// Bits of the mixed key the radix passes bin on: a multiple of 8 large enough
// that an average bin of the largest station holds at most about 4
// elements, plus the four station bits when keys are tagged.
uint32_t bin_bits(uint64_t n_max, bool tagged) {
  uint32_t need = 0;
  while ((4ull << need) < n_max) ++need;
  if (tagged) need += 4;
  uint32_t B = (need + 7) / 8 * 8;
  return std::min<uint32_t>(32, std::max<uint32_t>(8, B));
}

// Table groups of the sub-key rows: one group when every shared table has to
// be seen anyway (v <= 2, or n_distinct wanted), else v - 1 groups so that a
// pair with v votes shares need = ceil(v / G) tables in some group.  `lines`:
// rows padded to the line-aligned pitch (fewer memory requests per random
// row read); otherwise packed (the bounded form, where memory is the limit).
Plan make_plan(uint32_t t, uint32_t v, bool distinct, bool lines) {
  Plan p;
  p.t = t;
  uint32_t G = (distinct || v <= 2) ? 1u : std::min(v - 1, t);
  p.TG = (t + G - 1) / G;
  p.G = (t + p.TG - 1) / p.TG;
  p.need = (v + p.G - 1) / p.G;
  p.row_dw = row_dwords(p.TG);
  p.row_pitch = lines ? row_pitch_lines(p.row_dw) : p.row_dw;
  return p;
}

// Counters the host reads back.  Sums that many workgroups update live in
// the spread buffer ([S][kSpread] slots each) and are folded per station
// into st_sum by k_spread_reduce.
struct Ctrl {
  unsigned long long n_flagged;  // all stations
  unsigned int big_count, bin_count, out_count;
  int err;
  unsigned long long st_flagged[FAST_LSH_MAX_STATIONS];
  unsigned long long st_sum[4 * FAST_LSH_MAX_STATIONS];  // e_raw, max_bucket, e_voted, n_distinct
  unsigned long long st_offs[FAST_LSH_MAX_STATIONS + 1];
  unsigned long long work[3];  // tiled buckets: voted pairs, members, in-bucket pairs
};

// Everything the fixed-shape prefix launches read.
struct Job {
  uint32_t S;
  uint64_t N;
  uint32_t t, B;
  bool minmax;
  Plan pl;
  TuneChoice tc;
  std::vector<uint64_t> base;  // S + 1
  std::vector<int> cap;
  std::vector<bool> vec;
  const fast_lsh_fps* f;
  const fast_lsh_hash* h;
  uint32_t* dhash;
  Ctrl* ctrl;
  unsigned long long *er, *ev, *nd;
  unsigned int* mb;
  uint64_t *mkeys, *ak, *bk;
  uint32_t *av, *bv, *rows, *hist, *sums;
  uint8_t *flags, *marks;
  uint64_t* sbase;
  uint4 *bdesc, *bins;
  uint32_t bigbin_grid;
  uint64_t spread_bytes;
  unsigned long long* work;  // [3][kSpread]: tiled buckets' voted pairs, members, in-bucket pairs
  uint32_t rswl;
  unsigned long long* redo_tally = nullptr;  // votes of second pair runs, discarded
  uint32_t parts = 0;  // > 0: partitioned search with the dynamic occurrence filter (no pair launch in the prefix)
  BucketArgs ba;
  PairArgs pa;
  // the radix passes leave the sorted keys/ids in (sorted_k, sorted_v)
  uint64_t *sorted_k, *scratch_k;
  uint32_t *sorted_v, *scratch_v;
};

// Time one launch sequence with events on stream s (used by the tuner);
// `setup` is enqueued before the timed interval.
template <typename P, typename F>
int time_launch(hipStream_t s, P&& setup, F&& f, float* ms) {
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  setup();
  HIPCK(hipEventRecord(e0, s));
  f();
  hipError_t le = hipGetLastError();
  HIPCK(hipEventRecord(e1, s));
  HIPCK(hipEventSynchronize(e1));
  HIPCK(hipEventElapsedTime(ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (le != hipSuccess) return fl_fail(FAST_LSH_E_DEVICE, "kernel launch while tuning: %s", hipGetErrorString(le));
  return FAST_LSH_OK;
}

void wave_marks_clear(const PairArgs& a, uint32_t S, hipStream_t s);

// Enqueue the fixed-shape prefix on stream s.  With `tune`, the first radix
// pass and the bucket kernel are run once per candidate shape (each run
// produces the same data) and the fastest shapes are stored in j.tc; tuning
// synchronises, so it is never combined with graph capture.
int enqueue_prefix(fast_lsh_ctx* c, Job& j, hipStream_t s, bool prof, bool tune) {
  auto pb = [&](int st) {
    if (prof) prof_begin(c, st);
  };
  auto pe = [&]() {
    if (prof) prof_end(c);
  };
  fill_u8(reinterpret_cast<uint8_t*>(j.ctrl), sizeof(Ctrl), 0, s);
  fill_u8(reinterpret_cast<uint8_t*>(j.er), j.spread_bytes, 0, s);
  fill_u8(j.flags, j.N, 0, s);
  if (j.pa.qcap) fill_u32(j.pa.q_count, kSpread, 0, s);
  LAUNCHCK();

  // 1. signatures -> mixed keys (table-major) and sub-key rows, per station
  pb(FAST_LSH_STAGE_SIGNATURES);
  for (uint32_t st = 0; st < j.S; ++st) {
    if (j.f[st].n == 0) continue;
    SigArgs sa = fl_sig_args(j.h, &j.f[st], j.dhash, &j.ctrl->err);
    sa.table_begin = 0;
    sa.table_count = j.t;
    sa.vec_load = j.vec[st];
    sa.mkeys = j.mkeys;
    sa.rows = j.rows;
    sa.out_stride = j.N;
    sa.out_base = j.base[st];
    sa.mix = j.S > 1 ? kMixStation : kMixFull;
    sa.tag = (uint64_t)st << 60;
    sa.tables_per_group = j.pl.TG;
    sa.row_dw = j.pl.row_dw;
    sa.row_pitch = j.pl.row_pitch;
    launch_sig(j.cap[st], j.minmax, sa, s);
  }
  pe();
  LAUNCHCK();

  // 2. stable radix passes on the top B bits, all tables at once
  uint64_t *gk = j.ak, *gk2 = j.bk;
  uint32_t *gv = j.av, *gv2 = j.bv;
  if (tune) {
    float best = 1e30f;
    uint32_t bestv = 0;
    for (uint32_t v = 0; v < kRadixTileVariants; ++v) {
      float ms = 0;
      RC(time_launch(s, [] {}, [&] { radix_pass(j.mkeys, nullptr, gk, gv, j.N, j.t, 64 - j.B, j.hist, j.sums, v, s); },
                     &ms));
      if (ms < best) {
        best = ms;
        bestv = v;
      }
    }
    j.tc.radix_variant = bestv;
  }
  pb(FAST_LSH_STAGE_GROUP);
  for (uint32_t pass = 0; pass < j.B / 8; ++pass) {
    const uint32_t shift = 64 - j.B + 8 * pass;
    radix_pass(pass == 0 ? j.mkeys : gk2, pass == 0 ? nullptr : gv2, gk, gv, j.N, j.t, shift, j.hist, j.sums,
               j.tc.radix_variant, s);
    std::swap(gk, gk2);
    std::swap(gv, gv2);
  }
  pe();
  LAUNCHCK();
  j.sorted_k = gk2;
  j.sorted_v = gv2;
  j.scratch_k = gk;
  j.scratch_v = gv;

  // 3. buckets, deferred big bins, exclusion counts
  j.ba.keys = j.sorted_k;
  j.ba.vals = j.sorted_v;
  if (tune) {
    // The bucket kernel reorders the ids of each bin (the keys stay in radix
    // order), so every candidate starts from a saved copy of the radix output.
    const size_t vbytes = (size_t)j.t * j.N * sizeof(uint32_t);
    HIPCK(hipMemcpyAsync(j.scratch_v, j.sorted_v, vbytes, hipMemcpyDeviceToDevice, s));
    auto restore = [&] {
      (void)hipMemcpyAsync(j.sorted_v, j.scratch_v, vbytes, hipMemcpyDeviceToDevice, s);
      fill_u8(reinterpret_cast<uint8_t*>(j.er), j.spread_bytes, 0, s);
      fill_u32(&j.ctrl->big_count, 2, 0, s);  // big_count, bin_count
    };
    static const uint32_t chunks[] = {256, 512, 768, 1024};
    float best = 1e30f;
    uint32_t bestc = j.tc.bucket_chunk;
    for (uint32_t ch : chunks) {
      BucketArgs b = j.ba;
      b.chunk = ch;
      float ms = 0;
      RC(time_launch(s, restore, [&] { launch_bucket(b, j.t, s); }, &ms));
      if (ms < best) {
        best = ms;
        bestc = ch;
      }
    }
    j.tc.bucket_chunk = bestc;
    restore();
    LAUNCHCK();
  }
  j.ba.chunk = j.tc.bucket_chunk;
  pb(FAST_LSH_STAGE_BUCKETS);
  launch_bucket(j.ba, j.t, s);
  pe();
  LAUNCHCK();
  pb(FAST_LSH_STAGE_BIG_BINS);
  launch_bigbin(j.ba, j.bins, j.bigbin_grid, j.scratch_k, j.scratch_v, s);
  pe();
  LAUNCHCK();
  for (uint32_t st = 0; st < j.S; ++st)
    launch_count_flags(j.flags + j.base[st], j.base[st + 1] - j.base[st], &j.ctrl->st_flagged[st],
                       &j.ctrl->n_flagged, s);
  LAUNCHCK();

  // 4. pairs of small buckets
  j.pa.order = j.sorted_v;
  if (j.parts) return FAST_LSH_OK;  // the partitioned search launches its own pair passes
  wave_marks_clear(j.pa, j.t, s);
  pb(FAST_LSH_STAGE_PAIRS);
  launch_pairs_wave(j.pa, j.marks, j.t, j.rswl, j.ba.small_max, s);
  pe();
  LAUNCHCK();
  if (pair_launch_queues(j.pa)) {
    pb(FAST_LSH_STAGE_PAIR_CHECKS);
    launch_check_queue(j.pa, s);
    pe();
    LAUNCHCK();
  }
  return FAST_LSH_OK;
}

// The candidate queue of the pair kernels' need == 2 form: N / 64 entries
// per spread slot, between 64 and 32,768 (one launch of a 5-year station
// queues about 8,000 per slot on average, unevenly: at 16,384 a few chunks
// per search found their slot full and ran again).
int alloc_queue(fast_lsh_ctx* c, uint64_t N, uint32_t S, uint32_t T, Job* j) {
  // (a context with an HBM budget has no automatic queue: its searches'
  // memory stays what it was without one)
  const uint32_t cfg = c->config.queue_slot;
  uint32_t qcap = cfg == FAST_LSH_QUEUE_OFF || (cfg == 0 && c->budget) ? 0u
                  : cfg ? cfg : (uint32_t)std::min<uint64_t>(32768, std::max<uint64_t>(64, N / 64));
  if ((uint64_t)T * ((N + 63) / 64) >= (1ull << 32)) qcap = 0;  // queue entries name their chunk in 32 bits
  c->pair_redos = 0;
  uint4* q = nullptr;
  unsigned int *cnt = nullptr, *any = nullptr;
  uint8_t* ovf = nullptr;
  unsigned long long* tally = nullptr;
  if (qcap) {
    // an automatic queue that the free HBM does not hold is left out
    // (checks in place); a size asked for is an error
    int rc = ws<uint4>(c, "cand_queue", (uint64_t)kSpread * qcap, &q);
    if (rc == FAST_LSH_OK) rc = ws<unsigned int>(c, "cand_count", kSpread + 1, &cnt);
    // overflow marks of a small-bucket launch: one per 64 positions of a table
    const uint64_t marks = (uint64_t)T * ((N + 63) / 64);
    if (rc == FAST_LSH_OK) rc = ws<uint8_t>(c, "cand_ovf_wave", std::max<uint64_t>(marks, 1), &ovf);
    if (rc == FAST_LSH_OK) rc = ws<unsigned long long>(c, "redo_tally", 2ull * S * kSpread, &tally);
    if (rc == FAST_LSH_E_NOMEM && cfg == 0) qcap = 0;
    else RC(rc);
    any = cnt ? cnt + kSpread : nullptr;
  }
  c->last_qcap = qcap ? qcap : FAST_LSH_QUEUE_OFF;
  if (j) {
    j->pa.q = q;
    j->pa.q_count = cnt;
    j->pa.qcap = qcap;
    j->pa.q_any = any;
    j->pa.q_ovf = ovf;  // small-bucket launches; the tiled ones bring their own marks
    j->redo_tally = tally;
  }
  return FAST_LSH_OK;
}

// A second run of a pair launch's marked workgroups (checks in place, the
// votes already counted by the first run).
PairArgs redo_args(const Job& j, const PairArgs& a) {
  PairArgs r = a;
  r.redo = 1;
  r.qcap = 0;
  r.e_voted = j.redo_tally;
  r.n_distinct = j.redo_tally + (uint64_t)a.nstation * kSpread;
  r.big_voted = nullptr;
  return r;
}

// Before a small-bucket pair launch of S tables that queues: no chunk marked.
void wave_marks_clear(const PairArgs& a, uint32_t S, hipStream_t s) {
  if (!pair_launch_queues(a)) return;
  fill_u8(a.q_ovf, (uint64_t)S * ((a.n + 63) / 64), 0, s);
  fill_u32(a.q_any, 1, 0, s);
}

// After a small-bucket pair launch and its checks: the chunks that found
// their queue slot full run again (synchronises when the launch queued).
int wave_settle(fast_lsh_ctx* c, const Job& j, const PairArgs& a, const uint8_t* marks, uint32_t S,
                uint32_t small_max) {
  if (!pair_launch_queues(a)) return FAST_LSH_OK;
  unsigned int any = 0;
  RC(d2h(c, &any, a.q_any));
  if (!any) return FAST_LSH_OK;
  ++c->pair_redos;
  prof_begin(c, FAST_LSH_STAGE_PAIRS);
  launch_pairs_wave(redo_args(j, a), marks, S, j.rswl, small_max, c->stream);
  prof_end(c);
  LAUNCHCK();
  return FAST_LSH_OK;
}

// The exact checks of what a pair launch queued (they also empty the queue).
int pair_checks(fast_lsh_ctx* c, const PairArgs& a) {
  if (!pair_launch_queues(a)) return FAST_LSH_OK;
  prof_begin(c, FAST_LSH_STAGE_PAIR_CHECKS);
  launch_check_queue(a, c->stream);
  prof_end(c);
  LAUNCHCK();
  return FAST_LSH_OK;
}

// One small-bucket pair pass: the launch, its queued checks and the second
// run of chunks that found their queue slot full.
int wave_pass(fast_lsh_ctx* c, const Job& j, const PairArgs& a, const uint8_t* marks, uint32_t S, uint32_t small_max) {
  wave_marks_clear(a, S, c->stream);
  prof_begin(c, FAST_LSH_STAGE_PAIRS);
  launch_pairs_wave(a, marks, S, j.rswl, small_max, c->stream);
  prof_end(c);
  LAUNCHCK();
  RC(pair_checks(c, a));
  return wave_settle(c, j, a, marks, S, small_max);
}

// Pairs of the large buckets (tiled kernel).  Tile counts and their offsets
// are computed on the device (members are read in place from the sorted
// order, excluded ones marked dead); the host reads back the tile total to
// size the grid.
int run_big_pairs(fast_lsh_ctx* c, Job& j, uint32_t big_count, const PairArgs& args, unsigned long long* work) {
  if (big_count == 0) return FAST_LSH_OK;
  hipStream_t s = c->stream;
  uint64_t *toff, *sums;
  RC(ws<uint64_t>(c, "big_toff", big_count + 1, &toff));
  RC(ws<uint64_t>(c, "big_sums", scan_sums_elems(big_count, 1), &sums));
  // tile edge: 128 (two tiles of rows and ids in about 18 KB of LDS, so that
  // eight workgroups share a CU and hide the row reads), smaller when rows are
  // long enough that two tiles would exceed 64 KB
  const uint32_t fit = 65536 / (8 * j.rswl + 8);
  uint32_t tb = 128;
  while (tb > 16 && tb > fit) tb >>= 1;
  launch_tile_counts(j.bdesc, big_count, tb, toff, work, s);
  scan_u64(toff, big_count, 1, sums, toff + big_count, s);
  LAUNCHCK();
  uint64_t units = 0;
  RC(d2h(c, &units, toff + big_count));
  uint32_t* owner;  // bucket of every tile unit
  RC(ws<uint32_t>(c, "big_owner", units + 1, &owner));
  launch_unit_owner(toff, big_count, owner, s);
  LAUNCHCK();
  // at most 2^21 workgroups of 256 threads per launch (work-items per grid
  // dimension stay below 2^32, and one launch's queued candidates mostly fit
  // the queue)
  PairArgs pa = args;
  pa.big_voted = work;
  if (pair_launch_queues(pa)) {
    if (units >= (1ull << 32)) {
      pa.qcap = 0;  // (queue entries name their unit in 32 bits)
    } else {  // overflow marks per unit
      RC(ws<uint8_t>(c, "cand_ovf_tiles", std::max<uint64_t>(units, 1), &pa.q_ovf));
      fill_u8(pa.q_ovf, units, 0, s);
      fill_u32(pa.q_any, 1, 0, s);
    }
  }
  for (uint64_t u0 = 0; u0 < units; u0 += 1u << 21) {
    const uint32_t cnt = (uint32_t)std::min<uint64_t>(1u << 21, units - u0);
    prof_begin(c, FAST_LSH_STAGE_BIG_PAIRS);
    launch_pairs_tile(pa, toff, owner, u0, cnt, j.bdesc, tb, j.rswl, s);
    prof_end(c);
    LAUNCHCK();
    RC(pair_checks(c, pa));
  }
  if (pair_launch_queues(pa)) {  // units whose queue slot filled up run again
    unsigned int any = 0;
    RC(d2h(c, &any, pa.q_any));
    if (any) {
      ++c->pair_redos;
      const PairArgs r = redo_args(j, pa);
      for (uint64_t u0 = 0; u0 < units; u0 += 1u << 21) {
        const uint32_t cnt = (uint32_t)std::min<uint64_t>(1u << 21, units - u0);
        prof_begin(c, FAST_LSH_STAGE_BIG_PAIRS);
        launch_pairs_tile(r, toff, owner, u0, cnt, j.bdesc, tb, j.rswl, s);
        prof_end(c);
        LAUNCHCK();
      }
    }
  }
  return FAST_LSH_OK;
}

int set_out_buffers(fast_lsh_ctx* c, Job& j, uint64_t out_cap) {
  uint32_t *oi, *oj;
  uint8_t* ov;
  RC(ws<uint32_t>(c, "out_i", out_cap, &oi));
  RC(ws<uint32_t>(c, "out_j", out_cap, &oj));
  RC(ws<uint8_t>(c, "out_v", out_cap, &ov));
  j.pa.out_i = oi;
  j.pa.out_j = oj;
  j.pa.out_v = ov;
  j.pa.out_cap = (uint32_t)std::min<uint64_t>(out_cap, 0xFFFFFFFFull);
  return FAST_LSH_OK;
}

// 5. canonical order: sort the reported (i << 32 | j) by LSD radix over the
// bits in use, then per-station offsets and counters.
int finish_output(fast_lsh_ctx* c, Job& j, uint64_t cnt, bool distinct, fast_lsh_stats* per_station,
                  uint64_t* station_offsets) {
  hipStream_t s = c->stream;
  const uint32_t S = j.S;
  const uint64_t N = j.N;
  uint64_t *rk0, *rk1;
  uint32_t *rv0, *rv1;
  RC(ws<uint64_t>(c, "res_k0", cnt + 1, &rk0));
  RC(ws<uint64_t>(c, "res_k1", cnt + 1, &rk1));
  RC(ws<uint32_t>(c, "res_v0", cnt + 1, &rv0));
  RC(ws<uint32_t>(c, "res_v1", cnt + 1, &rv1));
  launch_pack_out(j.pa.out_i, j.pa.out_j, j.pa.out_v, cnt, rk0, rv0, s);
  LAUNCHCK();
  if (cnt > 1) {
    const uint32_t nb = fl_key_bits((uint32_t)std::max<uint64_t>(N, 2));
    const uint32_t ont = radix_tiles(cnt, 0);
    uint32_t *ohist, *osums;
    RC(ws<uint32_t>(c, "ohist", (uint64_t)256 * ont, &ohist));
    RC(ws<uint32_t>(c, "osums", scan_sums_elems((uint64_t)256 * ont, 1), &osums));
    std::vector<uint32_t> shifts;
    for (uint32_t sh = 0; sh < nb; sh += 8) shifts.push_back(sh);
    for (uint32_t sh = 0; sh < nb; sh += 8) shifts.push_back(32 + sh);
    for (uint32_t sh : shifts) {
      prof_begin(c, FAST_LSH_STAGE_OUTPUT);
      radix_pass(rk0, rv0, rk1, rv1, cnt, 1, sh, ohist, osums, 0, s);
      prof_end(c);
      LAUNCHCK();
      std::swap(rk0, rk1);
      std::swap(rv0, rv1);
    }
  }
  // keep the sorted result under the fixed names read by fast_lsh_copy_result
  if (c->ws["res_k0"].p != rk0) {
    std::swap(c->ws["res_k0"], c->ws["res_k1"]);
    std::swap(c->ws["res_v0"], c->ws["res_v1"]);
  }
  launch_station_offsets(rk0, cnt, j.sbase, S, j.ctrl->st_offs, s);
  launch_spread_reduce(j.er, j.mb, j.ev, j.nd, S, j.ctrl->st_sum, s);
  launch_work_reduce(j.work, j.ctrl->work, s);
  LAUNCHCK();
  Ctrl hc;
  RC(d2h(c, &hc, j.ctrl));
  prof_collect(c);
  c->last_work.big_voted = hc.work[0];
  c->last_work.big_members = hc.work[1];
  c->last_work.big_candidates = hc.work[2];
  c->last_work.search_calls += 1;
  c->last_work.pair_redos = c->pair_redos;
  c->res_count = cnt;
  c->res_valid = true;
  for (uint32_t st = 0; st < S; ++st) {
    if (station_offsets) station_offsets[st] = hc.st_offs[st];
    if (!per_station) continue;
    fast_lsh_stats& o = per_station[st];
    o.n_out = hc.st_offs[st + 1] - hc.st_offs[st];
    o.e_raw = hc.st_sum[4 * st + 0];
    o.max_bucket = hc.st_sum[4 * st + 1];
    o.e_voted = hc.st_sum[4 * st + 2];
    o.n_distinct = distinct ? hc.st_sum[4 * st + 3] : ~0ull;
    o.n_flagged = hc.st_flagged[st];
  }
  if (station_offsets) station_offsets[S] = hc.st_offs[S];
  return FAST_LSH_OK;
}

// Partitioned search with the dynamic occurrence filter (sections 6.4,
// 6.5), after the prefix has grouped and segmented every table without the
// static filter.  Partitions are consecutive id ranges taken in order; for
// partition p: (1) each of its fingerprints counts its candidates (distinct
// other fingerprints at least min_lag away, not excluded, sharing a bucket);
// (2) those over occ_num/occ_den of the partition's size are excluded with
// all their candidates; (3) the pairs whose smaller id lies in p are
// reported.  The exclusion bytes j.flags start at zero and only grow.
//
// The passes are merged across partitions where the exclusions allow it.
// A fingerprint's count depends only on the exclusions made before its
// partition, so one counting pass serves every partition from the current
// one to the last, until some partition excludes: then the partitions after
// it are counted again.  Partition p's pairs are reported with the
// exclusions as they stand after p, and those change only at a partition
// that excludes, so one reporting pass covers each run of partitions up to
// the next one that excludes.  Before all this, one pass counts and
// reports every partition at once (mode 4), which is the result when no
// partition excludes (the usual case) whatever the partition count; when
// some partition does, that pass's output is dropped and the scheme above
// runs: each partition that excludes adds an exclusion pass and at most one
// counting and one reporting pass to the first counting pass and the last
// reporting pass.
int run_partitions(fast_lsh_ctx* c, Job& j, const fast_lsh_filter& flt, uint32_t big_count, uint64_t out_cap,
                   Ctrl* hc_out) {
  hipStream_t s = c->stream;
  const uint64_t N = j.N;
  const uint32_t P = j.parts;
  uint32_t* cand;
  uint8_t *fp, *exn;
  unsigned long long *always, *dummy;
  unsigned int* nfp;
  RC(ws<uint32_t>(c, "part_cand", N, &cand));
  RC(ws<uint8_t>(c, "part_fp", N, &fp));
  RC(ws<uint8_t>(c, "part_exnext", N, &exn));
  RC(ws<unsigned long long>(c, "part_one", 1, &always));
  RC(ws<unsigned long long>(c, "part_work", 3 * kSpread, &dummy));
  RC(ws<unsigned int>(c, "part_nfp", std::max<uint32_t>(P, 1), &nfp));
  fill_u64(reinterpret_cast<uint64_t*>(always), 1, 1, s);  // the pair kernels always consult the exclusions
  auto lo_of = [&](uint32_t p) { return (uint32_t)(N * p / P); };
  // one pass of mode m over the pairs whose ids the mode restricts to [lo, hi)
  auto pass = [&](const PairArgs& base, int mode, uint32_t lo, uint32_t hi, unsigned long long* work) -> int {
    PairArgs m = base;
    m.part_mode = mode;
    m.plo = lo;
    m.phi = hi;
    RC(wave_pass(c, j, m, j.marks, j.t, j.ba.small_max));
    return run_big_pairs(c, j, big_count, m, work);
  };
  auto count_from = [&](const PairArgs& base, uint32_t p) -> int {
    fill_u32(cand + lo_of(p), N - lo_of(p), 0, s);
    return pass(base, 1, lo_of(p), (uint32_t)N, dummy);
  };
  Ctrl hc;
  for (int attempt = 0; attempt < 2; ++attempt) {
    RC(set_out_buffers(c, j, out_cap));
    fill_u8(reinterpret_cast<uint8_t*>(j.ev), 2ull * kSpread * sizeof(unsigned long long), 0, s);
    fill_u64(reinterpret_cast<uint64_t*>(j.work), 3 * kSpread, 0, s);
    fill_u32(&j.ctrl->out_count, 1, 0, s);
    fill_u8(j.flags, N, 0, s);
    fill_u8(fp, N, 0, s);
    fill_u8(exn, N, 0, s);
    PairArgs pa = j.pa;
    pa.n_flagged = always;
    pa.cand = cand;
    pa.fp = fp;
    pa.ex_next = exn;
    uint32_t unreported = 0;  // first partition whose pairs are not reported yet
    bool done = false;        // every partition's pairs are in the output
    if (flt.occ_den) {
      // First one pass that counts and reports every partition, right while
      // no partition excludes (the usual case); if one does, its output is
      // dropped and the partitions are taken as below.
      fill_u32(cand, N, 0, s);
      RC(pass(pa, 4, 0, (uint32_t)N, j.work));
      fill_u32(nfp, P, 0, s);
      for (uint32_t p = 0; p < P; ++p)
        launch_part_flag(j.flags, cand, lo_of(p), lo_of(p + 1), flt.occ_num, flt.occ_den, fp, nfp + p, s);
      LAUNCHCK();
      std::vector<unsigned int> hn(P, 0);
      RC(d2h(c, hn.data(), nfp, P));
      done = std::all_of(hn.begin(), hn.end(), [](unsigned int x) { return x == 0; });
      if (!done) {
        fill_u8(reinterpret_cast<uint8_t*>(j.ev), 2ull * kSpread * sizeof(unsigned long long), 0, s);
        fill_u64(reinterpret_cast<uint64_t*>(j.work), 3 * kSpread, 0, s);
        fill_u32(&j.ctrl->out_count, 1, 0, s);
        fill_u8(fp, N, 0, s);
      }
    }
    if (flt.occ_den && !done) {
      RC(count_from(pa, 0));
      for (uint32_t p = 0; p < P; ++p) {
        const uint32_t lo = lo_of(p), hi = lo_of(p + 1);
        if (hi == lo) continue;
        fill_u32(nfp, 1, 0, s);
        launch_part_flag(j.flags, cand, lo, hi, flt.occ_num, flt.occ_den, fp, nfp, s);
        LAUNCHCK();
        unsigned int hn = 0;
        RC(d2h(c, &hn, nfp));
        if (!hn) continue;
        // the partitions before p see the exclusions as they stand now
        if (unreported < p) RC(pass(pa, 3, lo_of(unreported), lo, j.work));
        unreported = p;
        RC(pass(pa, 2, lo, hi, dummy));
        launch_part_merge(j.flags, fp, exn, N, s);
        LAUNCHCK();
        if (p + 1 < P) RC(count_from(pa, p + 1));
      }
    }
    if (!done) RC(pass(pa, 3, lo_of(unreported), (uint32_t)N, j.work));
    RC(d2h(c, &hc, j.ctrl));
    if (hc.out_count <= out_cap) break;
    out_cap = (uint64_t)hc.out_count + 1024;
  }
  // final exclusions
  fill_u64(reinterpret_cast<uint64_t*>(&j.ctrl->n_flagged), 1, 0, s);
  fill_u64(reinterpret_cast<uint64_t*>(&j.ctrl->st_flagged[0]), 1, 0, s);
  launch_count_flags(j.flags, N, &j.ctrl->st_flagged[0], &j.ctrl->n_flagged, s);
  LAUNCHCK();
  *hc_out = hc;
  return FAST_LSH_OK;
}

}  // namespace

int fl_search_stations(fast_lsh_ctx* c, const fast_lsh_hash* h, uint32_t S, const fast_lsh_fps* f,
                       const fast_lsh_filter* flt_in, uint32_t flags, fast_lsh_stats* per_station,
                       uint64_t* station_offsets, uint32_t parts) {
  hipStream_t s = c->stream;
  const bool distinct = (flags & FAST_LSH_WANT_DISTINCT) != 0;
  // The partitioned search applies the occurrence filter dynamically per
  // partition; the bucket stage then runs without its static form.
  fast_lsh_filter flt_buckets = *flt_in;
  if (parts) flt_buckets.occ_num = flt_buckets.occ_den = 0;
  const fast_lsh_filter* flt = &flt_buckets;
  Job j;
  j.parts = parts;
  j.S = S;
  j.f = f;
  j.h = h;
  j.t = h->num_tables;
  j.minmax = h->scheme == FAST_LSH_MINMAX;
  j.base.assign(S + 1, 0);
  for (uint32_t st = 0; st < S; ++st) j.base[st + 1] = j.base[st] + f[st].n;
  j.N = j.base[S];
  c->res_valid = false;
  c->res_stations = S;
  if (j.N == 0) {
    c->res_count = 0;
    c->res_valid = true;
    for (uint32_t st = 0; st < S; ++st) {
      if (per_station) {
        memset(&per_station[st], 0, sizeof(fast_lsh_stats));
        if (!distinct) per_station[st].n_distinct = ~0ull;
      }
    }
    if (station_offsets) memset(station_offsets, 0, (S + 1) * sizeof(uint64_t));
    return FAST_LSH_OK;
  }
  const uint64_t N = j.N, t = j.t, tn = t * N;
  // the partitioned passes find each pair's first shared table: one table group
  j.pl = make_plan(j.t, flt->min_votes, distinct || parts > 0, true);
  uint64_t n_max = 0;
  for (uint32_t st = 0; st < S; ++st) n_max = std::max<uint64_t>(n_max, f[st].n);
  j.B = c->config.bin_bits ? c->config.bin_bits : bin_bits(n_max, S > 1);
  c->last_bin_bits = j.B;

  RC(fl_upload_hash(c, h, &j.dhash));
  j.cap.assign(S, 0);
  j.vec.assign(S, false);
  for (uint32_t st = 0; st < S; ++st) {
    if (f[st].n == 0) continue;
    int cp;
    bool vc;
    RC(fl_row_capacity(c, &f[st], &cp, &vc));
    j.cap[st] = cp;
    j.vec[st] = vc;
  }

  // workspace
  RC(ws<Ctrl>(c, "ctrl", 1, &j.ctrl));
  j.spread_bytes = (uint64_t)S * kSpread * (3 * sizeof(unsigned long long) + sizeof(unsigned int));
  uint8_t* spread;
  RC(ws<uint8_t>(c, "spread", j.spread_bytes, &spread));
  j.er = reinterpret_cast<unsigned long long*>(spread);
  j.ev = j.er + (uint64_t)S * kSpread;
  j.nd = j.ev + (uint64_t)S * kSpread;
  j.mb = reinterpret_cast<unsigned int*>(j.nd + (uint64_t)S * kSpread);
  RC(ws<unsigned long long>(c, "work", 3 * kSpread, &j.work));
  RC(ws<uint64_t>(c, "mkeys", tn, &j.mkeys));
  RC(ws<uint32_t>(c, "rows", (uint64_t)j.pl.G * N * j.pl.row_pitch, &j.rows));
  RC(ws<uint64_t>(c, "ak", tn, &j.ak));
  RC(ws<uint32_t>(c, "av", tn, &j.av));
  RC(ws<uint64_t>(c, "bk", tn, &j.bk));
  RC(ws<uint32_t>(c, "bv", tn, &j.bv));
  const uint32_t nt_max = radix_tiles(N, kRadixTileVariants - 1);  // the smallest tile has the most tiles
  RC(ws<uint32_t>(c, "hist", (uint64_t)256 * nt_max * t, &j.hist));
  RC(ws<uint32_t>(c, "sums", scan_sums_elems((uint64_t)256 * nt_max, j.t), &j.sums));
  RC(ws<uint8_t>(c, "flags", N, &j.flags));
  // station bases (S + 1) and each station's occurrence bound (S)
  RC(ws<uint64_t>(c, "station_base", 2 * S + 1, &j.sbase));
  // Buckets of at most smax members are marked in place and handled by the
  // wave-per-chunk pair kernel; larger ones go to the tiled kernel.
  const uint32_t smax = pair_small_max(j.pl.need, distinct, parts, j.pl.row_dw);
  const uint64_t cap_big = tn / (smax + 1) + 1 + bucket_desc_slack(tn / (smax + 1) + 1, t);
  const uint64_t cap_bin = tn / 129 + t + 1;  // oversized bins and mixed bins above 128 elements
  RC(ws<uint4>(c, "bdesc", cap_big, &j.bdesc));
  RC(ws<uint4>(c, "bins", cap_bin, &j.bins));
  RC(ws<uint8_t>(c, "marks", tn, &j.marks));
  j.bigbin_grid = (uint32_t)std::min<uint64_t>(cap_bin, 512);
  j.rswl = j.pl.row_dw | 1u;
  uint64_t out_cap = std::max<uint64_t>(1u << 20, N / 8);
  {
    std::vector<uint64_t> hb(j.base);
    for (uint32_t st = 0; st < S; ++st) hb.push_back(occ_bound(j.base[st + 1] - j.base[st], flt));
    RC(h2d(c, j.sbase, hb.data(), 2 * S + 1));
  }

  BucketArgs& ba = j.ba;
  memset(&ba, 0, sizeof ba);
  ba.n = N;
  ba.bin_shift = 64 - j.B;
  ba.station_base = j.sbase;
  ba.occ_max = j.sbase + S + 1;
  ba.nstation = S;
  ba.occ_num = flt->occ_num;
  ba.occ_den = flt->occ_den;
  ba.min_lag = flt->min_lag;
  ba.flags = j.flags;
  ba.small_max = smax;
  ba.marks = j.marks;
  ba.big_desc = j.bdesc;
  ba.big_count = &j.ctrl->big_count;
  ba.bin_desc = j.bins;
  ba.bin_count = &j.ctrl->bin_count;
  ba.e_raw = j.er;
  ba.max_bucket = j.mb;

  PairArgs& pa = j.pa;
  memset(&pa, 0, sizeof pa);
  pa.flags = j.flags;
  pa.rows = j.rows;
  pa.mkeys = j.mkeys;
  pa.n = N;
  pa.t = j.t;
  pa.G = j.pl.G;
  pa.tables_per_group = j.pl.TG;
  pa.row_dw = j.pl.row_dw;
  pa.row_pitch = j.pl.row_pitch;
  pa.min_lag = flt->min_lag;
  pa.min_votes = flt->min_votes;
  pa.need = j.pl.need;
  pa.want_distinct = distinct;
  pa.out_count = &j.ctrl->out_count;
  pa.e_voted = j.ev;
  pa.n_distinct = j.nd;
  pa.station_base = j.sbase;
  pa.nstation = S;
  pa.n_flagged = &j.ctrl->n_flagged;
  RC(alloc_queue(c, N, S, j.t, &j));
  RC(set_out_buffers(c, j, out_cap));

  // launch shapes: fixed, or tuned once per shape
  const std::vector<uint64_t> shape{S, N, t, j.B};
  bool tune = false;
  if (c->config.autotune) {
    auto it = c->tuned.find(shape);
    if (it != c->tuned.end()) {
      j.tc = it->second;
    } else {
      tune = true;
    }
  } else {
    j.tc.radix_variant = 0;
    for (uint32_t v = 0; v < kRadixTileVariants; ++v)
      if (radix_tile_elems(v) == c->config.radix_tile) j.tc.radix_variant = v;
    j.tc.bucket_chunk = c->config.bucket_chunk;
  }

  // 1-4: the fixed-shape prefix, eager or as a replayed graph
  const bool use_graph = (flags & FAST_LSH_USE_GRAPH) && !tune && !parts;
  if (use_graph) {
    std::vector<uint64_t> key{S, N, t, h->band_rows, h->scheme, h->dim, flt->min_lag, flt->min_votes,
                              flt->occ_num, flt->occ_den, flags, j.tc.radix_variant, j.tc.bucket_chunk,
                              c->ws_generation, (uint64_t)(uintptr_t)s, j.pa.qcap};
    for (uint32_t st = 0; st < S; ++st) {
      key.push_back((uint64_t)(uintptr_t)f[st].indices);
      key.push_back((uint64_t)(uintptr_t)f[st].offsets);
      key.push_back(f[st].fixed_nnz);
      key.push_back(f[st].n);
      key.push_back((uint64_t)j.cap[st] * 2 + (j.vec[st] ? 1 : 0));
    }
    if (!c->graph || key != c->graph_key) {
      if (c->graph) {
        HIPCK(hipGraphExecDestroy(c->graph));
        c->graph = nullptr;
      }
      if (!c->capture_stream) HIPCK(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
      HIPCK(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
      const int rc = enqueue_prefix(c, j, c->capture_stream, false, false);
      hipGraph_t g = nullptr;
      const hipError_t ee = hipStreamEndCapture(c->capture_stream, &g);
      if (rc != FAST_LSH_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      HIPCK(ee);
      hipGraphExec_t ex = nullptr;
      const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCK(ie);
      c->graph = ex;
      c->graph_key = key;
    } else {
      // the sorted arrays' location follows from the pass count only
      j.sorted_k = (j.B / 8) % 2 ? j.ak : j.bk;
      j.sorted_v = (j.B / 8) % 2 ? j.av : j.bv;
      j.scratch_k = (j.B / 8) % 2 ? j.bk : j.ak;
      j.scratch_v = (j.B / 8) % 2 ? j.bv : j.av;
      j.pa.order = j.sorted_v;
    }
    prof_begin(c, FAST_LSH_STAGE_GRAPH);
    HIPCK(hipGraphLaunch(c->graph, s));
    prof_end(c);
    ++c->graph_replays;
  } else {
    RC(enqueue_prefix(c, j, s, true, tune));
    if (tune) c->tuned[shape] = j.tc;
  }
  c->last_choice = j.tc;

  Ctrl hc;
  RC(d2h(c, &hc, j.ctrl));
  if (hc.err) return fl_fail(FAST_LSH_E_INVALID, "a fingerprint is empty or holds an index >= dim (%u)", h->dim);
  if (!parts) RC(wave_settle(c, j, j.pa, j.marks, j.t, j.ba.small_max));  // the prefix's small-bucket pairs
  if (parts) {
    RC(run_partitions(c, j, *flt_in, hc.big_count, out_cap, &hc));
    return finish_output(c, j, hc.out_count, distinct, per_station, station_offsets);
  }

  // 4b. large buckets; 4c. a second pair pass if the output overflowed
  for (int attempt = 0; attempt < 2; ++attempt) {
    fill_u64(reinterpret_cast<uint64_t*>(j.work), 3 * kSpread, 0, s);
    if (attempt == 1) {
      out_cap = (uint64_t)hc.out_count + 1024;
      RC(set_out_buffers(c, j, out_cap));
      fill_u8(reinterpret_cast<uint8_t*>(j.ev), 2ull * S * kSpread * sizeof(unsigned long long), 0, s);
      fill_u32(&j.ctrl->out_count, 1, 0, s);
      RC(wave_pass(c, j, j.pa, j.marks, j.t, j.ba.small_max));
    }
    RC(run_big_pairs(c, j, hc.big_count, j.pa, j.work));
    RC(d2h(c, &hc, j.ctrl));
    if (hc.out_count <= out_cap) break;
  }

  return finish_output(c, j, hc.out_count, distinct, per_station, station_offsets);
}

// ---------------------------------------------------------------------------
// Bounded-memory search: the same result, with the tables taken in groups of
// group_tables so that sorting needs room for one group only.  Pass 1 sorts
// every group and finds its buckets (sizes, counters, occurrence flags); it
// also writes each fingerprint's sub-key rows and the high words of its split
// mixed keys for every table.  Pass 2 runs the pair kernels on every group's
// tables with the final flags: for the groups pass 1 kept (bucket-ordered
// ids, marks and large-bucket descriptors, as many groups as HBM holds)
// directly, for the others after rebuilding the group's keys from the stored
// words and sorting and segmenting it again.  Exact key comparisons use
// sub-key plus high word, so no table's full keys stay resident.
// ---------------------------------------------------------------------------
int fl_search_bounded(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f, const fast_lsh_filter* flt,
                      uint32_t flags, uint32_t group_tables, fast_lsh_stats* stats) {
  hipStream_t s = c->stream;
  const bool distinct = (flags & FAST_LSH_WANT_DISTINCT) != 0;
  Job j;
  j.S = 1;
  j.f = f;
  j.h = h;
  j.t = h->num_tables;
  j.minmax = h->scheme == FAST_LSH_MINMAX;
  j.base = {0, f->n};
  j.N = f->n;
  c->res_valid = false;
  c->res_stations = 1;
  if (j.N == 0) {
    c->res_count = 0;
    c->res_valid = true;
    memset(stats, 0, sizeof *stats);
    if (!distinct) stats->n_distinct = ~0ull;
    return FAST_LSH_OK;
  }
  const uint64_t N = j.N;
  const uint32_t t = j.t;
  const uint32_t TGm = std::min(group_tables, t);
  const uint32_t ngroups = (t + TGm - 1) / TGm;
  const uint64_t gn = (uint64_t)TGm * N;
  j.pl = make_plan(t, flt->min_votes, distinct, false);
  j.B = c->config.bin_bits ? c->config.bin_bits : bin_bits(N, false);
  c->last_bin_bits = j.B;
  RC(fl_upload_hash(c, h, &j.dhash));
  j.cap.assign(1, 0);
  j.vec.assign(1, false);
  {
    int cp;
    bool vc;
    RC(fl_row_capacity(c, f, &cp, &vc));
    j.cap[0] = cp;
    j.vec[0] = vc;
  }
  // persistent: counters, rows, high words, flags; per group: sort buffers
  RC(ws<Ctrl>(c, "ctrl", 1, &j.ctrl));
  j.spread_bytes = (uint64_t)kSpread * (3 * sizeof(unsigned long long) + sizeof(unsigned int));
  uint8_t *spread, *spread2;
  RC(ws<uint8_t>(c, "spread", j.spread_bytes, &spread));
  RC(ws<uint8_t>(c, "spread_pass2", j.spread_bytes, &spread2));
  j.er = reinterpret_cast<unsigned long long*>(spread);
  j.ev = j.er + kSpread;
  j.nd = j.ev + kSpread;
  j.mb = reinterpret_cast<unsigned int*>(j.nd + kSpread);
  RC(ws<unsigned long long>(c, "work", 3 * kSpread, &j.work));
  uint32_t* hi32;
  RC(ws<uint32_t>(c, "rows", (uint64_t)j.pl.G * N * j.pl.row_pitch, &j.rows));
  RC(ws<uint32_t>(c, "hi32", (uint64_t)t * N, &hi32));
  RC(ws<uint8_t>(c, "flags", N, &j.flags));
  RC(ws<uint64_t>(c, "station_base", 3, &j.sbase));  // bases, occurrence bound
  RC(ws<uint64_t>(c, "ak", gn, &j.ak));
  RC(ws<uint32_t>(c, "av", gn, &j.av));
  RC(ws<uint64_t>(c, "bk", gn, &j.bk));  // also receives each group's mixed keys
  RC(ws<uint32_t>(c, "bv", gn, &j.bv));
  j.mkeys = j.bk;
  const uint32_t nt_max = radix_tiles(N, kRadixTileVariants - 1);
  RC(ws<uint32_t>(c, "hist", (uint64_t)256 * nt_max * TGm, &j.hist));
  RC(ws<uint32_t>(c, "sums", scan_sums_elems((uint64_t)256 * nt_max, TGm), &j.sums));
  const uint32_t smax = pair_small_max(j.pl.need, distinct, 0, j.pl.row_dw);
  const uint64_t cap_big = gn / (smax + 1) + 1 + bucket_desc_slack(gn / (smax + 1) + 1, TGm);
  const uint64_t cap_bin = gn / 129 + TGm + 1;
  RC(ws<uint4>(c, "bdesc", cap_big, &j.bdesc));
  RC(ws<uint4>(c, "bins", cap_bin, &j.bins));
  RC(ws<uint8_t>(c, "marks", gn, &j.marks));
  j.bigbin_grid = (uint32_t)std::min<uint64_t>(cap_bin, 512);
  j.rswl = j.pl.row_dw | 1u;
  RC(alloc_queue(c, N, 1, TGm, nullptr));  // before the keep budget counts free memory
  // Groups whose grouping pass 1 keeps for pass 2: at most keep_groups, as
  // many as the free HBM (less a margin) and the budget hold, counting what
  // earlier calls left allocated under these names.
  uint32_t kept = 0;
  uint32_t* keep_ids = nullptr;
  uint8_t* keep_marks = nullptr;
  uint4* keep_desc = nullptr;
  {
    const uint64_t per = gn * 4 + gn + cap_big * sizeof(uint4);
    uint64_t held = 0;
    for (const char* nm : {"keep_ids", "keep_marks", "keep_desc"}) {
      auto it = c->ws.find(nm);
      if (it != c->ws.end()) held += it->second.cap;
    }
    size_t fr = 0, tot = 0;
    HIPCK(hipMemGetInfo(&fr, &tot));
    const uint64_t margin = (4ull << 30) + tot / 50;
    uint64_t avail = (uint64_t)fr + held > margin ? (uint64_t)fr + held - margin : 0;
    if (c->budget) {
      // within a budget, leave room for what the search allocates later (the
      // output records and their sort, the large-bucket tile offsets)
      const uint64_t other = c->ws_total - held;
      const uint64_t later = (64ull << 20) + std::max<uint64_t>(1u << 20, N / 8) * 32 +
                             (gn / (smax + 1) + 2) * 24;
      avail = std::min<uint64_t>(avail, c->budget > other + later ? c->budget - other - later : 0);
    }
    kept = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(ngroups, avail / per), c->config.keep_groups);
    if (kept && (ws<uint32_t>(c, "keep_ids", (uint64_t)kept * gn, &keep_ids) != FAST_LSH_OK ||
                 ws<uint8_t>(c, "keep_marks", (uint64_t)kept * gn, &keep_marks) != FAST_LSH_OK ||
                 ws<uint4>(c, "keep_desc", (uint64_t)kept * cap_big, &keep_desc) != FAST_LSH_OK)) {
      // the memory was not there after all: release what was taken and sort
      // every group again in pass 2
      HIPCK(hipStreamSynchronize(s));
      for (const char* nm : {"keep_ids", "keep_marks", "keep_desc"}) {
        auto it = c->ws.find(nm);
        if (it == c->ws.end()) continue;
        if (it->second.p) {
          HIPCK(hipFree(it->second.p));
          c->ws_total -= it->second.cap;
        }
        c->ws.erase(it);
      }
      ++c->ws_generation;
      kept = 0;
    }
  }
  c->last_kept = kept;
  std::vector<uint32_t> kept_big(kept, 0);
  uint64_t out_cap = std::max<uint64_t>(1u << 20, N / 8);
  {
    const uint64_t hb[3] = {j.base[0], j.base[1], occ_bound(j.base[1] - j.base[0], flt)};
    RC(h2d(c, j.sbase, hb, 3));
  }

  BucketArgs& ba = j.ba;
  memset(&ba, 0, sizeof ba);
  ba.n = N;
  ba.bin_shift = 64 - j.B;
  ba.station_base = j.sbase;
  ba.occ_max = j.sbase + 2;
  ba.nstation = 1;
  ba.occ_num = flt->occ_num;
  ba.occ_den = flt->occ_den;
  ba.min_lag = flt->min_lag;
  ba.flags = j.flags;
  ba.small_max = smax;
  ba.marks = j.marks;
  ba.big_desc = j.bdesc;
  ba.big_count = &j.ctrl->big_count;
  ba.bin_desc = j.bins;
  ba.bin_count = &j.ctrl->bin_count;
  ba.chunk = c->config.bucket_chunk;
  PairArgs& pa = j.pa;
  memset(&pa, 0, sizeof pa);
  pa.flags = j.flags;
  pa.rows = j.rows;
  pa.hi32 = hi32;
  pa.n = N;
  pa.t = t;
  pa.G = j.pl.G;
  pa.tables_per_group = j.pl.TG;
  pa.row_dw = j.pl.row_dw;
  pa.row_pitch = j.pl.row_pitch;
  pa.min_lag = flt->min_lag;
  pa.min_votes = flt->min_votes;
  pa.need = j.pl.need;
  pa.want_distinct = distinct;
  pa.out_count = &j.ctrl->out_count;
  pa.e_voted = j.ev;
  pa.n_distinct = j.nd;
  pa.station_base = j.sbase;
  pa.nstation = 1;
  pa.n_flagged = &j.ctrl->n_flagged;
  RC(alloc_queue(c, N, 1, TGm, &j));
  uint32_t variant = 0;
  for (uint32_t v = 0; v < kRadixTileVariants; ++v)
    if (radix_tile_elems(v) == c->config.radix_tile) variant = v;
  c->last_choice.radix_variant = variant;
  c->last_choice.bucket_chunk = ba.chunk;

  // Signatures, grouping and buckets of tables [tb, tb + tc); pass 1 also
  // writes rows and high words and accounts the buckets.
  // Pass 2 rebuilds the group's mixed keys (mix48(key) << 16) from the high
  // words and sub-key rows pass 1 stored, instead of recomputing signatures.
  // keep_vals: where the last radix pass leaves the group's ids (a kept
  // grouping's slice, sorted in place there by the bucket kernels), or null.
  auto group = [&](uint32_t tb, uint32_t tc, bool first_pass, uint32_t* keep_vals) -> int {
    prof_begin(c, first_pass ? FAST_LSH_STAGE_SIGNATURES : FAST_LSH_STAGE_SPLIT_KEYS);
    if (first_pass) {
      SigArgs sa = fl_sig_args(h, f, j.dhash, &j.ctrl->err);
      sa.table_begin = tb;
      sa.table_count = tc;
      sa.vec_load = j.vec[0];
      sa.mkeys = j.bk;
      sa.rows = j.rows;
      sa.hi32 = hi32;
      sa.mix = kMixSplit;
      sa.tables_per_group = j.pl.TG;
      sa.row_dw = j.pl.row_dw;
      sa.row_pitch = j.pl.row_pitch;
      launch_sig(j.cap[0], j.minmax, sa, s);
    } else {
      launch_split_keys(hi32, j.rows, N, tb, tc, j.pl.TG, j.pl.row_pitch, j.bk, s);
    }
    prof_end(c);
    LAUNCHCK();
    uint64_t *gk = j.ak, *gk2 = j.bk;
    uint32_t *gv = j.av, *gv2 = j.bv;
    prof_begin(c, FAST_LSH_STAGE_GROUP);
    for (uint32_t pass = 0; pass < j.B / 8; ++pass) {
      const uint32_t shift = 64 - j.B + 8 * pass;
      uint32_t* vout = (keep_vals && pass + 1 == j.B / 8) ? keep_vals : gv;
      radix_pass(gk2, pass == 0 ? nullptr : gv2, gk, vout, N, tc, shift, j.hist, j.sums, variant, s);
      std::swap(gk, gk2);
      if (vout == gv)
        std::swap(gv, gv2);
      else
        gv2 = vout;  // gv stays free for the big-bin kernel
    }
    prof_end(c);
    LAUNCHCK();
    j.sorted_k = gk2;
    j.sorted_v = gv2;
    j.scratch_k = gk;
    j.scratch_v = gv;
    fill_u32(&j.ctrl->big_count, 2, 0, s);  // big_count, bin_count
    BucketArgs b = ba;
    b.keys = j.sorted_k;
    b.vals = j.sorted_v;
    // pass 2 repeats the bucket accounting into a scratch copy of the counters
    uint8_t* sp = first_pass ? spread : spread2;
    b.e_raw = reinterpret_cast<unsigned long long*>(sp);
    b.max_bucket = reinterpret_cast<unsigned int*>(sp + (uint64_t)kSpread * 3 * sizeof(unsigned long long));
    prof_begin(c, FAST_LSH_STAGE_BUCKETS);
    launch_bucket(b, tc, s);
    prof_end(c);
    prof_begin(c, FAST_LSH_STAGE_BIG_BINS);
    launch_bigbin(b, j.bins, j.bigbin_grid, j.scratch_k, j.scratch_v, s);
    prof_end(c);
    LAUNCHCK();
    return FAST_LSH_OK;
  };

  fill_u8(reinterpret_cast<uint8_t*>(j.ctrl), sizeof(Ctrl), 0, s);
  fill_u8(spread, j.spread_bytes, 0, s);
  fill_u8(j.flags, N, 0, s);
  Ctrl hc;
  for (uint32_t g = 0; g < ngroups; ++g) {
    const uint32_t tb = g * TGm, tc = std::min(TGm, t - tb);
    // a kept group's marks and descriptors go straight to its own slices
    ba.marks = g < kept ? keep_marks + (uint64_t)g * gn : j.marks;
    ba.big_desc = g < kept ? keep_desc + (uint64_t)g * cap_big : j.bdesc;
    RC(group(tb, tc, true, g < kept ? keep_ids + (uint64_t)g * gn : nullptr));
    if (g < kept) {
      RC(d2h(c, &hc, j.ctrl));
      kept_big[g] = hc.big_count;
    }
  }
  ba.marks = j.marks;
  ba.big_desc = j.bdesc;
  launch_count_flags(j.flags, N, &j.ctrl->st_flagged[0], &j.ctrl->n_flagged, s);
  LAUNCHCK();
  RC(d2h(c, &hc, j.ctrl));
  if (hc.err) return fl_fail(FAST_LSH_E_INVALID, "a fingerprint is empty or holds an index >= dim (%u)", h->dim);

  for (int attempt = 0; attempt < 2; ++attempt) {
    RC(set_out_buffers(c, j, out_cap));
    fill_u8(reinterpret_cast<uint8_t*>(j.ev), 2ull * kSpread * sizeof(unsigned long long), 0, s);
    fill_u64(reinterpret_cast<uint64_t*>(j.work), 3 * kSpread, 0, s);
    fill_u32(&j.ctrl->out_count, 1, 0, s);
    if (j.pa.qcap) fill_u32(j.pa.q_count, kSpread, 0, s);
    for (uint32_t g = 0; g < ngroups; ++g) {
      const uint32_t tb = g * TGm, tc = std::min(TGm, t - tb);
      if (g < kept) {  // pass 1's grouping of this group, with the final flags
        j.pa.order = keep_ids + (uint64_t)g * gn;
        j.pa.table_offset = tb;
        RC(wave_pass(c, j, j.pa, keep_marks + (uint64_t)g * gn, tc, ba.small_max));
        uint4* shared_desc = j.bdesc;
        j.bdesc = keep_desc + (uint64_t)g * cap_big;
        const int rc = run_big_pairs(c, j, kept_big[g], j.pa, j.work);
        j.bdesc = shared_desc;
        RC(rc);
        continue;
      }
      fill_u8(spread2, j.spread_bytes, 0, s);
      RC(group(tb, tc, false, nullptr));
      j.pa.order = j.sorted_v;
      j.pa.table_offset = tb;
      RC(wave_pass(c, j, j.pa, j.marks, tc, j.ba.small_max));
      RC(d2h(c, &hc, j.ctrl));
      RC(run_big_pairs(c, j, hc.big_count, j.pa, j.work));
    }
    RC(d2h(c, &hc, j.ctrl));
    if (hc.out_count <= out_cap) break;
    out_cap = (uint64_t)hc.out_count + 1024;
  }
  return finish_output(c, j, hc.out_count, distinct, stats, nullptr);
}

// ---------------------------------------------------------------------------
// Public entry points
// ---------------------------------------------------------------------------
static int check_filter(const fast_lsh_filter* flt, uint32_t flags) {
  if (!flt) return fl_fail(FAST_LSH_E_INVALID, "filter is NULL");
  if (flt->min_votes < 1) return fl_fail(FAST_LSH_E_INVALID, "min_votes must be >= 1");
  if (flt->occ_den && flt->occ_num > flt->occ_den)
    return fl_fail(FAST_LSH_E_INVALID, "occurrence filter fraction %u/%u above 1", flt->occ_num, flt->occ_den);
  if (flags & ~(uint32_t)(FAST_LSH_WANT_DISTINCT | FAST_LSH_USE_GRAPH))
    return fl_fail(FAST_LSH_E_INVALID, "unknown flags 0x%x", flags);
  return FAST_LSH_OK;
}

extern "C" {

int fast_lsh_copy_result(fast_lsh_ctx* c, uint32_t* oi, uint32_t* oj, uint8_t* ov, uint64_t capacity) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  if (!c->res_valid) return fl_fail(FAST_LSH_E_INVALID, "no search result in this context");
  if (c->res_count > capacity)
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)c->res_count,
                   (unsigned long long)capacity);
  if (c->res_count == 0) return FAST_LSH_OK;
  if (!oi || !oj || !ov) return fl_fail(FAST_LSH_E_INVALID, "output pointer is NULL");
  HIPCK(hipSetDevice(c->device));
  launch_split_out(static_cast<uint64_t*>(c->ws["res_k0"].p), static_cast<uint32_t*>(c->ws["res_v0"].p),
                   c->res_count, oi, oj, ov, static_cast<uint64_t*>(c->ws["station_base"].p), c->res_stations,
                   c->stream);
  LAUNCHCK();
  HIPCK(hipStreamSynchronize(c->stream));
  return FAST_LSH_OK;
}

int fast_lsh_search_batched(fast_lsh_ctx* c, const fast_lsh_hash* h, uint32_t n_stations,
                            const fast_lsh_fps* stations, const fast_lsh_filter* flt, uint32_t flags,
                            uint32_t* oi, uint32_t* oj, uint8_t* ov, uint64_t capacity, uint64_t* station_offsets,
                            fast_lsh_stats* per_station) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  RC(fl_check_hash(h));
  RC(check_filter(flt, flags));
  if (n_stations < 1 || n_stations > FAST_LSH_MAX_STATIONS)
    return fl_fail(FAST_LSH_E_INVALID, "n_stations %u outside [1, %d]", n_stations, FAST_LSH_MAX_STATIONS);
  if (!stations) return fl_fail(FAST_LSH_E_INVALID, "stations is NULL");
  uint64_t total = 0;
  for (uint32_t st = 0; st < n_stations; ++st) {
    RC(fl_check_fps(&stations[st]));
    total += stations[st].n;
  }
  if (total >= (1ull << 31))
    return fl_fail(FAST_LSH_E_INVALID, "total n = %llu must be below 2^31", (unsigned long long)total);
  if (n_stations > 1 && (uint64_t)fl_key_bits(h->dim) * h->band_rows > 60)
    return fl_fail(FAST_LSH_E_INVALID, "band key of %u bits leaves no room for the station tag (at most 60)",
                   fl_key_bits(h->dim) * h->band_rows);
  HIPCK(hipSetDevice(c->device));
  std::vector<fast_lsh_stats> local(n_stations);
  RC(fl_search_stations(c, h, n_stations, stations, flt, flags, local.data(), station_offsets));
  if (per_station) std::copy(local.begin(), local.end(), per_station);
  if (c->res_count > capacity)
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)c->res_count,
                   (unsigned long long)capacity);
  return fast_lsh_copy_result(c, oi, oj, ov, capacity);
}

int fast_lsh_search_ex(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f, const fast_lsh_filter* flt,
                       uint32_t flags, uint32_t* oi, uint32_t* oj, uint8_t* ov, uint64_t capacity,
                       fast_lsh_stats* st) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  RC(fl_check_hash(h));
  RC(fl_check_fps(f));
  RC(check_filter(flt, flags));
  HIPCK(hipSetDevice(c->device));
  fast_lsh_stats local;
  RC(fl_search_stations(c, h, 1, f, flt, flags, &local, nullptr));
  if (st) *st = local;
  if (local.n_out > capacity)
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)local.n_out,
                   (unsigned long long)capacity);
  return fast_lsh_copy_result(c, oi, oj, ov, capacity);
}

int fast_lsh_search_bounded(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f,
                            const fast_lsh_filter* flt, uint32_t flags, uint32_t group_tables, uint32_t* oi,
                            uint32_t* oj, uint8_t* ov, uint64_t capacity, fast_lsh_stats* st) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  RC(fl_check_hash(h));
  RC(fl_check_fps(f));
  RC(check_filter(flt, flags));
  if (flags & FAST_LSH_USE_GRAPH) return fl_fail(FAST_LSH_E_INVALID, "the bounded search is not captured as a graph");
  if (group_tables < 1) return fl_fail(FAST_LSH_E_INVALID, "group_tables must be >= 1");
  if ((uint64_t)fl_key_bits(h->dim) * h->band_rows > 48)
    return fl_fail(FAST_LSH_E_INVALID, "the bounded search needs band keys of at most 48 bits (got %u)",
                   fl_key_bits(h->dim) * h->band_rows);
  HIPCK(hipSetDevice(c->device));
  fast_lsh_stats local;
  RC(fl_search_bounded(c, h, f, flt, flags, group_tables, &local));
  if (st) *st = local;
  if (local.n_out > capacity)
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)local.n_out,
                   (unsigned long long)capacity);
  return fast_lsh_copy_result(c, oi, oj, ov, capacity);
}

int fast_lsh_search_partitioned(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f,
                                const fast_lsh_filter* flt, uint32_t flags, uint32_t n_partitions, uint32_t* oi,
                                uint32_t* oj, uint8_t* ov, uint64_t capacity, fast_lsh_stats* st) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  RC(fl_check_hash(h));
  RC(fl_check_fps(f));
  RC(check_filter(flt, flags));
  if (flags & FAST_LSH_USE_GRAPH) return fl_fail(FAST_LSH_E_INVALID, "the partitioned search is not captured as a graph");
  if (n_partitions < 1) return fl_fail(FAST_LSH_E_INVALID, "n_partitions must be >= 1");
  HIPCK(hipSetDevice(c->device));
  fast_lsh_stats local;
  RC(fl_search_stations(c, h, 1, f, flt, flags, &local, nullptr, (uint32_t)std::min<uint64_t>(n_partitions,
                                                                                               std::max<uint64_t>(f->n, 1))));
  if (st) *st = local;
  if (local.n_out > capacity)
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)local.n_out,
                   (unsigned long long)capacity);
  return fast_lsh_copy_result(c, oi, oj, ov, capacity);
}

int fast_lsh_search(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f, const fast_lsh_filter* flt,
                    uint32_t* oi, uint32_t* oj, uint8_t* ov, uint64_t capacity, fast_lsh_stats* st) {
  return fast_lsh_search_ex(c, h, f, flt, 0, oi, oj, ov, capacity, st);
}

}  // extern "C"
