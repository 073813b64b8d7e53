// Candidate pairs and votes (section 6.1 "Search"; section 7.1 self-match
// exclusion; section 6.5 occurrence filter; section 6.3 "at least m of t").
//
// The search never builds a global (i, j) -> votes map.  Every in-bucket pair
// of table u is checked where it is found: each fingerprint carries a row of
// 16-bit sub-keys (low bits of the mixed band key), one per table, split into
// G contiguous table groups.  A pair with at least v votes shares buckets in
// at least need = ceil(v / G) tables of some group (pigeonhole), so table u
// only has to compare the sub-keys of its own group; equal band keys always
// have equal sub-keys, so a pair below `need` there cannot be the pair's
// reporting table and is dropped exactly.  The rare survivors compute the
// exact shared-table set S from the full mixed keys and are reported only
// by their owner: the smallest table of the first group holding at least
// `need` tables of S.  Every qualifying pair is therefore reported once,
// with its exact vote count |S|, and no atomics are spent on votes.
#include <algorithm>

#include "common.hpp"
#include "host.hpp"

namespace fl {

constexpr int kPT = 256;

__device__ __forceinline__ void tri_decode(uint32_t m, uint32_t q, uint32_t& x, uint32_t& y) {
  // Row x of the upper triangle holds m-1-x pairs; S(x) = x*m - x(x+1)/2 precede it.
  const float fm = 2.0f * (float)m - 1.0f;
  const float disc = fm * fm - 8.0f * (float)q;
  int xx = (int)((fm - sqrtf(fmaxf(disc, 0.0f))) * 0.5f);
  const int top = (int)m - 2;
  xx = xx < 0 ? 0 : (xx > top ? top : xx);
  auto S = [m](int r) { return (uint32_t)r * m - (uint32_t)(r * (r + 1) / 2); };
  while (xx > 0 && S(xx) > q) --xx;
  while (xx < top && S(xx + 1) <= q) ++xx;
  x = (uint32_t)xx;
  y = q - S(xx) + (uint32_t)xx + 1;
}

// Band keys of i and j in table tab are equal (their sub-keys are equal).
__device__ __forceinline__ bool keys_equal(const PairArgs& a, uint32_t tab, uint32_t i, uint32_t j) {
  const uint64_t o = (uint64_t)tab * a.n;
  return a.hi32 ? a.hi32[o + i] == a.hi32[o + j] : a.mkeys[o + i] == a.mkeys[o + j];
}

// Bit k: fields f0 + k of rows ri and rj (nd <= 16 dwords from dword f0 / 2)
// hold equal sub-keys.
__device__ __forceinline__ uint32_t field_eq_mask(const uint32_t* ri, const uint32_t* rj, uint32_t nd) {
  uint32_t m = 0;
#pragma unroll 4
  for (uint32_t d = 0; d < nd; ++d) {
    const uint32_t x = ri[d] ^ rj[d];
    m |= ((x & 0xFFFFu) == 0 ? 1u : 0u) << (2 * d);
    m |= ((x >> 16) == 0 ? 1u : 0u) << (2 * d + 1);
  }
  return m;
}

// Tables tb + k (bit k of m, lowest first) whose full keys of i and j are
// equal, counted until `limit`; the keys of four candidates are read at once.
__device__ __forceinline__ uint32_t count_shared(const PairArgs& a, uint32_t m, uint32_t tb, uint32_t i, uint32_t j,
                                                 uint32_t limit) {
  uint32_t cnt = 0;
  while (m && cnt < limit) {
    uint32_t tab[4];
    bool live[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      live[q] = m != 0;
      tab[q] = tb + (live[q] ? (uint32_t)__builtin_ctz(m) : 0u);  // a dead slot re-reads table tb
      m &= m - 1;
    }
    bool eq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) eq[q] = keys_equal(a, tab[q], i, j);
#pragma unroll
    for (int q = 0; q < 4; ++q) cnt += (live[q] && eq[q] && cnt < limit) ? 1u : 0u;
  }
  return cnt;
}

// Shared tables among the first `fields` tables of rows ri / rj's group
// (its first table tb), counted until `limit`: candidates are the fields
// with equal sub-keys, the full keys decide.
__device__ __forceinline__ uint32_t group_shared(const PairArgs& a, const uint32_t* ri, const uint32_t* rj, uint32_t tb,
                                                 uint32_t i, uint32_t j, uint32_t fields, uint32_t limit) {
  uint32_t cnt = 0;
  for (uint32_t f0 = 0; f0 < fields && cnt < limit; f0 += 32) {
    uint32_t m = field_eq_mask(ri + f0 / 2, rj + f0 / 2, min(16u, (fields - f0 + 1) / 2));
    if (fields - f0 < 32) m &= (1u << (fields - f0)) - 1;
    cnt += count_shared(a, m, tb + f0, i, j, limit - cnt);
  }
  return cnt;
}

// Owner rule: a pair is reported by the smallest shared table of the first
// group holding at least `need` shared tables, with its exact vote count.
// Called for table u after lower_in_group found no shared table below u in
// u's group, so u owns the pair exactly when no earlier group holds `need`
// shared tables and u's group does.  An earlier group stops being counted
// (and the check ends) as soon as it reaches `need`.
__device__ void exact_and_report(const PairArgs& a, uint32_t u, uint32_t i, uint32_t j) {
  const uint32_t gu = u / a.tables_per_group;
  uint32_t votes = 0;
  for (uint32_t g = 0; g < a.G; ++g) {
    const uint32_t fields = min(a.tables_per_group, a.t - g * a.tables_per_group);
    const uint32_t* ri = a.rows + ((uint64_t)g * a.n + i) * a.row_pitch;
    const uint32_t* rj = a.rows + ((uint64_t)g * a.n + j) * a.row_pitch;
    const uint32_t cnt = group_shared(a, ri, rj, g * a.tables_per_group, i, j, fields, g < gu ? a.need : 0xFFFFFFFFu);
    if (g < gu && cnt >= a.need) return;   // the owner lies in group g
    if (g == gu && cnt < a.need) return;   // the owner, if any, lies in a later group
    votes += cnt;
  }
  if (votes >= a.min_votes) {
    const uint32_t q = atomicAdd(a.out_count, 1u);
    if (q < a.out_cap) {
      a.out_i[q] = i;
      a.out_j[q] = j;
      a.out_v[q] = (uint8_t)votes;
    }
  }
}

// Some table of u's group below u exactly shares a bucket with (i, j);
// rl, rr: the two rows of that group (in LDS).  Such a table precedes u in
// the pair's shared set within the group, so u cannot own the pair, and with
// one group holding every table u is then not the pair's first shared table.
// A pair sharing s tables thus gets its full check (reading every group)
// only from the smallest shared table of each group, not from all s.
__device__ __forceinline__ bool lower_in_group(const PairArgs& a, uint32_t u, uint32_t i, uint32_t j,
                                               const uint32_t* rl, const uint32_t* rr) {
  const uint32_t g = u / a.tables_per_group, own = u - g * a.tables_per_group;
  return group_shared(a, rl, rr, g * a.tables_per_group, i, j, own, 1) != 0;
}

// Some table of u's group above u exactly shares a bucket with (i, j); rl,
// rr: the pair's rows of that group (in LDS).  With need == 2 and no lower
// table of the group sharing, u can own the pair only if one does: a pair
// whose sub-keys agree by chance is then turned away after one key check,
// without the owner check's reads of the other groups' rows.
__device__ __forceinline__ bool upper_in_group(const PairArgs& a, uint32_t u, uint32_t i, uint32_t j,
                                               const uint32_t* rl, const uint32_t* rr) {
  const uint32_t g = u / a.tables_per_group, own = u - g * a.tables_per_group;
  const uint32_t tb = g * a.tables_per_group;
  const uint32_t fields = min(a.tables_per_group, a.t - tb);
  for (uint32_t f0 = (own + 1) & ~31u; f0 < fields; f0 += 32) {
    uint32_t m = field_eq_mask(rl + f0 / 2, rr + f0 / 2, min(16u, (fields - f0 + 1) / 2));
    if (fields - f0 < 32) m &= (1u << (fields - f0)) - 1;
    if (f0 <= own) m &= ~((2u << (own - f0)) - 1u);  // fields f0 .. own dropped
    if (count_shared(a, m, tb + f0, i, j, 1) != 0) return true;
  }
  return false;
}

// The exact checks of a pair (i < j) of table u's bucket whose sub-keys
// passed the group test (need == 2): u owns it only if no lower table of
// u's group shares a bucket with it and some higher one does; the owner
// check then settles the earlier groups and the votes.  rl, rr: the pair's
// rows of u's group (in LDS or in memory).
__device__ __forceinline__ void check_candidate(const PairArgs& a, uint32_t u, uint32_t i, uint32_t j,
                                                const uint32_t* rl, const uint32_t* rr) {
  if (!lower_in_group(a, u, i, j, rl, rr) && upper_in_group(a, u, i, j, rl, rr)) exact_and_report(a, u, i, j);
}

// Appends the calling lane's candidate (want) of chunk blk to the queue of
// the workgroup's spread slot: one atomic per wavefront for all its active
// lanes that want to.  False when the slot is full.
__device__ __forceinline__ bool enqueue_candidate(const PairArgs& a, bool want, uint32_t u, uint32_t i, uint32_t j,
                                                  uint32_t blk) {
  const uint64_t m = __ballot(want);
  if (m == 0) return true;
  // (the lane's own bit is read back from the ballot, so that `want` stays a
  // lane mask and is never spilled to a vector register)
  const uint32_t lane = threadIdx.x & 63, lead = (uint32_t)__ffsll((long long)m) - 1;
  const uint32_t slot = spread_slot();
  uint32_t base = 0;
  if (lane == lead) base = atomicAdd(a.q_count + slot, (unsigned int)__popcll(m));
  base = __shfl(base, lead, 64);
  if (((m >> lane) & 1u) == 0) return true;
  const uint32_t q = base + (uint32_t)__popcll(m & __lanemask_lt());
  if (q >= a.qcap) return false;
  a.q[(uint64_t)slot * a.qcap + q] = make_uint4(i, j, u, blk);
  return true;
}

// Per-lane vote tallies of one station; [lo, hi) is that station's id range
// (looked up again only when a pair falls outside it).
struct PairTally {
  unsigned long long ev, nd;
  uint32_t station;
  uint32_t lo, hi;
  uint32_t blk = 0;  // the lane's chunk (tiled: unit), for the candidate queue
};

constexpr uint32_t kDead = 0xFFFFFFFFu;  // member excluded by the occurrence filter

// Resident one-wave workgroups per CU for the small-bucket kernel: its
// register limit (four waves per SIMD at 113 VGPRs).
constexpr uint32_t kPairWavesPerCU = 16;

// Row of sub-keys of one member of table u's group.  RSW > 0: the row length
// is a compile-time constant and the left row of a pair lives in registers;
// RSW == 0: runtime length, both rows read from LDS.
template <int RSW>
struct RowReg {
  static constexpr int kW = RSW > 0 ? RSW : 1;
  uint32_t w[kW];
  const uint32_t* lds;
  __device__ __forceinline__ void load(const uint32_t* src, uint32_t rsw) {
    if (RSW > 0) {
#pragma unroll
      for (int k = 0; k < kW; ++k) w[k] = src[k];
    } else {
      lds = src;
    }
    (void)rsw;
  }
  // Number of equal 16-bit sub-keys against another row.  RSW > 0: the
  // unequal ones are counted in packed halves (min(a ^ b, 1) is 0 for an
  // equal field, 1 otherwise), two fields per instruction.
  __device__ __forceinline__ uint32_t eq(const uint32_t* other, uint32_t rsw) const {
    if (RSW > 0) {
      typedef unsigned short half2 __attribute__((ext_vector_type(2)));
      const half2 one = {1, 1};
      half2 ne = {0, 0};
#pragma unroll
      for (int k = 0; k < kW; ++k) ne += __builtin_elementwise_min(__builtin_bit_cast(half2, w[k] ^ other[k]), one);
      return 2u * kW - ((uint32_t)ne.x + (uint32_t)ne.y);
    }
    uint32_t e = 0;
#pragma unroll 4
    for (uint32_t k = 0; k < rsw; ++k) e += eq2(lds[k], other[k]);
    return e;
  }
  __device__ __forceinline__ static uint32_t eq2(uint32_t a, uint32_t b) {
    return (uint32_t)((uint16_t)a == (uint16_t)b) + (uint32_t)((a >> 16) == (b >> 16));
  }
  // Non-zero when some sub-key in a field below `u` is equal (one group
  // holding every table).  RSW > 0: the fields at or above u are forced
  // unequal by a mask (u is uniform over the wave, so the masks are scalar)
  // and the packed minimum of a ^ b over the row finds a zero half.
  __device__ __forceinline__ uint32_t eq_below(const uint32_t* other, uint32_t rsw, uint32_t u) const {
    (void)rsw;
    if (RSW > 0) {
      typedef unsigned short half2 __attribute__((ext_vector_type(2)));
      half2 acc = {0xFFFF, 0xFFFF};
#pragma unroll
      for (int k = 0; k < kW; ++k) {
        const uint32_t m = (2u * k >= u ? 0x0000FFFFu : 0u) | (2u * k + 1 >= u ? 0xFFFF0000u : 0u);
        acc = __builtin_elementwise_min(acc, __builtin_bit_cast(half2, (w[k] ^ other[k]) | m));
      }
      return (uint32_t)(acc.x == 0) + (uint32_t)(acc.y == 0);
    }
    uint32_t e = 0;
    for (uint32_t f = 0; f < u; ++f) e += row_field(lds, f) == row_field(other, f);
    return e;
  }
  // Left row for the "another table shares the bucket" test (RSW > 0): the
  // field of the pair's own table (equal for every pair of its bucket) and
  // the padding fields (zero in every row) are inverted, so they never
  // compare equal.
  __device__ __forceinline__ void load_masked(const uint32_t* src, uint32_t own, uint32_t valid) {
#pragma unroll
    for (int k = 0; k < kW; ++k) {
      const uint32_t f = 2u * k;
      const uint32_t m = ((f == own || f >= valid) ? 0x0000FFFFu : 0u) |
                         ((f + 1 == own || f + 1 >= valid) ? 0xFFFF0000u : 0u);
      w[k] = src[k] ^ m;
    }
  }
  // The other row in registers (all loads issued at once).
  __device__ __forceinline__ static void fetch(const uint32_t* src, uint32_t (&v)[kW]) {
#pragma unroll
    for (int k = 0; k < kW; ++k) v[k] = src[k];
  }
  // Some field equal to the other row's (after load_masked): the unsigned
  // minimum of the 16-bit halves of a ^ b over the row (packed, two halves
  // per instruction) is zero exactly when a half is zero.
  __device__ __forceinline__ bool any_equal(const uint32_t* other) const {
    typedef unsigned short half2 __attribute__((ext_vector_type(2)));
    half2 acc = {0xFFFF, 0xFFFF};
#pragma unroll
    for (int k = 0; k < kW; ++k) acc = __builtin_elementwise_min(acc, __builtin_bit_cast(half2, w[k] ^ other[k]));
    // a zero half: (v - 0x00010001) & ~v has bit 15 or 31 set exactly when
    // some half is zero (a borrow out of a zero low half can only touch the
    // high half's test, and then the low half already answers)
    const uint32_t v = __builtin_bit_cast(uint32_t, acc);
    return ((v - 0x00010001u) & ~v & 0x80008000u) != 0u;
  }
};

// One in-bucket pair of table u: i < j, `rl` and `ry` the rows of i and j
// in LDS; `rx` holds one of the two rows in registers and `ro` is the other
// one (in LDS).
// FAST (need == 2, no distinct count, rx from load_masked): the group test
// is "some other table of the group shares a bucket", decided without
// counting; otherwise the equal fields are counted.  QUEUE (FAST only): a
// pair that passes the group test goes to the candidate queue.
template <int RSW, bool FAST, bool QUEUE>
__device__ __forceinline__ void visit_pair(const PairArgs& a, uint32_t u, uint32_t i, uint32_t j,
                                           const RowReg<RSW>& rx, const uint32_t* rl, const uint32_t* ry,
                                           const uint32_t* ro, uint32_t rsw, uint32_t pad, PairTally& tl) {
  // FAST: the right row is read before the id checks, so that its loads and
  // the partner id's share one LDS round trip
  uint32_t rv[RowReg<RSW>::kW];
  if (FAST) {
    RowReg<RSW>::fetch(ro, rv);
#pragma unroll
    for (int k = 0; k < RowReg<RSW>::kW; ++k) asm volatile("" : "+v"(rv[k]));  // keep the loads above the branch
  }
  if (i == kDead || j == kDead || j - i < a.min_lag) return;
  if (a.part_mode == 3 && (i < a.plo || i >= a.phi)) return;  // pairs of the partitions reported
  if (!FAST && (a.part_mode == 1 || a.part_mode == 2)) {
    // partitioned search: counts and exclusions at the pair's first shared
    // table only, tested after the cheaper checks that can skip the pair
    if (a.part_mode == 1) {
      const bool ii = i >= a.plo && i < a.phi, jj = j >= a.plo && j < a.phi;
      if (!(ii || jj)) return;
      if (rx.eq_below(ro, rsw, u) != 0 && lower_in_group(a, u, i, j, rl, ry)) return;
      if (ii) atomicAdd(a.cand + i, 1u);
      if (jj) atomicAdd(a.cand + j, 1u);
      return;
    }
    const bool fi = a.fp[i] != 0, fj = a.fp[j] != 0;
    if (fi == fj) return;
    if (rx.eq_below(ro, rsw, u) != 0 && lower_in_group(a, u, i, j, rl, ry)) return;
    a.ex_next[fi ? j : i] = 1;
    return;
  }
  if (a.nstation > 1 && (i < tl.lo || i >= tl.hi)) {
    const uint32_t st = station_of(a.station_base, a.nstation, i);
    if (st != tl.station) {
      const uint64_t o = (uint64_t)tl.station * kSpread + spread_slot();
      if (tl.ev) atomicAdd(a.e_voted + o, tl.ev);
      if (tl.nd) atomicAdd(a.n_distinct + o, tl.nd);
      tl.ev = tl.nd = 0;
      tl.station = st;
    }
    tl.lo = (uint32_t)a.station_base[st];
    tl.hi = (uint32_t)a.station_base[st + 1];
  }
  ++tl.ev;
  if (!FAST && a.part_mode == 4) {
    // partitioned search, every partition counted and reported in one pass
    // (valid while no partition excludes): at its first shared table the
    // pair adds one to both members' counts, and it is reported as in the
    // plain search
    const bool lower = rx.eq_below(ro, rsw, u) != 0 && lower_in_group(a, u, i, j, rl, ry);
    if (lower) return;
    atomicAdd(a.cand + i, 1u);
    atomicAdd(a.cand + j, 1u);
    if (a.want_distinct) ++tl.nd;
    if (rx.eq(ro, rsw) - pad >= a.need) exact_and_report(a, u, i, j);
    return;
  }
  if (FAST) {
    const bool cand = rx.any_equal(rv);
    if (QUEUE) {
      // (no checks in place here: they would cost the loop registers)
      if (!enqueue_candidate(a, cand, u, i, j, tl.blk)) {
        a.q_ovf[tl.blk] = 1;
        *a.q_any = 1;
      }
    } else if (cand) {
      check_candidate(a, u, i, j, rl, ry);
    }
    return;
  }
  const uint32_t eq = rx.eq(ro, rsw);
  if (a.want_distinct) {  // one group: "lower" is "a table below u shares"
    const bool lower = rx.eq_below(ro, rsw, u) != 0 && lower_in_group(a, u, i, j, rl, ry);
    if (!lower) {
      ++tl.nd;
      if (eq - pad >= a.need) exact_and_report(a, u, i, j);
    }
    return;
  }
  if (eq - pad >= a.need && !lower_in_group(a, u, i, j, rl, ry)) exact_and_report(a, u, i, j);
}

// Called by every lane of the wave.  When all lanes with a non-zero tally
// hold one station the tallies are summed over the wave first; at a station
// boundary each lane adds its own.
__device__ void flush_tally(const PairArgs& a, PairTally tl) {
  const bool live = (tl.ev | tl.nd) != 0;
  const uint64_t act = __ballot(live);
  if (act == 0) return;
  const uint32_t s0 = __shfl(tl.station, __ffsll((long long)act) - 1, 64);
  if (!__all(!live || tl.station == s0)) {
    if (!live) return;
    const uint64_t o = (uint64_t)tl.station * kSpread + spread_slot();
    if (tl.ev) atomicAdd(a.e_voted + o, tl.ev);
    if (tl.nd) atomicAdd(a.n_distinct + o, tl.nd);
    if (tl.ev && a.big_voted) atomicAdd(a.big_voted + spread_slot(), tl.ev);
    return;
  }
  unsigned long long ev = tl.ev, nd = tl.nd;
  for (int o = 32; o > 0; o >>= 1) {
    ev += __shfl_xor(ev, o, 64);
    nd += __shfl_xor(nd, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    const uint64_t o = (uint64_t)s0 * kSpread + spread_slot();
    if (ev) atomicAdd(a.e_voted + o, ev);
    if (nd) atomicAdd(a.n_distinct + o, nd);
    if (ev && a.big_voted) atomicAdd(a.big_voted + spread_slot(), ev);
  }
}

template <typename T>
__device__ __forceinline__ T block_scan_excl(T v, T* ws, T* total) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  T inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += y;
  }
  if (lane == 63) ws[wave] = inc;
  __syncthreads();
  T add = 0, all = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) {
    if (w < wave) add += ws[w];
    all += ws[w];
  }
  __syncthreads();
  *total = all;
  return add + inc - v;
}

// Copy one row of sub-keys from HBM into LDS; with a compile-time length all
// its loads are issued before the first store.
template <int RSW>
__device__ __forceinline__ void stage_row(const uint32_t* src, uint32_t* dst, uint32_t rsw) {
  if (RSW > 0) {
    uint32_t v[RSW > 0 ? RSW : 1];
#pragma unroll
    for (int w = 0; w < (RSW > 0 ? RSW : 1); ++w) v[w] = src[w];
#pragma unroll
    for (int w = 0; w < (RSW > 0 ? RSW : 1); ++w) dst[w] = v[w];
  } else {
    uint32_t w = 0;
    for (; w + 4 <= rsw; w += 4) {
      const uint32_t v0 = src[w], v1 = src[w + 1], v2 = src[w + 2], v3 = src[w + 3];
      dst[w] = v0;
      dst[w + 1] = v1;
      dst[w + 2] = v2;
      dst[w + 3] = v3;
    }
    for (; w < rsw; ++w) dst[w] = src[w];
  }
}

// Last index b in [0, cnt) with arr[b] <= key (arr ascending, arr[0] <= key).
__device__ __forceinline__ uint32_t last_le(const uint32_t* arr, uint32_t cnt, uint32_t key) {
  uint32_t L = 0, R = cnt;
  while (R - L > 1) {
    const uint32_t M = (L + R) / 2;
    if (arr[M] <= key) L = M; else R = M;
  }
  return L;
}

// Fields of table u's group row that hold no table (zero in every row, so
// always equal).
__device__ __forceinline__ uint32_t group_pad(const PairArgs& a, uint32_t u, uint32_t rsw) {
  const uint32_t g = u / a.tables_per_group;
  const uint32_t valid = min(a.tables_per_group, a.t - g * a.tables_per_group);
  return row_fields(rsw) - valid;
}

// Small buckets of one table, in chunks of 64 positions: a chunk holds the
// buckets that start in its positions (a bucket marked at position q holds
// the ids at positions q .. q+size-1).  One-wave workgroups stay resident
// and walk the chunks of their segment with a stride of the grid width; the
// marks and ids of a wave's next chunk are loaded before the current one is
// processed, so they arrive while its rows load and its pairs run.  The
// member rows are staged in LDS with each lane issuing a whole row's loads at
// once, and every lane then walks a contiguous range of the chunk's pairs
// (row-major within each bucket) with the left row in registers.  Heads and
// pair offsets come from ballots and lane shuffles, so the only barriers are
// the LDS hand-offs of a single wave.
template <int RSW, bool FAST, bool QUEUE>
__global__ __launch_bounds__(64) void k_pairs_wave(PairArgs a, const uint8_t* marks_all, uint32_t rswl,
                                                   uint32_t nchunk, uint32_t span) {
  // span = 64 + small_max - 1: heads in 64 positions, members up to small_max
  // (at most kSmallBucket) after them
  extern __shared__ uint32_t smem[];
  uint32_t* lrows = smem;                   // span * rswl
  uint32_t* lids = lrows + span * rswl;     // span
  uint32_t* hinfo = lids + span;            // 64: head position | size << 16
  uint32_t* bpof = hinfo + 64;              // 65: pair prefix
  const uint32_t lane = threadIdx.x;
  const uint32_t rsw = RSW > 0 ? (uint32_t)RSW : a.row_dw;
  const uint32_t seg = blockIdx.y;           // launch segment (positions in order/marks)
  const uint32_t u = seg + a.table_offset;    // its table
  const uint8_t* marks = marks_all + (uint64_t)seg * a.n;
  const uint32_t* order = a.order + (uint64_t)seg * a.n;
  const bool use_flags = *a.n_flagged != 0;
  const uint32_t g = u / a.tables_per_group;
  const uint32_t* R = a.rows + (uint64_t)g * a.n * a.row_pitch;
  const uint32_t pad = group_pad(a, u, rsw);
  const uint32_t own = u % a.tables_per_group, valid = row_fields(rsw) - pad;
  // Tallies of the wave's station; with several stations the empty range
  // makes the first pair look its station up.
  PairTally tl{0ull, 0ull, 0u, 0u, a.nstation > 1 ? 0u : 0xFFFFFFFFu};

  // The chunk's marks and ids (span positions, clipped at n).
  uint32_t nsize = 0, nid0 = 0, nid1 = 0;
  auto fetch = [&](uint32_t c) {
    const uint64_t p0 = (uint64_t)c * 64;
    const uint64_t left = a.n - p0;
    nsize = lane < left ? marks[p0 + lane] : 0u;
    nid0 = lane < left ? order[p0 + lane] : 0u;
    nid1 = (64 + lane < left && lane < span - 64) ? order[p0 + 64 + lane] : 0u;
  };
  uint32_t c = blockIdx.x;
  if (c < nchunk) fetch(c);
  for (; c < nchunk; c += gridDim.x) {
    const uint32_t size = nsize, id0 = nid0, id1 = nid1;
    if (c + gridDim.x < nchunk) fetch(c + gridDim.x);
    tl.blk = seg * nchunk + c;  // (the host keeps S * nchunk below 2^32 when queueing)
    if (a.redo && !a.q_ovf[tl.blk]) continue;  // a second run takes the marked chunks only
    const uint64_t heads = __ballot(size != 0);
    if (heads == 0) continue;
    __syncthreads();  // the previous chunk's LDS reads are complete
    lids[lane] = id0;
    if (lane < span - 64) lids[64 + lane] = id1;
    const uint64_t lt = __lanemask_lt();
    const uint32_t hidx = __popcll(heads & lt);
    const uint32_t nh = __popcll(heads);
    const uint32_t pc = size * (size - (size > 0)) / 2;
    uint32_t inc = pc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, 64);
      if (lane >= (uint32_t)o) inc += y;
    }
    const uint32_t P = __shfl(inc, 63, 64);
    if (size) {
      hinfo[hidx] = lane | (size << 16);
      bpof[hidx] = inc - pc;
    }
    if (lane == 0) bpof[nh] = P;
    __syncthreads();
    // Member positions: q belongs to the last head h <= q when q < h + size(h).
    bool mem[2];
    uint32_t mid[2];
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
      const uint32_t q = lane + 64 * r;
      const uint64_t upto = q >= 63 ? heads : (heads & ((2ull << q) - 1));
      const uint32_t h = upto ? 63 - (uint32_t)__clzll(upto) : 0u;
      const uint32_t hs = __shfl(size, h, 64);  // every lane active here
      mem[r] = upto && q < span && q < h + hs;
      mid[r] = mem[r] ? lids[q] : 0u;
    }
    if (RSW > 0 && RSW <= 32) {  // both rows' loads (each only where that member exists) before either store
      constexpr int kW = RSW > 0 ? RSW : 1;
      uint32_t v0[kW], v1[kW];
      if (mem[0]) RowReg<RSW>::fetch(R + (uint64_t)mid[0] * a.row_pitch, v0);
      if (mem[1]) RowReg<RSW>::fetch(R + (uint64_t)mid[1] * a.row_pitch, v1);
      if (mem[0])
#pragma unroll
        for (int w = 0; w < kW; ++w) lrows[lane * rswl + w] = v0[w];
      if (mem[1])
#pragma unroll
        for (int w = 0; w < kW; ++w) lrows[(lane + 64) * rswl + w] = v1[w];
    } else {
#pragma unroll
      for (uint32_t r = 0; r < 2; ++r)
        if (mem[r]) stage_row<RSW>(R + (uint64_t)mid[r] * a.row_pitch, lrows + (lane + 64 * r) * rswl, rsw);
    }
    if (use_flags) {
#pragma unroll
      for (uint32_t r = 0; r < 2; ++r)
        if (mem[r] && a.flags[mid[r]]) lids[lane + 64 * r] = kDead;
    }
    __syncthreads();
    const uint32_t per = (P + 63) / 64;
    uint32_t p = lane * per;
    const uint32_t pend = min(P, p + per);
    if (p < pend) {
      uint32_t b = last_le(bpof, nh, p);
      uint32_t base = hinfo[b] & 0xFFFFu, m = hinfo[b] >> 16;
      uint32_t x, y;
      tri_decode(m, p - bpof[b], x, y);
      uint32_t idx = lids[base + x];
      RowReg<RSW> rx;
      const uint32_t* rl = lrows + (base + x) * rswl;
      const uint32_t* ry = lrows + (base + y) * rswl;  // stepped with y (no multiply per pair)
      if (FAST) rx.load_masked(rl, own, valid); else rx.load(rl, rsw);
      for (; p < pend; ++p) {
        visit_pair<RSW, FAST, QUEUE>(a, u, idx, lids[base + y], rx, rl, ry, ry, rsw, pad, tl);
        ry += rswl;
        if (++y == m) {
          if (++x == m - 1) {
            if (++b >= nh) break;
            base = hinfo[b] & 0xFFFFu;
            m = hinfo[b] >> 16;
            x = 0;
          }
          y = x + 1;
          idx = lids[base + x];
          rl = lrows + (base + x) * rswl;
          ry = rl + rswl;
          if (FAST) rx.load_masked(rl, own, valid); else rx.load(rl, rsw);
        }
      }
    }
  }
  flush_tally(a, tl);
}

// Tiles of each large bucket: the upper triangle, diagonal included, of its
// ceil(m / tb) x ceil(m / tb) grid of tb x tb tiles (m members; an empty
// descriptor has none).  Also adds the buckets' members and in-bucket pairs
// C(m, 2) to work[kSpread..2 kSpread) and work[2 kSpread..3 kSpread)
// (measurement counters, summed by k_work_reduce).
__global__ __launch_bounds__(kPT) void k_tile_counts(const uint4* big, uint32_t nbig, uint32_t tb, uint64_t* tiles,
                                                     unsigned long long* work) {
  const uint64_t b = (uint64_t)blockIdx.x * kPT + threadIdx.x;
  const uint64_t m = b < nbig ? big[b].z : 0;
  if (b < nbig) {
    const uint64_t ntl = (m + tb - 1) / tb;
    tiles[b] = m < 2 ? 0 : ntl * (ntl + 1) / 2;
  }
  unsigned long long mem = m < 2 ? 0 : m, cand = m < 2 ? 0 : m * (m - 1) / 2;
  for (int o = 32; o > 0; o >>= 1) {
    mem += __shfl_xor(mem, o, 64);
    cand += __shfl_xor(cand, o, 64);
  }
  if ((threadIdx.x & 63) == 0 && mem) {
    const uint32_t slot = spread_slot();
    atomicAdd(work + kSpread + slot, mem);
    atomicAdd(work + 2 * kSpread + slot, cand);
  }
}

// work[3][kSpread] summed into out[3] (one workgroup).
__global__ __launch_bounds__(kPT) void k_work_reduce(const unsigned long long* work, unsigned long long* out) {
  __shared__ unsigned long long part[3][kPT / 64];
  for (int f = 0; f < 3; ++f) {
    unsigned long long x = 0;
    for (uint32_t k = threadIdx.x; k < kSpread; k += kPT) x += work[f * kSpread + k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) part[f][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long x = 0;
    for (uint32_t w = 0; w < kPT / 64; ++w) x += part[threadIdx.x][w];
    out[threadIdx.x] = x;
  }
}

// The bucket of every tile unit: owner[q] = b for q in [toff[b], toff[b+1])
// (one wavefront per bucket, its lanes on consecutive units, the waves
// striding over the buckets: the largest bucket's million tiles take
// sixteen thousand stores of a wave instead of a million of one thread).
__global__ __launch_bounds__(kPT) void k_unit_owner(const uint64_t* toff, uint32_t nbig, uint32_t* owner) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t waves = gridDim.x * (kPT / 64);
  for (uint32_t b = blockIdx.x * (kPT / 64) + threadIdx.x / 64; b < nbig; b += waves)
    for (uint64_t q = toff[b] + lane, e = toff[b + 1]; q < e; q += 64) owner[q] = b;
}

// One tile (ta, tb) of the upper triangle of a large bucket's pair matrix.
// Workgroup unit_base + blockIdx.x takes bucket owner[unit] (whose tile range
// [toff[b], toff[b+1]) holds the unit) and within it the tile of that rank.
template <int RSW, bool FAST, bool QUEUE>
__global__ __launch_bounds__(kPT) void k_pairs_tile(PairArgs a, const uint64_t* toff, const uint32_t* owner,
                                                    uint64_t unit_base, const uint4* big, uint32_t tb_size,
                                                    uint32_t rswl) {
  extern __shared__ uint32_t smem[];
  // (units stay in launch order across the XCDs: contiguous unit ranges per
  // XCD balance badly, tiles of a range differing widely in cost)
  const uint64_t unit = unit_base + blockIdx.x;
  if (a.redo && !a.q_ovf[unit]) return;  // a second run takes the marked units only
  const uint32_t bk = owner[unit];
  const uint4 d = big[bk];  // {position, segment, members}
  const uint32_t m = d.z;
  const uint32_t ntl = (m + tb_size - 1) / tb_size;
  uint32_t tx, ty;
  tri_decode(ntl + 1, (uint32_t)(unit - toff[bk]), tx, ty);  // pairs x < y of ntl + 1 items: tile (x, y - 1)
  const uint32_t ta = tx, tbi = ty - 1;
  const uint32_t rsw = RSW > 0 ? (uint32_t)RSW : a.row_dw;
  const uint32_t u = d.y + a.table_offset;  // table of the bucket
  const uint32_t* bid = a.order + (uint64_t)d.y * a.n + d.x;  // members, ids ascending
  const uint32_t a0 = ta * tb_size, b0 = tbi * tb_size;
  const uint32_t na = min(tb_size, m - a0);
  const bool diag = ta == tbi;
  const uint32_t nbm = diag ? na : min(tb_size, m - b0);
  uint32_t* rowsA = smem;
  uint32_t* rowsB = diag ? rowsA : rowsA + tb_size * rswl;
  uint32_t* idsA = smem + 2 * tb_size * rswl;
  uint32_t* idsB = diag ? idsA : idsA + tb_size;
  const uint32_t g = u / a.tables_per_group;
  const uint32_t* R = a.rows + (uint64_t)g * a.n * a.row_pitch;
  // Each thread stages the rows of the ids it loads (no barrier between);
  // members excluded by the occurrence filter stay in place, marked dead.
  // B's members start half a block on, so that for tiles of up to kPT / 2
  // members every thread has one load chain.
  const bool use_flags = *a.n_flagged != 0;
  for (uint32_t q = threadIdx.x; q < na; q += kPT) {
    const uint32_t id = bid[a0 + q];
    stage_row<RSW>(R + (uint64_t)id * a.row_pitch, rowsA + q * rswl, rsw);
    idsA[q] = use_flags && a.flags[id] ? kDead : id;
  }
  if (!diag)
    for (uint32_t q = (threadIdx.x + kPT / 2) % kPT; q < nbm; q += kPT) {
      const uint32_t id = bid[b0 + q];
      stage_row<RSW>(R + (uint64_t)id * a.row_pitch, rowsB + q * rswl, rsw);
      idsB[q] = use_flags && a.flags[id] ? kDead : id;
    }
  __syncthreads();
  const uint32_t pad = group_pad(a, u, rsw);
  PairTally tl{0ull, 0ull, 0u, 0u, 0u};
  tl.blk = (uint32_t)unit;
  const uint32_t own = u % a.tables_per_group, valid = row_fields(rsw) - pad;
  if (!diag && tb_size == kPT / 2 && na > kPT / 4 && nbm >= 16) {
    // Full tiles off the diagonal: thread t holds left row t mod tb_size in
    // registers and takes the columns of parity t / tb_size; the lanes of a
    // wave share every column, so its id and row are one LDS broadcast.
    // (y0 is uniform over a wave: a scalar, so the column loop's control
    // stays off the vector unit)
    const uint32_t x = threadIdx.x % tb_size;
    const uint32_t y0 = __builtin_amdgcn_readfirstlane(threadIdx.x / tb_size);
    if (__ballot(x < na)) {
      const bool live = x < na;
      const uint32_t xs = live ? x : 0u;
      RowReg<RSW> rx;
      if (FAST) rx.load_masked(rowsA + xs * rswl, own, valid); else rx.load(rowsA + xs * rswl, rsw);
      const uint32_t idx = idsA[xs];
      const uint32_t* rowx = rowsA + xs * rswl;
      const uint32_t* rowy = rowsB + y0 * rswl;  // stepped with y (no multiply per pair)
      // A clean tile (one station, no member excluded anywhere, the plain
      // search, and B's smallest id at least min_lag above A's largest: ids
      // ascend within a bucket and B's follow A's) has every pair alive and
      // far enough apart, so the loop skips those checks and each lane adds
      // its pair count to the tally once.
      const bool clean = FAST && !use_flags && a.nstation == 1 && a.part_mode == 0 &&
                         idsB[0] - idsA[na - 1] >= a.min_lag;
      if (clean) {
        // (the partner's id is read only when some lane's pair passes the
        // sub-key test, which few do)
        for (uint32_t y = y0; y < nbm; y += 2, rowy += 2 * rswl)
          if (live) {
            uint32_t rv[RowReg<RSW>::kW];
            RowReg<RSW>::fetch(rowy, rv);
            const uint64_t m = __ballot(rx.any_equal(rv));
            if (m != 0) {
              const bool cand = ((m >> (threadIdx.x & 63)) & 1u) != 0;
              const uint32_t idy = idsB[y];
              if (QUEUE) {
                if (!enqueue_candidate(a, cand, u, idx, idy, tl.blk)) {
                  a.q_ovf[tl.blk] = 1;
                  *a.q_any = 1;
                }
              } else if (cand) {
                check_candidate(a, u, idx, idy, rowx, rowy);
              }
            }
          }
        if (live) tl.ev += (nbm - y0 + 1) / 2;
      } else {
        for (uint32_t y = y0; y < nbm; y += 2, rowy += 2 * rswl)
          if (live) visit_pair<RSW, FAST, QUEUE>(a, u, idx, idsB[y], rx, rowx, rowy, rowy, rsw, pad, tl);
      }
    }
  } else if (diag && tb_size == kPT / 2) {
    // Diagonal tiles: the pairs {x, (x + k) mod na} for k = 1 .. na / 2 are
    // each unordered pair once (for even na the round k = na / 2 meets
    // every pair twice and is taken from its smaller position only).
    // Thread t holds row x = t mod tb_size in registers and takes the rounds
    // of parity t / tb_size; in a round the wave's lanes read consecutive
    // rows (conflict-free at the odd row stride).
    // (the round parity is uniform over a wave: a scalar, so the loop
    // control stays off the vector unit)
    const uint32_t x = threadIdx.x % tb_size;
    const uint32_t k0 = 1 + __builtin_amdgcn_readfirstlane(threadIdx.x / tb_size);
    if (__ballot(x < na)) {
      const bool live = x < na;
      const uint32_t xs = live ? x : 0u;
      RowReg<RSW> rx;
      if (FAST) rx.load_masked(rowsA + xs * rswl, own, valid); else rx.load(rowsA + xs * rswl, rsw);
      const uint32_t idx = idsA[xs];
      const uint32_t* rowx = rowsA + xs * rswl;
      // y = (x + k) mod na and its row, stepped by two rows per round
      uint32_t y = xs + k0 < na ? xs + k0 : xs + k0 - na;
      const uint32_t* rowy = rowsA + y * rswl;
      // The plain search (FAST, one station, no member excluded): every pair
      // is alive, so the loop runs the sub-key test alone, and the lag test
      // and the partner's id wait for the few rounds in which some lane's
      // pair passes it.  The tally is exact without a per-pair count: the
      // threads of the first round parity add, for their row x, the pairs
      // {x, y > x} less those closer than min_lag (ids ascend within a
      // bucket, so those are the next few rows).
      const bool plain = FAST && !use_flags && a.nstation == 1 && a.part_mode == 0;
      if (plain) {
        if (live && k0 == 1) {
          uint32_t close = 0;
          for (uint32_t z = x + 1; z < na && idsA[z] - idx < a.min_lag; ++z) ++close;
          tl.ev += na - 1 - x - close;
        }
        // only y's row offset is carried (y itself is recovered in the rare
        // path); past the tile it wraps by an unsigned minimum, oy - span
        // being the smaller exactly when oy >= span
        uint32_t oy = y * rswl;
        const uint32_t span = na * rswl;
        for (uint32_t k = k0; 2 * k <= na; k += 2) {
          if (live) {
            const uint32_t* ry = rowsA + oy;
            uint32_t rv[RowReg<RSW>::kW];
            RowReg<RSW>::fetch(ry, rv);
            const uint64_t m = __ballot(rx.any_equal(rv));
            if (m != 0) {
              const uint32_t yy = oy / rswl;
              const uint32_t idy = idsA[yy];
              const bool fw = yy > x;
              const uint32_t i = fw ? idx : idy, j = fw ? idy : idx;
              const bool cand = ((m >> (threadIdx.x & 63)) & 1u) != 0 && j - i >= a.min_lag &&
                                !(2 * k == na && x >= k);
              if (QUEUE) {
                if (!enqueue_candidate(a, cand, u, i, j, tl.blk)) {
                  a.q_ovf[tl.blk] = 1;
                  *a.q_any = 1;
                }
              } else if (cand) {
                check_candidate(a, u, i, j, fw ? rowx : ry, fw ? ry : rowx);
              }
            }
          }
          oy += 2 * rswl;
          oy = min(oy, oy - span);
        }
      } else {
        for (uint32_t k = k0; 2 * k <= na; k += 2) {
          if (live && !(2 * k == na && x >= k)) {
            const uint32_t idy = idsA[y];
            const bool fw = y > x;  // selects, not branches: one inlined visit per lane
            visit_pair<RSW, FAST, QUEUE>(a, u, fw ? idx : idy, fw ? idy : idx, rx, fw ? rowx : rowy, fw ? rowy : rowx,
                                         rowy, rsw, pad, tl);
          }
          // next round: two rows on, wrapping past na (selects, no branch)
          y += 2;
          rowy += 2 * rswl;
          const bool wrap = y >= na;
          y = wrap ? y - na : y;
          rowy = wrap ? rowy - na * rswl : rowy;
        }
      }
    }
  } else {
    // Partial tiles: every thread walks a contiguous range of the tile's
    // pairs.
    const uint32_t P = diag ? na * (na - 1) / 2 : na * nbm;
    const uint32_t per = (P + kPT - 1) / kPT;
    uint32_t p = threadIdx.x * per;
    const uint32_t pend = min(P, p + per);
    if (p < pend) {
      uint32_t x, y;
      if (diag) {
        tri_decode(na, p, x, y);
      } else {
        x = p / nbm;
        y = p - x * nbm;
      }
      // rows and the left id follow x and y (no multiply per pair)
      const uint32_t* rl = rowsA + x * rswl;
      const uint32_t* ry = rowsB + y * rswl;
      uint32_t idx = idsA[x];
      RowReg<RSW> rx;
      if (FAST) rx.load_masked(rl, own, valid); else rx.load(rl, rsw);
      for (; p < pend; ++p) {
        visit_pair<RSW, FAST, QUEUE>(a, u, idx, idsB[y], rx, rl, ry, ry, rsw, pad, tl);
        ry += rswl;
        if (++y == nbm) {
          ++x;
          y = diag ? x + 1 : 0;
          if (x < na) {
            rl = rowsA + x * rswl;
            ry = rowsB + y * rswl;
            idx = idsA[x];
            if (FAST) rx.load_masked(rl, own, valid); else rx.load(rl, rsw);
          }
        }
      }
    }
  }
  flush_tally(a, tl);
}

// Split sorted (i << 32 | j, votes) records into the caller's arrays, ids
// made local to their station.
__global__ __launch_bounds__(kPT) void k_split_out(const uint64_t* key, const uint32_t* val, uint64_t count,
                                                   uint32_t* oi, uint32_t* oj, uint8_t* ov, const uint64_t* base,
                                                   uint32_t nb) {
  for (uint64_t e = (uint64_t)blockIdx.x * kPT + threadIdx.x; e < count; e += (uint64_t)gridDim.x * kPT) {
    const uint64_t k = key[e];
    const uint32_t i = (uint32_t)(k >> 32), j = (uint32_t)k;
    const uint32_t b = (uint32_t)base[station_of(base, nb, i)];
    oi[e] = i - b;
    oj[e] = j - b;
    ov[e] = (uint8_t)val[e];
  }
}

// Offsets of each station's pairs in the sorted records: the first record
// whose i is at or above the station's base.
__global__ void k_station_offsets(const uint64_t* key, uint64_t count, const uint64_t* base, uint32_t nb,
                                  unsigned long long* offs) {
  const uint32_t s = threadIdx.x;
  if (s > nb) return;
  const uint64_t target = base[s] << 32;
  uint64_t L = 0, R = count;
  while (L < R) {
    const uint64_t M = (L + R) / 2;
    if (key[M] >= target) R = M; else L = M + 1;
  }
  offs[s] = L;
}

__global__ __launch_bounds__(kPT) void k_pack_out(const uint32_t* oi, const uint32_t* oj, const uint8_t* ov,
                                                  uint64_t count, uint64_t* key, uint32_t* val) {
  for (uint64_t e = (uint64_t)blockIdx.x * kPT + threadIdx.x; e < count; e += (uint64_t)gridDim.x * kPT) {
    key[e] = ((uint64_t)oi[e] << 32) | oj[e];
    val[e] = ov[e];
  }
}

// Excluded fingerprints of one station (flags[0, n)): added to its counter
// and to the total.
__global__ __launch_bounds__(kPT) void k_count_flags(const uint8_t* flags, uint64_t n, unsigned long long* out,
                                                     unsigned long long* total) {
  unsigned long long c = 0;
  for (uint64_t e = (uint64_t)blockIdx.x * kPT + threadIdx.x; e < n; e += (uint64_t)gridDim.x * kPT) c += flags[e] != 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) {
    atomicAdd(out, c);
    atomicAdd(total, c);
  }
}

template <typename T>
__global__ __launch_bounds__(kPT) void k_fill(T* p, uint64_t count, T v) {
  for (uint64_t e = (uint64_t)blockIdx.x * kPT + threadIdx.x; e < count; e += (uint64_t)gridDim.x * kPT) p[e] = v;
}

// Per-station sums of the spread counters: out[4s..4s+3] = e_raw,
// max_bucket, e_voted, n_distinct of station s (one workgroup per station).
__global__ __launch_bounds__(kPT) void k_spread_reduce(const unsigned long long* e_raw,
                                                       const unsigned int* max_bucket,
                                                       const unsigned long long* e_voted,
                                                       const unsigned long long* n_distinct,
                                                       unsigned long long* out) {
  __shared__ unsigned long long part[3][kPT / 64];
  __shared__ unsigned int pmax[kPT / 64];
  const uint64_t o = (uint64_t)blockIdx.x * kSpread;
  unsigned long long er = 0, ev = 0, nd = 0;
  unsigned int mx = 0;
  for (uint32_t k = threadIdx.x; k < kSpread; k += kPT) {
    er += e_raw[o + k];
    ev += e_voted[o + k];
    nd += n_distinct[o + k];
    mx = max(mx, max_bucket[o + k]);
  }
  for (int d = 32; d > 0; d >>= 1) {
    er += __shfl_xor(er, d, 64);
    ev += __shfl_xor(ev, d, 64);
    nd += __shfl_xor(nd, d, 64);
    mx = max(mx, (unsigned int)__shfl_xor(mx, d, 64));
  }
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][w] = er;
    part[1][w] = ev;
    part[2][w] = nd;
    pmax[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a = 0, b = 0, c = 0;
    unsigned int m = 0;
    for (uint32_t q = 0; q < kPT / 64; ++q) {
      a += part[0][q];
      b += part[1][q];
      c += part[2][q];
      m = max(m, pmax[q]);
    }
    out[4 * blockIdx.x + 0] = a;
    out[4 * blockIdx.x + 1] = m;
    out[4 * blockIdx.x + 2] = b;
    out[4 * blockIdx.x + 3] = c;
  }
}

// Partitioned search, one partition [lo, hi) of size psize: fp[i] = 1 for
// every fingerprint of it not excluded whose candidate count exceeds the
// threshold (cand * den > psize * num); *nfp counts them.
__global__ __launch_bounds__(kPT) void k_part_flag(const uint8_t* ex, const uint32_t* cand, uint64_t lo, uint64_t hi,
                                                   uint32_t num, uint32_t den, uint8_t* fp, unsigned int* nfp) {
  const uint64_t psize = hi - lo;
  unsigned int c = 0;
  for (uint64_t i = lo + (uint64_t)blockIdx.x * kPT + threadIdx.x; i < hi; i += (uint64_t)gridDim.x * kPT) {
    const bool f = !ex[i] && (unsigned __int128)cand[i] * den > (unsigned __int128)psize * num;
    fp[i] = f ? 1 : 0;
    c += f ? 1u : 0u;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(nfp, c);
}

// ex[i] |= fp[i] | ex_next[i] over [0, n); fp and ex_next cleared.
__global__ __launch_bounds__(kPT) void k_part_merge(uint8_t* ex, uint8_t* fp, uint8_t* ex_next, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * kPT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kPT) {
    if (fp[i] | ex_next[i]) ex[i] = 1;
    fp[i] = 0;
    ex_next[i] = 0;
  }
}

// check_candidate for rows held in registers (RSW dwords each, read from
// memory once): the fields with equal sub-keys are found in one pass, then
// those below u's field and those above it are settled by exact key checks.
template <int RSW>
__device__ __forceinline__ void check_candidate_regs(const PairArgs& a, uint32_t u, uint32_t i, uint32_t j,
                                                     const uint32_t (&ri)[RSW], const uint32_t (&rj)[RSW]) {
  constexpr int kC = (RSW + 15) / 16;  // chunks of 32 fields
  const uint32_t g = u / a.tables_per_group, own = u - g * a.tables_per_group;
  const uint32_t tb = g * a.tables_per_group;
  const uint32_t fields = min(a.tables_per_group, a.t - tb);
  uint32_t lo[kC], hi[kC];
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    uint32_t m = 0;
#pragma unroll
    for (int d = 0; d < 16; ++d) {
      const int k = c * 16 + d;
      if (k < RSW) {
        const uint32_t x = ri[k] ^ rj[k];
        m |= ((x & 0xFFFFu) == 0 ? 1u : 0u) << (2 * d);
        m |= ((x >> 16) == 0 ? 1u : 0u) << (2 * d + 1);
      }
    }
    const uint32_t f0 = 32u * c;
    const uint32_t nf = fields > f0 ? min(32u, fields - f0) : 0u;  // fields of the group in this chunk
    m &= nf == 32 ? 0xFFFFFFFFu : (1u << nf) - 1u;
    const uint32_t below = own <= f0 ? 0u : (own - f0 >= 32 ? 0xFFFFFFFFu : (1u << (own - f0)) - 1u);
    const uint32_t upto = own < f0 ? 0u : (own - f0 >= 31 ? 0xFFFFFFFFu : (2u << (own - f0)) - 1u);
    lo[c] = m & below;
    hi[c] = m & ~upto;
  }
#pragma unroll
  for (int c = 0; c < kC; ++c)
    if (lo[c] && count_shared(a, lo[c], tb + 32u * c, i, j, 1) != 0) return;  // a lower table shares
#pragma unroll
  for (int c = 0; c < kC; ++c)
    if (hi[c] && count_shared(a, hi[c], tb + 32u * c, i, j, 1) != 0) {
      exact_and_report(a, u, i, j);
      return;
    }
}

// The queued candidates of spread slot blockIdx.x, one lane per pair (the
// slot's entries split over kCheckSplit workgroups), each pair's two rows
// read from memory once.
constexpr uint32_t kCheckSplit = 16;
template <int RSW>
__global__ __launch_bounds__(kPT) void k_check_queue(PairArgs a) {
  const uint32_t slot = blockIdx.x;
  const uint32_t cnt = min(a.q_count[slot], a.qcap);
  const uint4* q = a.q + (uint64_t)slot * a.qcap;
  for (uint32_t e = blockIdx.y * kPT + threadIdx.x; e < cnt; e += kCheckSplit * kPT) {
    const uint4 c = q[e];
    if (a.q_ovf[c.w]) continue;  // its workgroup runs again with the checks in place
    const uint32_t g = c.z / a.tables_per_group;
    const uint32_t* R = a.rows + (uint64_t)g * a.n * a.row_pitch;
    const uint32_t* pi = R + (uint64_t)c.x * a.row_pitch;
    const uint32_t* pj = R + (uint64_t)c.y * a.row_pitch;
    uint32_t ri[RSW], rj[RSW];
#pragma unroll
    for (int k = 0; k < RSW; ++k) {
      ri[k] = pi[k];
      rj[k] = pj[k];
    }
    check_candidate_regs<RSW>(a, c.z, c.x, c.y, ri, rj);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
static unsigned grid_for(uint64_t count) {
  const uint64_t b = (count + kPT - 1) / kPT;
  return (unsigned)(b == 0 ? 1 : (b < 65535 ? b : 65535));
}

// The group test reduces to "another table shares a bucket" when a pair
// needs two shared tables in its group and no distinct count is wanted (the
// partitioned passes always take the counting form).
// The reporting pass of a partition (mode 3) is the plain search restricted
// to a range of i, so it takes the same form.
static bool fast_test(const PairArgs& a) {
  return a.need == 2 && !a.want_distinct && (a.part_mode == 0 || a.part_mode == 3);
}

// Persistent: one resident round of one-wave workgroups (as many as a CU
// holds by LDS, at most kPairWavesPerCU) spread over the segments.
uint32_t pair_small_max(uint32_t need, bool distinct, uint32_t parts, uint32_t row_dw) {
  return (need == 2 && !distinct && parts == 0 && (row_dw == 10 || row_dw == 17)) ? kSmallBucket
                                                                                  : kSmallBucketGeneral;
}

void launch_pairs_wave(const PairArgs& a, const uint8_t* marks, uint32_t S, uint32_t rswl, uint32_t small_max,
                       hipStream_t s) {
  if (a.n == 0 || S == 0) return;
  const uint32_t span = 64 + small_max - 1;
  const size_t smem = (size_t)(span * rswl + span + 64 + 65) * 4;
  const uint32_t nchunk = (uint32_t)((a.n + 63) / 64);
  const uint32_t per_cu = (uint32_t)std::max<size_t>(1, std::min<size_t>(kPairWavesPerCU, (160u << 10) / smem));
  const uint32_t per_seg = std::max<uint32_t>(1u, std::min<uint32_t>(nchunk, per_cu * device_cus() / S));
  const dim3 grid(per_seg, S);
  const bool fast = fast_test(a), queue = fast && a.qcap != 0;
#define FL_WAVE(R, F, Q) \
  hipLaunchKernelGGL((k_pairs_wave<R, F, Q>), grid, dim3(64), smem, s, a, marks, rswl, nchunk, span)
  switch (a.row_dw) {
    case 10: if (queue) FL_WAVE(10, true, true); else if (fast) FL_WAVE(10, true, false); else FL_WAVE(10, false, false); break;
    case 17: if (queue) FL_WAVE(17, true, true); else if (fast) FL_WAVE(17, true, false); else FL_WAVE(17, false, false); break;
    case 50:  // one group of 100 tables
      if (queue) FL_WAVE(50, true, true); else if (fast) FL_WAVE(50, true, false); else FL_WAVE(50, false, false);
      break;
    default: FL_WAVE(0, false, false); break;
  }
#undef FL_WAVE
}

bool pair_launch_queues(const PairArgs& a) {
  return a.qcap != 0 && fast_test(a) && (a.row_dw == 10 || a.row_dw == 17 || a.row_dw == 50);
}

void launch_check_queue(const PairArgs& a, hipStream_t s) {
  if (!pair_launch_queues(a)) return;
  const dim3 grid(kSpread, kCheckSplit);
  switch (a.row_dw) {
    case 10: hipLaunchKernelGGL(k_check_queue<10>, grid, dim3(kPT), 0, s, a); break;
    case 17: hipLaunchKernelGGL(k_check_queue<17>, grid, dim3(kPT), 0, s, a); break;
    default: hipLaunchKernelGGL(k_check_queue<50>, grid, dim3(kPT), 0, s, a); break;  // 50 (pair_launch_queues)
  }
  fill_u32(a.q_count, kSpread, 0, s);  // the queue is empty again
}

void launch_tile_counts(const uint4* big, uint32_t nbig, uint32_t tb, uint64_t* tiles, unsigned long long* work,
                        hipStream_t s) {
  if (nbig)
    hipLaunchKernelGGL(k_tile_counts, dim3((nbig + kPT - 1) / kPT), dim3(kPT), 0, s, big, nbig, tb, tiles, work);
}

void launch_part_flag(const uint8_t* ex, const uint32_t* cand, uint64_t lo, uint64_t hi, uint32_t num, uint32_t den,
                      uint8_t* fp, unsigned int* nfp, hipStream_t s) {
  if (hi > lo) hipLaunchKernelGGL(k_part_flag, dim3(grid_for(hi - lo)), dim3(kPT), 0, s, ex, cand, lo, hi, num, den, fp, nfp);
}

void launch_part_merge(uint8_t* ex, uint8_t* fp, uint8_t* ex_next, uint64_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_part_merge, dim3(grid_for(n)), dim3(kPT), 0, s, ex, fp, ex_next, n);
}

void launch_work_reduce(const unsigned long long* work, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_work_reduce, dim3(1), dim3(kPT), 0, s, work, out);
}

void launch_unit_owner(const uint64_t* toff, uint32_t nbig, uint32_t* owner, hipStream_t s) {
  if (nbig) {
    const uint32_t blocks = std::min<uint32_t>((nbig + kPT / 64 - 1) / (kPT / 64), 16 * device_cus());
    hipLaunchKernelGGL(k_unit_owner, dim3(blocks), dim3(kPT), 0, s, toff, nbig, owner);
  }
}

void launch_pairs_tile(const PairArgs& a, const uint64_t* toff, const uint32_t* owner, uint64_t unit_base, uint32_t nunits,
                       const uint4* big, uint32_t tb_size, uint32_t rswl, hipStream_t s) {
  if (nunits == 0) return;
  const size_t smem = (size_t)tb_size * rswl * 8 + (size_t)tb_size * 8;
  const bool fast = fast_test(a), queue = fast && a.qcap != 0;
#define FL_TILE(R, F, Q)                                                                                        \
  hipLaunchKernelGGL((k_pairs_tile<R, F, Q>), dim3(nunits), dim3(kPT), smem, s, a, toff, owner, unit_base, big, \
                     tb_size, rswl)
  switch (a.row_dw) {
    case 10: if (queue) FL_TILE(10, true, true); else if (fast) FL_TILE(10, true, false); else FL_TILE(10, false, false); break;
    case 17: if (queue) FL_TILE(17, true, true); else if (fast) FL_TILE(17, true, false); else FL_TILE(17, false, false); break;
    case 50: if (queue) FL_TILE(50, true, true); else if (fast) FL_TILE(50, true, false); else FL_TILE(50, false, false); break;
    default: FL_TILE(0, false, false); break;
  }
#undef FL_TILE
}

void launch_split_out(const uint64_t* key, const uint32_t* val, uint64_t count, uint32_t* oi, uint32_t* oj,
                      uint8_t* ov, const uint64_t* base, uint32_t nb, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_split_out, dim3(grid_for(count)), dim3(kPT), 0, s, key, val, count, oi, oj, ov, base, nb);
}

void launch_station_offsets(const uint64_t* key, uint64_t count, const uint64_t* base, uint32_t nb,
                            unsigned long long* offs, hipStream_t s) {
  hipLaunchKernelGGL(k_station_offsets, dim3(1), dim3(64), 0, s, key, count, base, nb, offs);
}

void launch_pack_out(const uint32_t* oi, const uint32_t* oj, const uint8_t* ov, uint64_t count, uint64_t* key,
                     uint32_t* val, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_pack_out, dim3(grid_for(count)), dim3(kPT), 0, s, oi, oj, ov, count, key, val);
}

void launch_count_flags(const uint8_t* flags, uint64_t n, unsigned long long* out, unsigned long long* total,
                        hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_count_flags, dim3(grid_for(n) < 1024 ? grid_for(n) : 1024), dim3(kPT), 0, s, flags, n, out,
                     total);
}

void launch_spread_reduce(const unsigned long long* e_raw, const unsigned int* max_bucket,
                          const unsigned long long* e_voted, const unsigned long long* n_distinct, uint32_t S,
                          unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_spread_reduce, dim3(S), dim3(kPT), 0, s, e_raw, max_bucket, e_voted, n_distinct, out);
}

void fill_u8(uint8_t* p, uint64_t count, uint8_t v, hipStream_t s) {
  if (count) hipLaunchKernelGGL((k_fill<uint8_t>), dim3(grid_for(count)), dim3(kPT), 0, s, p, count, v);
}
void fill_u32(uint32_t* p, uint64_t count, uint32_t v, hipStream_t s) {
  if (count) hipLaunchKernelGGL((k_fill<uint32_t>), dim3(grid_for(count)), dim3(kPT), 0, s, p, count, v);
}
void fill_u64(uint64_t* p, uint64_t count, uint64_t v, hipStream_t s) {
  if (count) hipLaunchKernelGGL((k_fill<uint64_t>), dim3(grid_for(count)), dim3(kPT), 0, s, p, count, v);
}

}  // namespace fl
