// Grouping of band keys into hash-table buckets (section 6.1 "Hash table
// construction").
//
// Every table's (key, id) pairs are grouped by stable least-significant-
// digit radix passes over the top B bits of fmix64(band key) (the mix spreads
// the highly skewed packed-argmin keys evenly; B is 8, 16, 24 or 32 so that
// an average bin holds a few dozen elements at most), which leaves each bin
// contiguous with its ids ascending.  A bin then holds a few whole buckets,
// nearly always a single key; bins that mix keys are ranked by (key, id)
// inside LDS.  Bucket boundaries, sizes, the raw candidate count and the
// occurrence filter are derived in the same pass.  Bins too large for LDS
// (huge buckets) take a slower single-workgroup path.
//
// Radix pass = tile histogram -> segmented exclusive scan -> stable scatter.
// The scatter ranks equal digits inside a wavefront with eight 64-lane
// ballots (no LDS atomics, so the ranking is deterministic and stable), then
// stages the tile in LDS in digit order so that global writes are runs of
// consecutive addresses.
#include <algorithm>

#include "common.hpp"

namespace fl {

constexpr int kThreads = 256;
constexpr int kRadix = 256;
constexpr int kScanBlock = 4096;

__device__ __forceinline__ uint64_t lanemask_lt() { return __lanemask_lt(); }

// Lanes of the wave whose 8-bit digit equals this lane's.
__device__ __forceinline__ uint64_t match_digit(uint32_t d) {
  uint64_t peers = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint32_t bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    peers &= bit ? bal : ~bal;
  }
  return peers;
}

// ---------------------------------------------------------------------------
// Radix pass kernels.  Segment s occupies [s*n, (s+1)*n) of every array.
// vin == nullptr means the value of element e is e (its id).
// ---------------------------------------------------------------------------
// Default radix-pass tile: 16,384 elements (1024 threads x 16).  Large tiles
// make each digit's run of output addresses long (64 elements on average),
// which is what lets the scatter write at a large fraction of HBM bandwidth.
// Smaller tiles (8,192 and 4,096) run more workgroups per CU and are offered
// to the launch-shape tuner.
constexpr int kRThreads = 1024;
constexpr int kRItems = 16;
constexpr int kTile = kRThreads * kRItems;

template <int THREADS = kRThreads, int ITEMS = kRItems>
__global__ __launch_bounds__(THREADS) void k_hist(const uint64_t* keys, uint64_t n, uint32_t shift,
                                                  uint32_t* hist, uint32_t ntiles) {
  constexpr int kRWaves = THREADS / 64;
  constexpr int kRThreads = THREADS;
  constexpr int kRItems = ITEMS;
  constexpr int kTile = THREADS * ITEMS;
  __shared__ uint32_t cnt[kRWaves][kRadix];
  const uint32_t tid = threadIdx.x, wave = tid >> 6;
  for (uint32_t q = tid; q < kRWaves * kRadix; q += kRThreads) (&cnt[0][0])[q] = 0;
  __syncthreads();
  const uint64_t seg = blockIdx.y, tile = blockIdx.x;
  const uint64_t* K = keys + seg * n;
  const uint64_t e0 = tile * kTile;
#pragma unroll
  for (int k = 0; k < kRItems; ++k) {
    const uint64_t e = e0 + (uint64_t)k * kRThreads + tid;
    if (e < n) atomicAdd(&cnt[wave][(K[e] >> shift) & 0xFF], 1u);
  }
  __syncthreads();
  if (tid < kRadix) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kRWaves; ++w) t += cnt[w][tid];
    hist[(seg * kRadix + tid) * ntiles + tile] = t;
  }
}

template <int THREADS = kRThreads, int ITEMS = kRItems>
__global__ __launch_bounds__(THREADS) void k_scatter(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                                                     uint32_t* vout, uint64_t n, uint32_t shift,
                                                     const uint32_t* hist, uint32_t ntiles) {
  constexpr int kRWaves = THREADS / 64;
  constexpr int kRThreads = THREADS;
  constexpr int kRItems = ITEMS;
  constexpr int kTile = THREADS * ITEMS;
  __shared__ uint32_t wcnt[kRWaves][kRadix];
  __shared__ uint32_t tstart[kRadix];
  __shared__ uint32_t gbase[kRadix];
  __shared__ uint32_t wsum[4];
  __shared__ uint64_t sk[kTile];  // staging: keys, then values
  uint32_t* sv = reinterpret_cast<uint32_t*>(sk);
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (uint32_t q = tid; q < kRWaves * kRadix; q += kRThreads) (&wcnt[0][0])[q] = 0;
  __syncthreads();
  const uint64_t seg = blockIdx.y, tile = blockIdx.x;
  const uint64_t* K = kin + seg * n;
  const uint32_t* V = vin ? vin + seg * n : nullptr;
  // wave w owns the contiguous slice [w*512, (w+1)*512) of the tile, in
  // kRItems steps of 64 elements: stable order is (wave, step, lane).
  const uint64_t e0 = tile * kTile + (uint64_t)wave * (kTile / kRWaves);
  const uint64_t lt = lanemask_lt();

  uint64_t key[kRItems];
  uint32_t val[kRItems], rank[kRItems];
#pragma unroll
  for (int k = 0; k < kRItems; ++k) {
    const uint64_t e = e0 + (uint64_t)k * 64 + lane;
    const bool ok = e < n;
    key[k] = ok ? K[e] : ~0ull;
    val[k] = ok ? (V ? V[e] : (uint32_t)e) : 0u;
  }
#pragma unroll
  for (int k = 0; k < kRItems; ++k) {
    const uint64_t e = e0 + (uint64_t)k * 64 + lane;
    const uint32_t d = e < n ? (uint32_t)(key[k] >> shift) & 0xFF : 0xFFu;
    const uint64_t peers = match_digit(d);
    const uint32_t before = __popcll(peers & lt);
    const uint32_t base = wcnt[wave][d];
    rank[k] = base + before;
    if ((peers >> lane) == 1ull) wcnt[wave][d] = base + __popcll(peers);  // highest lane of the group
  }
  __syncthreads();
  // Per digit: prefix over waves and the tile total; then the tile-level
  // digit start (exclusive scan over digits by the first four waves).
  uint32_t tot = 0;
  if (tid < kRadix) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kRWaves; ++w) {
      const uint32_t c = wcnt[w][tid];
      wcnt[w][tid] = s;
      s += c;
    }
    tot = s;
    gbase[tid] = hist[(seg * kRadix + tid) * ntiles + tile];
  }
  uint32_t inc = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += y;
  }
  if (tid < kRadix && lane == 63) wsum[wave] = inc;
  __syncthreads();
  if (tid < kRadix) {
    uint32_t add = 0;
    for (uint32_t w = 0; w < wave; ++w) add += wsum[w];
    tstart[tid] = add + inc - tot;
  }
  __syncthreads();
  const uint64_t tile0 = tile * kTile;
  const uint32_t nvalid = (uint32_t)((n - tile0) < (uint64_t)kTile ? (n - tile0) : (uint64_t)kTile);
  uint32_t pos[kRItems];
#pragma unroll
  for (int k = 0; k < kRItems; ++k) {
    const uint64_t e = e0 + (uint64_t)k * 64 + lane;
    if (e < n) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & 0xFF;
      pos[k] = tstart[d] + wcnt[wave][d] + rank[k];
      sk[pos[k]] = key[k];
    }
  }
  __syncthreads();
  uint64_t* KO = kout + seg * n;
  uint32_t* VO = vout + seg * n;
  uint32_t gq[kRItems];  // global position of staged element tid + k*kRThreads
#pragma unroll
  for (int k = 0; k < kRItems; ++k) {
    const uint32_t q = tid + k * kRThreads;
    if (q < nvalid) {
      const uint64_t kk = sk[q];
      const uint32_t d = (uint32_t)(kk >> shift) & 0xFF;
      gq[k] = gbase[d] + (q - tstart[d]);
      KO[gq[k]] = kk;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRItems; ++k) {
    const uint64_t e = e0 + (uint64_t)k * 64 + lane;
    if (e < n) sv[pos[k]] = val[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRItems; ++k) {
    const uint32_t q = tid + k * kRThreads;
    if (q < nvalid) VO[gq[k]] = sv[q];
  }
}

// ---------------------------------------------------------------------------
// Segmented exclusive scan: S segments of len elements each, in blocks of
// kScanBlock.  (1) block sums, (2) per-segment scan of block sums by one
// workgroup, (3) block-local scan plus block offset.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* wsum, T* total) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  T inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += y;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  T add = 0, all = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) {
    if (w < wave) add += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  if (total) *total = all;
  return add + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_sums(const T* data, uint64_t len, T* sums, uint32_t nblk) {
  const uint64_t seg = blockIdx.y, blk = blockIdx.x;
  const T* d = data + seg * len;
  const uint64_t b0 = blk * (uint64_t)kScanBlock;
  T s = 0;
  for (uint32_t q = threadIdx.x; q < kScanBlock; q += kThreads) {
    const uint64_t e = b0 + q;
    if (e < len) s += d[e];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ T ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) sums[seg * nblk + blk] = ws[0] + ws[1] + ws[2] + ws[3];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_blocksums(T* sums, uint32_t nblk, T* seg_total) {
  __shared__ T ws[4];
  __shared__ T carry;
  const uint64_t seg = blockIdx.x;
  T* s = sums + seg * nblk;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < nblk; b0 += kThreads) {
    const uint32_t b = b0 + threadIdx.x;
    const T v = b < nblk ? s[b] : (T)0;
    T tot;
    const T ex = block_excl_scan<T>(v, ws, &tot);
    const T c = carry;
    if (b < nblk) s[b] = c + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + tot;
    __syncthreads();
  }
  if (seg_total && threadIdx.x == 0) seg_total[seg] = carry;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_apply(T* data, uint64_t len, const T* sums, uint32_t nblk) {
  __shared__ T ws[4];
  const uint64_t seg = blockIdx.y, blk = blockIdx.x;
  T* d = data + seg * len;
  const uint64_t b0 = blk * (uint64_t)kScanBlock;
  constexpr int per = kScanBlock / kThreads;  // 16 consecutive elements per thread
  T v[per];
  T s = 0;
  const uint64_t base = b0 + (uint64_t)threadIdx.x * per;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const uint64_t e = base + q;
    v[q] = e < len ? d[e] : (T)0;
    s += v[q];
  }
  T tot;
  T ex = block_excl_scan<T>(s, ws, &tot) + sums[seg * nblk + blk];
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const uint64_t e = base + q;
    if (e < len) d[e] = ex;
    ex += v[q];
  }
}

// ---------------------------------------------------------------------------
// Buckets from the bin-sorted order.
//
// One wavefront per span of `chunk` consecutive positions of a table: it owns
// the bins whose first position lies in the span.  The span (with the
// position before it and kSpanExt positions after it) is staged in the
// wave's own LDS slice, and the wave walks it kWin positions at a time from
// one bin start (kWinQ positions per lane): ballots of bin starts give every
// complete bin of the window, its size and its first and last member.  A
// bin holding a single key is one bucket already in id order; a bin that
// mixes keys is ranked from LDS (each member counts the (key, position)
// pairs below it).  A bin that does not end inside the window is read from
// HBM; mixed ones above kRankLong members and all above kLongDefer go to
// the big-bin list.  No workgroup barriers: the waves are independent.
// ---------------------------------------------------------------------------
constexpr uint32_t kWinQ = 1;         // window positions per lane
constexpr uint32_t kWin = 64 * kWinQ; // positions per window
constexpr uint32_t kSpanExt = kWin;   // positions staged past a span for its last bins
constexpr uint32_t kStageB = 5;       // 64-position loads in flight per lane while staging
constexpr uint32_t kBucketWaves = 4;  // independent wavefronts per workgroup
constexpr uint32_t kRankLong = 128;   // largest mixed bin ranked by one wave from HBM
constexpr uint32_t kLongDefer = 2048; // larger bins go to the big-bin kernel

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Per-thread bucket counters.  With several stations the station of a
// bucket is the top four bits of its mixed key, and stations are contiguous
// in every sorted table, so a thread's buckets change station only at a
// station boundary, where bucket_account flushes the open totals.
// station == kNoStation: no bucket accounted yet.
constexpr uint32_t kNoStation = 0xFFFFFFFFu;

struct BucketTotals {
  unsigned long long e_raw;
  unsigned int max_bucket;
  uint32_t station;
  uint64_t occ_max;  // largest bucket of `station` within the occurrence threshold
};

// Occurrence filter (section 6.5): a bucket of `size` members is over the
// threshold of its station (fingerprint count ns) when size / ns > num / den,
// that is size * den > ns * num, which for an integer size is
// size > floor(ns * num / den) = occ_max[station] (computed on the host).

// Called by every lane of the wave.  When all lanes that accounted a bucket
// hold one station the totals are reduced over the wave first; at a station
// boundary each lane adds its own.
__device__ void flush_totals(const BucketArgs& a, BucketTotals tot) {
  const uint64_t act = __ballot(tot.station != kNoStation);
  if (act == 0) return;
  const uint32_t s0 = __shfl(tot.station, __ffsll((long long)act) - 1, 64);
  if (!__all(tot.station == kNoStation || tot.station == s0)) {
    if (tot.station == kNoStation) return;
    const uint64_t o = (uint64_t)tot.station * kSpread + spread_slot();
    if (tot.e_raw) atomicAdd(a.e_raw + o, tot.e_raw);
    if (tot.max_bucket) atomicMax(a.max_bucket + o, tot.max_bucket);
    return;
  }
  unsigned long long e = tot.e_raw;
  unsigned int m = tot.max_bucket;
  for (int o = 32; o > 0; o >>= 1) {
    e += __shfl_xor(e, o, 64);
    const unsigned int om = __shfl_xor(m, o, 64);
    m = om > m ? om : m;
  }
  if ((threadIdx.x & 63) == 0) {
    const uint64_t o = (uint64_t)s0 * kSpread + spread_slot();
    if (e) atomicAdd(a.e_raw + o, e);
    if (m) atomicMax(a.max_bucket + o, m);
  }
}

// The station's bound is recomputed when the station changes (a lane's keys
// change station only at station boundaries of the sorted order).
struct OccCache {
  uint32_t st = kNoStation;
  uint64_t occ_max = 0;
};
__device__ __forceinline__ bool bucket_over(const BucketArgs& a, uint64_t size, uint64_t key, OccCache& oc) {
  if (!a.occ_den) return false;
  const uint32_t st = a.nstation > 1 ? (uint32_t)(key >> 60) : 0u;
  if (st != oc.st) {
    oc.st = st;
    oc.occ_max = a.occ_max[st];
  }
  return size > oc.occ_max;
}

// Counters of one bucket (this lane heads it) and its descriptor class:
// 0 none (one member, over the occurrence threshold, or an id span below
// the lag), 1 small, 2 big.  The members' flags are the caller's.
__device__ __forceinline__ int head_account(const BucketArgs& a, uint64_t size, uint32_t first_id, uint32_t last_id,
                                            uint64_t key, BucketTotals& tot) {
  const uint32_t st = a.nstation > 1 ? (uint32_t)(key >> 60) : 0u;
  if (st != tot.station) {
    if (tot.station != kNoStation) {  // counters of another station: add the open totals directly
      const uint64_t o = (uint64_t)tot.station * kSpread + spread_slot();
      if (tot.e_raw) atomicAdd(a.e_raw + o, tot.e_raw);
      if (tot.max_bucket) atomicMax(a.max_bucket + o, tot.max_bucket);
    }
    tot.e_raw = 0;
    tot.max_bucket = 0;
    tot.station = st;
    tot.occ_max = a.occ_max[st];
  }
  tot.e_raw += (unsigned long long)(size * (size - 1) / 2);
  if (size > tot.max_bucket) tot.max_bucket = (unsigned int)size;
  if (size > tot.occ_max) return 0;
  if (size < 2 || last_id - first_id < a.min_lag) return 0;
  return size <= a.small_max ? 1 : 2;
}

// Account one bucket (run of equal keys) of `size` members; ids(q) gives the
// q-th member (ascending); flags the members of a bucket over the
// occurrence threshold.  Returns the descriptor class (head_account).
template <typename IdAt>
__device__ __forceinline__ int bucket_account(const BucketArgs& a, uint64_t size, IdAt ids, uint32_t first_id,
                                              uint64_t key, BucketTotals& tot) {
  const int cls = head_account(a, size, first_id, ids(size - 1), key, tot);
  OccCache oc;
  if (cls == 0 && bucket_over(a, size, key, oc))
    for (uint64_t q = 0; q < size; ++q) a.flags[ids(q)] = 1;
  return cls;
}

// Big-bucket descriptors.  A wave reserves kSlab slots of the list at a time
// (one atomic per reservation: a counter that every bucket bumped would
// serialise all waves on one L2 channel) and fills the slots it leaves
// unused with empty descriptors (size 0), which every reader skips.
constexpr uint32_t kSlab = 64;
struct DescSlab {
  uint32_t pos = 0, end = 0;  // wave-uniform
};

// Descriptors of the big buckets that lanes with `want` head (called by
// every lane of the wave), in consecutive slots.
__device__ __forceinline__ void slab_put(const BucketArgs& a, DescSlab& sl, bool want, uint64_t pos, uint32_t seg,
                                         uint64_t size) {
  const uint64_t m = __ballot(want);
  if (m == 0) return;
  const uint32_t k = (uint32_t)__popcll(m), lane = threadIdx.x & 63;
  if (sl.pos + k > sl.end) {
    for (uint32_t q = sl.pos + lane; q < sl.end; q += 64) a.big_desc[q] = make_uint4(0u, 0u, 0u, 0u);
    const uint32_t take = k > kSlab ? k : kSlab;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(a.big_count, take);
    base = __shfl(base, 0, 64);
    sl.pos = base;
    sl.end = base + take;
  }
  if (want) a.big_desc[sl.pos + __popcll(m & lanemask_lt())] = make_uint4((uint32_t)pos, seg, (uint32_t)size, 0);
  sl.pos += k;
}

// The wave's last reservation: its unused slots become empty descriptors.
__device__ __forceinline__ void slab_close(const BucketArgs& a, const DescSlab& sl) {
  for (uint32_t q = sl.pos + (threadIdx.x & 63); q < sl.end; q += 64) a.big_desc[q] = make_uint4(0u, 0u, 0u, 0u);
}

// One element of a bucket after ranking: its new position in the bin, the
// bucket it belongs to (size, first and last id) and whether it heads it;
// writes its mark and id, flags it if the bucket is over the threshold, and
// accounts the bucket at its head.  Returns the class at the head, else 0.
__device__ __forceinline__ int place(const BucketArgs& a, uint8_t* M, uint32_t* V, uint64_t at, uint64_t key,
                                     uint32_t id, bool head, uint64_t size, uint32_t first_id, uint32_t last_id,
                                     bool write_id, BucketTotals& tot, OccCache& oc) {
  if (bucket_over(a, size, key, oc)) a.flags[id] = 1;
  const int cls = head ? head_account(a, size, first_id, last_id, key, tot) : 0;
  M[at] = cls == 1 ? (uint8_t)size : (uint8_t)0;
  if (write_id) V[at] = id;
  return cls;
}

// A bin [b, end) that did not end inside the wave's window, from HBM (every
// lane calls it): its end, whether it mixes keys, and then either one bucket
// (one key), a ranking of up to kRankLong members, or the big-bin list (bins
// above kLongDefer members, and mixed ones above kRankLong, go there, to the
// kernel that spreads a bin over a whole workgroup).  Returns the bin's end.
__device__ uint64_t long_bin(const BucketArgs& a, uint32_t seg, uint64_t b, const uint64_t* K, uint32_t* V,
                             uint8_t* M, BucketTotals& tot, OccCache& oc, DescSlab& sl) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t n = a.n;
  const uint32_t bsh = a.bin_shift;
  const uint64_t k0 = K[b], bin0 = k0 >> bsh;
  // The bin's end among the next kScan positions (one round trip of loads),
  // else by galloping and then bisecting over the ascending bin bits.
  constexpr uint32_t kScanQ = 4;  // 64-position blocks per round trip
  uint64_t end = n;
  bool mixed = false, found = false;
  for (uint64_t c = b; c < n && !found; c += 64 * kScanQ) {
    uint64_t kp[kScanQ];
#pragma unroll
    for (uint32_t q = 0; q < kScanQ; ++q) {
      const uint64_t p = c + 64 * q + lane;
      kp[q] = p < n ? K[p] : k0;
    }
#pragma unroll
    for (uint32_t q = 0; q < kScanQ; ++q) {
      if (found) continue;
      const uint64_t p = c + 64 * q + lane;
      const bool in = p < n;
      const uint64_t stop = __ballot(in && (kp[q] >> bsh) != bin0);
      const uint64_t before = stop ? ((1ull << (__ffsll((long long)stop) - 1)) - 1) : ~0ull;
      if (__ballot(in && kp[q] != k0) & before) mixed = true;
      if (stop) {
        end = c + 64 * q + (uint64_t)__ffsll((long long)stop) - 1;
        found = true;
      } else if (!__ballot(in)) {
        found = true;  // end of the table: end = n
      }
    }
    // the round reached the table's end without leaving the bin: the bin
    // ends with the table (end = n)
    if (!found && c + 64 * kScanQ >= n) found = true;
    if (!found && c + 64 * kScanQ - b >= kLongDefer) break;  // long: bisect below
  }
  if (!found) {
    uint64_t lo = b + 64 * kScanQ, step = 64 * kScanQ;  // bin(lo - 1) == bin0
    uint64_t hi = n;
    while (lo < n) {  // gallop: first probe past the bin bounds the search
      const uint64_t pr = lo + step < n ? lo + step : n - 1;
      if ((K[pr] >> bsh) != bin0) {
        hi = pr;
        break;
      }
      lo = pr + 1;
      step *= 2;
    }
    while (lo < hi) {  // first position in [lo, hi) outside the bin
      const uint64_t mid = (lo + hi) / 2;
      if ((K[mid] >> bsh) != bin0) hi = mid; else lo = mid + 1;
    }
    end = lo;
  }
  const uint64_t s = end - b;
  if (s > kLongDefer || (mixed && s > kRankLong) || (!found && s > 64 * kScanQ)) {
    if (lane == 0) {
      const uint32_t q = atomicAdd(a.bin_count, 1u);
      a.bin_desc[q] = make_uint4((uint32_t)b, (uint32_t)end, seg, 0);
    }
    return end;
  }
  if (!mixed) {
    const uint32_t first = V[b], last = V[end - 1];
    int cls = 0;
    if (lane == 0) cls = head_account(a, s, first, last, k0, tot);
    cls = __shfl(cls, 0, 64);
    const bool over = bucket_over(a, s, k0, oc);
    for (uint64_t c = b; c < end; c += 64) {
      const uint64_t p = c + lane;
      if (p < end) {
        M[p] = (p == b && cls == 1) ? (uint8_t)s : (uint8_t)0;
        if (over) a.flags[V[p]] = 1;
      }
    }
    slab_put(a, sl, lane == 0 && cls == 2, b, seg, s);
    return end;
  }
  // Rank: element e = lane + 64 q counts the members below it in (key, position).
  constexpr int kQ = kRankLong / 64;
  uint64_t kk[kQ];
  uint32_t vv[kQ], less[kQ], eqb[kQ], eqc[kQ], lastv[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const uint32_t e = lane + 64u * q;
    kk[q] = e < s ? K[b + e] : ~0ull;
    vv[q] = e < s ? V[b + e] : 0u;
    less[q] = eqb[q] = eqc[q] = 0;
    lastv[q] = vv[q];
  }
  for (uint32_t f = 0; f < (uint32_t)s; ++f) {
    const uint64_t kf = K[b + f];
    const uint32_t vf = V[b + f];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const uint32_t e = lane + 64u * q;
      less[q] += kf < kk[q] ? 1u : 0u;
      eqb[q] += (kf == kk[q] && f < e) ? 1u : 0u;
      eqc[q] += kf == kk[q] ? 1u : 0u;
      lastv[q] = kf == kk[q] ? vf : lastv[q];
    }
  }
  // every read of the bin precedes the writes below
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const uint32_t e = lane + 64u * q;
    int cls = 0;
    if (e < s)
      cls = place(a, M, V, b + less[q] + eqb[q], kk[q], vv[q], eqb[q] == 0, eqc[q], vv[q], lastv[q], true, tot, oc);
    slab_put(a, sl, cls == 2, b + less[q], seg, eqc[q]);
  }
  return end;
}

// Bit masks over a window of kWin positions, kWinQ words (word w holds
// positions 64w .. 64w + 63).  Indices into the arrays are compile-time
// after unrolling, so they stay in registers.
// Highest set position <= p (position 0 is always set).
__device__ __forceinline__ uint32_t win_prev(const uint64_t (&H)[kWinQ], uint32_t p) {
  const uint32_t q = p >> 6, l = p & 63;
  uint32_t r = 0;
#pragma unroll
  for (uint32_t w = 0; w < kWinQ; ++w) {
    uint64_t m = w < q ? H[w] : (w == q ? H[w] & (l == 63 ? ~0ull : ((2ull << l) - 1)) : 0ull);
    if (m) r = 64 * w + 63 - (uint32_t)__clzll(m);
  }
  return r;
}
// Lowest set position > p, or kWin.
__device__ __forceinline__ uint32_t win_next(const uint64_t (&H)[kWinQ], uint32_t p) {
  const uint32_t q = p >> 6, l = p & 63;
  uint32_t r = kWin;
#pragma unroll
  for (int w = kWinQ - 1; w >= 0; --w) {
    uint64_t m = (uint32_t)w > q ? H[w] : ((uint32_t)w == q ? H[w] & (l == 63 ? 0ull : ~((2ull << l) - 1)) : 0ull);
    if (m) r = 64 * (uint32_t)w + (uint32_t)__ffsll((long long)m) - 1;
  }
  return r;
}
// Some set position in (lo, hi).
__device__ __forceinline__ bool win_any(const uint64_t (&C)[kWinQ], uint32_t lo, uint32_t hi) {
  bool any = false;
#pragma unroll
  for (uint32_t w = 0; w < kWinQ; ++w) {
    const uint32_t a = lo + 1 > 64 * w ? lo + 1 : 64 * w, b = hi < 64 * w + 64 ? hi : 64 * w + 64;
    if (a < b) {
      const uint64_t m = ((b - 64 * w) == 64 ? ~0ull : ((1ull << (b - 64 * w)) - 1)) & ~((1ull << (a - 64 * w)) - 1);
      any |= (C[w] & m) != 0;
    }
  }
  return any;
}

__global__ __launch_bounds__(kBucketWaves * 64, 5) void k_bucket(BucketArgs a, uint32_t nspans) {
  extern __shared__ uint64_t bucket_lds[];
  const uint32_t span = a.chunk;
  const uint32_t cap = span + kSpanExt + 1;  // staged positions per wave
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint64_t* sk = bucket_lds + (size_t)wave * cap;
  uint32_t* sv = reinterpret_cast<uint32_t*>(bucket_lds + (size_t)kBucketWaves * cap) + (size_t)wave * cap;
  const uint32_t seg = blockIdx.y;
  const uint32_t bsh = a.bin_shift;
  const uint64_t n = a.n;
  const uint64_t* K = a.keys + (uint64_t)seg * n;
  uint32_t* V = a.vals + (uint64_t)seg * n;
  uint8_t* M = a.marks + (uint64_t)seg * n;
  BucketTotals tot{0ull, 0u, kNoStation, 0u};
  OccCache oc;
  DescSlab sl;
  // The waves sweep the table together: the spans in flight at any time are
  // neighbours, so they share pages of the key, id and mark arrays.
  for (uint32_t sp = blockIdx.x * kBucketWaves + wave; sp < nspans; sp += gridDim.x * kBucketWaves) {
    const uint64_t s0 = (uint64_t)sp * span;
    const uint64_t s1 = s0 + span < n ? s0 + span : n;
    const uint64_t w0 = s0 ? s0 - 1 : 0;  // staged: [w0, w0 + wn)
    const uint32_t wn = (uint32_t)(n - w0 < (uint64_t)cap ? n - w0 : (uint64_t)cap);
    const bool tail = w0 + wn == n;       // the staged positions reach the table's end
    wave_sync();                          // the previous span's reads are done
    for (uint32_t e0 = 0; e0 < wn; e0 += 64 * kStageB) {  // kStageB loads in flight, then LDS
      uint64_t kb[kStageB];
      uint32_t vb[kStageB];
#pragma unroll
      for (uint32_t q = 0; q < kStageB; ++q) {
        const uint32_t e = e0 + 64 * q + lane;
        kb[q] = e < wn ? K[w0 + e] : 0ull;
        vb[q] = e < wn ? V[w0 + e] : 0u;
      }
#pragma unroll
      for (uint32_t q = 0; q < kStageB; ++q) {
        const uint32_t e = e0 + 64 * q + lane;
        if (e < wn) {
          sk[e] = kb[q];
          sv[e] = vb[q];
        }
      }
    }
    wave_sync();
    // The span's first bin start (earlier positions belong to an earlier span's bin).
    uint64_t b = s1;
    for (uint64_t c = s0; c < s1; c += 64) {
      const uint64_t p = c + lane;
      const uint32_t e = (uint32_t)(p - w0);
      const bool h = p < s1 && (p == 0 || (sk[e] >> bsh) != (sk[e - 1] >> bsh));
      const uint64_t hm = __ballot(h);
      if (hm) {
        b = c + (uint64_t)__ffsll((long long)hm) - 1;
        break;
      }
    }
    while (b < s1) {
      const uint32_t o = (uint32_t)(b - w0);
      const uint32_t avail = wn - o;  // staged positions from b, at least 1
      uint64_t kq[kWinQ], H[kWinQ], C[kWinQ];
      uint32_t vq[kWinQ];
#pragma unroll
      for (uint32_t q = 0; q < kWinQ; ++q) {
        const uint32_t P = 64 * q + lane;
        const bool valid = P < avail;
        kq[q] = valid ? sk[o + P] : 0ull;
        vq[q] = valid ? sv[o + P] : 0u;
        const uint64_t kprev = (valid && P > 0) ? sk[o + P - 1] : kq[q];
        const bool bh = valid && (P == 0 || (kq[q] >> bsh) != (kprev >> bsh));
        H[q] = __ballot(bh);
        C[q] = __ballot(valid && !bh && kq[q] != kprev);
      }
      if (avail < kWin && tail) {  // the table's end closes the last bin
#pragma unroll
        for (uint32_t q = 0; q < kWinQ; ++q)
          if (avail >> 6 == q) H[q] |= 1ull << (avail & 63);
      }
      uint32_t hl = 0;  // last start: its bin may go on
#pragma unroll
      for (uint32_t q = 0; q < kWinQ; ++q)
        if (H[q]) hl = 64 * q + 63 - (uint32_t)__clzll(H[q]);
      if (hl == 0) {
        b = long_bin(a, seg, b, K, V, M, tot, oc, sl);
        continue;
      }
      // Complete bins: those starting below hl.
      uint32_t hd[kWinQ], en[kWinQ], size[kWinQ], first[kWinQ], last[kWinQ], pos[kWinQ];
      bool act[kWinQ], mixed[kWinQ], head[kWinQ];
      uint32_t ms = 0;
#pragma unroll
      for (uint32_t q = 0; q < kWinQ; ++q) {
        const uint32_t P = 64 * q + lane;
        hd[q] = win_prev(H, P);
        en[q] = win_next(H, hd[q]);
        act[q] = P < hl && b + hd[q] < s1;
        mixed[q] = act[q] && win_any(C, hd[q], en[q]);
        pos[q] = P;
        size[q] = en[q] - hd[q];
        head[q] = P == hd[q];
        first[q] = act[q] ? sv[o + hd[q]] : 0u;
        last[q] = act[q] ? sv[o + en[q] - 1] : 0u;
        if (mixed[q]) ms = max(ms, size[q]);
      }
      if (__ballot(ms != 0)) {  // rank inside the bins that mix keys, from LDS
        for (int d = 32; d > 0; d >>= 1) ms = max(ms, (uint32_t)__shfl_xor(ms, d, 64));
        uint32_t less[kWinQ], eqb[kWinQ], eqc[kWinQ], lastv[kWinQ];
#pragma unroll
        for (uint32_t q = 0; q < kWinQ; ++q) {
          less[q] = eqb[q] = eqc[q] = 0;
          lastv[q] = vq[q];
        }
        for (uint32_t j = 0; j < ms; ++j) {
#pragma unroll
          for (uint32_t q = 0; q < kWinQ; ++q) {
            const uint32_t f = hd[q] + j;
            if (mixed[q] && f < en[q]) {
              const uint64_t kf = sk[o + f];
              const uint32_t vf = sv[o + f];
              less[q] += kf < kq[q] ? 1u : 0u;
              eqb[q] += (kf == kq[q] && f < 64 * q + lane) ? 1u : 0u;
              eqc[q] += kf == kq[q] ? 1u : 0u;
              lastv[q] = kf == kq[q] ? vf : lastv[q];
            }
          }
        }
#pragma unroll
        for (uint32_t q = 0; q < kWinQ; ++q) {
          if (mixed[q]) {
            pos[q] = hd[q] + less[q] + eqb[q];
            size[q] = eqc[q];
            first[q] = vq[q];
            last[q] = lastv[q];
            head[q] = eqb[q] == 0;
          }
        }
      }
      // every LDS read of the window precedes these writes to HBM
      bool big[kWinQ];
#pragma unroll
      for (uint32_t q = 0; q < kWinQ; ++q) {
        int cls = 0;
        if (act[q]) cls = place(a, M, V, b + pos[q], kq[q], vq[q], head[q], size[q], first[q], last[q], mixed[q], tot, oc);
        big[q] = cls == 2;
      }
#pragma unroll
      for (uint32_t q = 0; q < kWinQ; ++q) slab_put(a, sl, big[q], b + pos[q], seg, size[q]);
      b += hl;
    }
  }
  slab_close(a, sl);
  flush_totals(a, tot);
}

// ---------------------------------------------------------------------------
// Oversized bins: one workgroup sorts [lo, hi) by the key bits below the bin with
// stable 8-bit LSD passes through the scratch arrays (ids stay ascending
// within equal keys) and then accounts the buckets.
// ---------------------------------------------------------------------------
// Persistent: a fixed grid walks the bins the bucket kernel deferred (their
// count is read on the device, so the launch shape does not depend on it).
__global__ __launch_bounds__(kThreads) void k_bigbin(BucketArgs a, const uint4* bins, uint64_t* tk, uint32_t* tv) {
  __shared__ uint32_t cnt[kRadix];
  __shared__ uint32_t wc[4][kRadix];
  __shared__ uint32_t ws[8];
  __shared__ uint64_t kmin, kmax;
  __shared__ uint32_t heads[kThreads];
  __shared__ uint32_t s_carry;
  const uint32_t nbins = *a.bin_count;
  for (uint32_t q = blockIdx.x; q < nbins; q += gridDim.x) {
  __syncthreads();
  const uint4 bd = bins[q];
  const uint64_t lo = bd.x, hi = bd.y;
  const uint32_t seg = bd.z;
  const uint64_t off = (uint64_t)seg * a.n;
  uint64_t* K = const_cast<uint64_t*>(a.keys) + off;
  uint32_t* V = a.vals + off;
  uint64_t* TK = tk + off;
  uint32_t* TV = tv + off;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  if (tid == 0) { kmin = ~0ull; kmax = 0; }
  __syncthreads();
  {
    uint64_t mn = ~0ull, mx = 0;
    for (uint64_t p = lo + tid; p < hi; p += kThreads) {
      const uint64_t k = K[p];
      mn = k < mn ? k : mn;
      mx = k > mx ? k : mx;
    }
    atomicMin((unsigned long long*)&kmin, (unsigned long long)mn);
    atomicMax((unsigned long long*)&kmax, (unsigned long long)mx);
  }
  __syncthreads();
  if (kmin != kmax) {
    uint64_t *sK = K, *dK = TK;
    uint32_t *sV = V, *dV = TV;
    for (uint32_t shift = 0; shift < a.bin_shift; shift += 8) {
      for (uint32_t d = tid; d < kRadix; d += kThreads) cnt[d] = 0;
      __syncthreads();
      for (uint64_t p = lo + tid; p < hi; p += kThreads) atomicAdd(&cnt[(sK[p] >> shift) & 0xFF], 1u);
      __syncthreads();
      {
        uint32_t tot;
        const uint32_t ex = block_excl_scan<uint32_t>(cnt[tid], ws, &tot);
        __syncthreads();
        cnt[tid] = ex;  // running output offset of each digit
      }
      __syncthreads();
      const uint64_t lt = lanemask_lt();
      for (uint64_t c = lo; c < hi; c += kThreads) {
        for (uint32_t q = tid; q < 4 * kRadix; q += kThreads) (&wc[0][0])[q] = 0;
        __syncthreads();
        const uint64_t p = c + tid;
        const bool ok = p < hi;
        const uint64_t k = ok ? sK[p] : ~0ull;
        const uint32_t v = ok ? sV[p] : 0u;
        const uint32_t d = ok ? (uint32_t)(k >> shift) & 0xFF : 0xFFu;
        const uint64_t peers = match_digit(d);
        const uint32_t before = __popcll(peers & lt);
        if ((peers >> lane) == 1ull) wc[wave][d] = __popcll(peers);
        __syncthreads();
        uint32_t cross = 0;
        for (uint32_t w = 0; w < wave; ++w) cross += wc[w][d];
        if (ok) {
          const uint64_t dst = lo + cnt[d] + cross + before;
          dK[dst] = k;
          dV[dst] = v;
        }
        __syncthreads();
        {
          const uint32_t dd = tid;
          cnt[dd] += wc[0][dd] + wc[1][dd] + wc[2][dd] + wc[3][dd];
        }
        __syncthreads();
      }
      uint64_t* t1 = sK; sK = dK; dK = t1;
      uint32_t* t2 = sV; sV = dV; dV = t2;
    }
    if (sK != K) {  // odd number of passes: the sorted data is in the scratch arrays
      for (uint64_t p = lo + tid; p < hi; p += kThreads) {
        K[p] = sK[p];
        V[p] = sV[p];
      }
      __syncthreads();
    }
  }
  // Account buckets, scanning the range in chunks of kThreads with the
  // currently open run carried across chunks.
  BucketTotals tot{0ull, 0u, kNoStation, 0u};
  if (tid == 0) s_carry = 0;
  __syncthreads();
  uint8_t* marks = a.marks + off;
  for (uint64_t p = lo + tid; p < hi; p += kThreads) marks[p] = 0;
  __syncthreads();
  auto emit = [&](uint64_t s, uint64_t e) {
    const int cls = bucket_account(a, e - s, [&](uint64_t q) { return V[s + q]; }, V[s], K[s], tot);
    if (cls == 1) {
      marks[s] = (uint8_t)(e - s);
    } else if (cls == 2) {
      const uint32_t q = atomicAdd(a.big_count, 1u);
      a.big_desc[q] = make_uint4((uint32_t)s, seg, (uint32_t)(e - s), 0);
    }
  };
  for (uint64_t c = lo; c < hi; c += kThreads) {
    const uint64_t p = c + tid;
    const uint32_t h = (p < hi && p > lo && K[p] != K[p - 1]) ? 1u : 0u;
    uint32_t nh;
    const uint32_t x = block_excl_scan<uint32_t>(h, ws, &nh);
    if (h) heads[x] = (uint32_t)(p - lo);
    __syncthreads();
    const uint32_t carry = s_carry;
    for (uint32_t q = tid; q < nh; q += kThreads) {
      const uint64_t s = lo + (q == 0 ? carry : heads[q - 1]);
      emit(s, lo + heads[q]);
    }
    __syncthreads();
    if (tid == 0 && nh) s_carry = heads[nh - 1];
    __syncthreads();
  }
  if (tid == 0) emit(lo + s_carry, hi);
  flush_totals(a, tot);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
// Radix tile shapes (threads x items): 1024 x 16, 512 x 16, 256 x 16.
uint32_t radix_tile_elems(uint32_t variant) { return variant == 0 ? 16384u : (variant == 1 ? 8192u : 4096u); }

uint32_t radix_tiles(uint64_t n, uint32_t variant) {
  const uint64_t e = radix_tile_elems(variant);
  return (uint32_t)((n + e - 1) / e);
}

template <typename T>
static void seg_scan(T* data, uint64_t len, uint32_t S, T* sums, T* seg_total, hipStream_t s) {
  const uint32_t nblk = (uint32_t)((len + kScanBlock - 1) / kScanBlock);
  if (nblk == 0) return;
  hipLaunchKernelGGL((k_scan_sums<T>), dim3(nblk, S), dim3(kThreads), 0, s, data, len, sums, nblk);
  hipLaunchKernelGGL((k_scan_blocksums<T>), dim3(S), dim3(kThreads), 0, s, sums, nblk, seg_total);
  hipLaunchKernelGGL((k_scan_apply<T>), dim3(nblk, S), dim3(kThreads), 0, s, data, len, sums, nblk);
}

uint64_t scan_sums_elems(uint64_t len, uint32_t S) { return ((len + kScanBlock - 1) / kScanBlock) * S + 1; }

void scan_u32(uint32_t* data, uint64_t len, uint32_t S, uint32_t* sums, uint32_t* seg_total, hipStream_t s) {
  seg_scan<uint32_t>(data, len, S, sums, seg_total, s);
}
void scan_u64(uint64_t* data, uint64_t len, uint32_t S, uint64_t* sums, uint64_t* seg_total, hipStream_t s) {
  seg_scan<uint64_t>(reinterpret_cast<uint64_t*>(data), len, S, sums, seg_total, s);
}

// The three launches of one pass for one tile shape.
template <int TH, int IT>
static void radix_pass_t(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, uint64_t n,
                         uint32_t S, uint32_t shift, uint32_t* hist, uint32_t* sums, uint32_t nt, hipStream_t s) {
  hipLaunchKernelGGL((k_hist<TH, IT>), dim3(nt, S), dim3(TH), 0, s, kin, n, shift, hist, nt);
  seg_scan<uint32_t>(hist, (uint64_t)kRadix * nt, S, sums, nullptr, s);
  hipLaunchKernelGGL((k_scatter<TH, IT>), dim3(nt, S), dim3(TH), 0, s, kin, vin, kout, vout, n, shift, hist, nt);
}

// One stable pass by the 8-bit digit at `shift`; hist needs 256 * tiles * S
// entries for the variant's tile count.
void radix_pass(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, uint64_t n, uint32_t S,
                uint32_t shift, uint32_t* hist, uint32_t* sums, uint32_t variant, hipStream_t s) {
  if (n == 0) return;
  const uint32_t nt = radix_tiles(n, variant);
  switch (variant) {
    case 0: radix_pass_t<1024, 16>(kin, vin, kout, vout, n, S, shift, hist, sums, nt, s); break;
    case 1: radix_pass_t<512, 16>(kin, vin, kout, vout, n, S, shift, hist, sums, nt, s); break;
    default: radix_pass_t<256, 16>(kin, vin, kout, vout, n, S, shift, hist, sums, nt, s); break;
  }
}

// Compute units of the current device (queried once).
uint32_t device_cus() {
  static uint32_t cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cus = (uint32_t)v;
  }
  return cus;
}

// Most descriptor slots the bucket kernel reserves beyond the big buckets it
// finds, for S segments: every wave's last reservation, and at most two
// slots lost per reservation (a request holds at most three descriptors).
uint64_t bucket_desc_slack(uint64_t big_max, uint32_t S) {
  const uint64_t waves = (uint64_t)kBucketWaves * std::max<uint64_t>(S, 8ull * device_cus());
  return waves * kSlab + 2 * ((big_max + waves * kSlab) / (kSlab - 2) + 1);
}

// Persistent: one resident round of workgroups (as many as the LDS of the
// staged spans lets a CU hold, at most 8) spread over the segments.
void launch_bucket(const BucketArgs& a, uint32_t S, hipStream_t s) {
  if (a.n == 0) return;
  const uint32_t nspans = (uint32_t)((a.n + a.chunk - 1) / a.chunk);
  const size_t lds = (size_t)kBucketWaves * (a.chunk + kSpanExt + 1) * 12;
  const uint32_t per_cu = (uint32_t)std::max<size_t>(1, std::min<size_t>(8, (160u << 10) / lds));
  const uint32_t need = (nspans + kBucketWaves - 1) / kBucketWaves;
  const uint32_t per_seg = std::max<uint32_t>(1u, std::min<uint32_t>(need, per_cu * device_cus() / S));
  hipLaunchKernelGGL(k_bucket, dim3(per_seg, S), dim3(kBucketWaves * 64), lds, s, a, nspans);
}

void launch_bigbin(const BucketArgs& a, const uint4* bins, uint32_t grid, uint64_t* tk, uint32_t* tv,
                   hipStream_t s) {
  if (a.n == 0 || grid == 0) return;
  hipLaunchKernelGGL(k_bigbin, dim3(grid), dim3(kThreads), 0, s, a, bins, tk, tv);
}

// Mixed keys of tables [tb, tb + tc) rebuilt from what an earlier signature
// pass stored, for keys of the form mix48(band key) << 16: the high word
// (bits 32-63, hi32[u][i]) and the sub-key (bits 16-31, field u mod TG of the
// row of table u's group, rows row_pitch dwords apart).  One thread per
// fingerprint.
__global__ __launch_bounds__(256) void k_split_keys(const uint32_t* hi32, const uint32_t* rows, uint64_t n,
                                                    uint32_t tb, uint32_t tc, uint32_t tables_per_group,
                                                    uint32_t row_pitch, uint64_t* mkeys) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    for (uint32_t q = 0; q < tc; ++q) {
      const uint32_t u = tb + q, g = u / tables_per_group, k = u - g * tables_per_group;
      const uint32_t w = rows[((uint64_t)g * n + i) * row_pitch + (k >> 1)];
      const uint64_t field = (w >> (16 * (k & 1))) & 0xFFFFu;
      mkeys[(uint64_t)q * n + i] = ((uint64_t)hi32[(uint64_t)u * n + i] << 32) | (field << 16);
    }
  }
}

void launch_split_keys(const uint32_t* hi32, const uint32_t* rows, uint64_t n, uint32_t tb, uint32_t tc,
                       uint32_t tables_per_group, uint32_t row_pitch, uint64_t* mkeys, hipStream_t s) {
  if (n == 0 || tc == 0) return;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_split_keys, dim3((unsigned)(blocks < 65535 ? blocks : 65535)), dim3(256), 0, s, hi32, rows, n,
                     tb, tc, tables_per_group, row_pitch, mkeys);
}

}  // namespace fl
