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
// ---------------------------------------------------------------------------
// Elements one bucket workgroup holds in LDS: 7 per thread, an odd count so
// that threads walking their own consecutive elements start on different
// LDS banks.  Chunks are at most 1536 positions, so the bins that start in a
// chunk (all but its last) always fit.
constexpr int kBinCap = 1792;
constexpr uint32_t kRankMax = 128;  // largest mixed bin ranked in LDS

__device__ __forceinline__ bool kv_less(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb) {
  return ka < kb || (ka == kb && va < vb);
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
  uint32_t ns;  // fingerprints of `station`
};

// Account one bucket (run of equal keys) of `size` members; ids(q) gives the
// q-th member (ascending).  Returns the descriptor class: 0 none, 1 small,
// 2 big.  Buckets that cannot hold a reportable pair get no descriptor: a
// single member, every member excluded by the occurrence filter (the bucket
// itself is over the threshold), or an id span below the lag.
template <typename IdAt>
__device__ __forceinline__ int bucket_account(const BucketArgs& a, uint64_t size, IdAt ids, uint32_t first_id,
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
    tot.ns = (uint32_t)(a.station_base[st + 1] - a.station_base[st]);
  }
  tot.e_raw += (unsigned long long)(size * (size - 1) / 2);
  if (size > tot.max_bucket) tot.max_bucket = (unsigned int)size;
  if (a.occ_den) {
    const uint64_t ns = tot.ns;
    if ((unsigned __int128)size * a.occ_den > (unsigned __int128)ns * a.occ_num) {
      for (uint64_t q = 0; q < size; ++q) a.flags[ids(q)] = 1;
      return 0;
    }
  }
  if (size < 2 || ids(size - 1) - first_id < a.min_lag) return 0;
  return size <= a.small_max ? 1 : 2;
}

// The descriptor class bucket_account returns, without side effects.
__device__ __forceinline__ int bucket_class(const BucketArgs& a, uint64_t size, uint32_t first_id, uint32_t last_id,
                                            uint64_t key) {
  if (a.occ_den) {
    const uint32_t st = a.nstation > 1 ? (uint32_t)(key >> 60) : 0u;
    const uint64_t ns = a.station_base[st + 1] - a.station_base[st];
    if ((unsigned __int128)size * a.occ_den > (unsigned __int128)ns * a.occ_num) return 0;
  }
  if (size < 2 || last_id - first_id < a.min_lag) return 0;
  return size <= a.small_max ? 1 : 2;
}

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

// End of the run of equal keys starting at e inside bin b0: the bin's end
// for a single-key bin, else a short scan (mixed bins here hold at most
// kRankMax elements).
__device__ __forceinline__ uint32_t run_end(const uint64_t* sk, uint32_t e, uint32_t b0, const uint16_t* be,
                                            const uint8_t* mixed) {
  const uint32_t b1 = be[b0];
  if (!mixed[b0]) return b1;
  uint32_t f = e + 1;
  while (f < b1 && sk[f] == sk[e]) ++f;
  return f;
}

// Copy positions [lo, lo + m) of segment seg (m <= kBinCap) into sk / sv,
// consecutive lanes on consecutive elements.
__device__ void load_bins(const BucketArgs& a, uint32_t seg, uint64_t lo, uint32_t m, uint64_t* sk, uint32_t* sv) {
  const uint64_t* K = a.keys + (uint64_t)seg * a.n;
  const uint32_t* V = a.vals + (uint64_t)seg * a.n;
#pragma unroll
  for (uint32_t q = 0; q < kBinCap / kThreads; ++q) {
    const uint32_t e = q * kThreads + threadIdx.x;
    if (e < m) {
      sk[e] = K[lo + e];
      sv[e] = V[lo + e];
    }
  }
  __syncthreads();
}

// Order positions [lo, lo + m) of segment seg (whole bins, already in
// sk / sv) by (key, id) in LDS, write the ids back in that order, and
// account every bucket.  Elements arrive grouped by bin with ids ascending
// inside a bin, so a bin holding a single key is already in order; only
// bins that mix keys are ranked, by counting the (key, position) pairs
// below each element.
__device__ void process_bins(const BucketArgs& a, uint32_t seg, uint64_t lo, uint32_t m, uint64_t* sk, uint32_t* sv,
                             uint16_t* bs, uint16_t* be, uint16_t* np, uint8_t* mixed, uint32_t* sh,
                             BucketTotals& tot) {
  uint32_t* V = a.vals + (uint64_t)seg * a.n;
  const uint32_t bsh = a.bin_shift;
  constexpr uint32_t kPer = kBinCap / kThreads;  // elements per thread, consecutive
  const uint32_t e0 = threadIdx.x * kPer;
  for (uint32_t e = threadIdx.x; e < m; e += kThreads) mixed[e] = 0;  // read only after the barriers below
  // Each thread's running bin start over its own consecutive elements.
  uint32_t run = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t e = e0 + q;
    if (e < m && (e == 0 || (sk[e] >> bsh) != (sk[e - 1] >> bsh))) run = e;
  }
  // Exclusive max-scan of the per-thread last head gives the open bin start.
  uint32_t carry = run;
  {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = carry;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, 64);
      if (lane >= (uint32_t)o) inc = max(inc, y);
    }
    if (lane == 63) sh[8 + wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t w = 0; w < wave; ++w) before = max(before, sh[8 + w]);
    const uint32_t prev = __shfl_up(inc, 1, 64);
    carry = max(before, lane ? prev : 0u);
    __syncthreads();
  }
  uint32_t cur = carry;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t e = e0 + q;
    if (e < m) {
      if (e == 0 || (sk[e] >> bsh) != (sk[e - 1] >> bsh)) cur = e;
      bs[e] = (uint16_t)cur;
      if (e + 1 == m || (sk[e + 1] >> bsh) != (sk[e] >> bsh)) be[cur] = (uint16_t)(e + 1);
      if (sk[e] != sk[cur]) mixed[cur] = 1;
    }
  }
  __syncthreads();
  // Mixed bins above kRankMax elements are left in id order and handed to
  // the single-workgroup path (k_bigbin): ranking them here costs O(m^2).
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t e = e0 + q;
    if (e < m && bs[e] == e && mixed[e] && be[e] - e > kRankMax) {
      mixed[e] = 2;
      const uint32_t slot = atomicAdd(a.bin_count, 1u);
      a.bin_desc[slot] = make_uint4((uint32_t)(lo + e), (uint32_t)(lo + be[e]), seg, 0);
    }
  }
  __syncthreads();
  // Rank inside mixed bins.
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t e = e0 + q;
    if (e < m) {
      const uint32_t b0 = bs[e];
      uint32_t pos = e;
      if (mixed[b0] == 1) {
        const uint32_t b1 = be[b0];
        const uint64_t k = sk[e];
        pos = b0;
        for (uint32_t f = b0; f < b1; ++f) {
          const uint64_t kf = sk[f];
          pos += (kf < k) || (kf == k && f < e);
        }
      }
      np[e] = (uint16_t)pos;
    }
  }
  __syncthreads();
  uint64_t rk[kPer];
  uint32_t rv[kPer];
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t e = e0 + q;
    rk[q] = e < m ? sk[e] : 0ull;
    rv[q] = e < m ? sv[e] : 0u;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t e = e0 + q;
    if (e < m) {
      sk[np[e]] = rk[q];
      sv[np[e]] = rv[q];
    }
  }
  __syncthreads();
  // only bins that mixed keys changed order
  for (uint32_t e = threadIdx.x; e < m; e += blockDim.x)
    if (mixed[bs[e]] == 1) V[lo + e] = sv[e];
  // Buckets: every position gets its mark (the size of a small pair-capable
  // bucket starting there, else 0); large buckets go to a list.
  uint8_t* marks = a.marks + (uint64_t)seg * a.n + lo;
  uint32_t nbig = 0;
  for (uint32_t e = threadIdx.x; e < m; e += blockDim.x) {
    const uint32_t b0 = bs[e];
    if (mixed[b0] == 2) continue;
    uint8_t mk = 0;
    if (e == 0 || sk[e] != sk[e - 1]) {
      const uint32_t f = run_end(sk, e, b0, be, mixed);
      const int cls = bucket_account(a, f - e, [&](uint64_t q) { return sv[e + q]; }, sv[e], sk[e], tot);
      if (cls == 1) mk = (uint8_t)(f - e);
      nbig += cls == 2;
    }
    marks[e] = mk;
  }
  uint32_t* ws = sh;        // 4 entries
  uint32_t* base = sh + 4;  // 1 entry
  uint32_t tbig;
  const uint32_t xb = block_excl_scan<uint32_t>(nbig, ws, &tbig);
  if (tbig) {
    if (threadIdx.x == 0) base[0] = atomicAdd(a.big_count, tbig);
    __syncthreads();
    uint32_t pb = base[0] + xb;
    if (nbig) {
      for (uint32_t e = threadIdx.x; e < m; e += blockDim.x) {
        const uint32_t b0 = bs[e];
        if (mixed[b0] == 2) continue;
        if (e > 0 && sk[e] == sk[e - 1]) continue;
        const uint32_t f = run_end(sk, e, b0, be, mixed);
        if (bucket_class(a, f - e, sv[e], sv[f - 1], sk[e]) == 2)
          a.big_desc[pb++] = make_uint4((uint32_t)(lo + e), seg, f - e, 0);
      }
    }
  }
  __syncthreads();
}

// Persistent over the chunks of one segment (table): chunk c covers
// positions [c * chunk, (c + 1) * chunk) and owns the bins that start in it.
// Its window, one position before the chunk up to kBinCap positions, is
// staged in LDS in one pass; bin boundaries, the end of its last bin (when
// inside the window) and the buckets all come from there, while the next
// chunk's window is already being read into registers.
__global__ __launch_bounds__(kThreads, 4) void k_bucket(BucketArgs a, uint32_t nchunks) {
  __shared__ uint64_t sk[kBinCap];
  __shared__ uint32_t sv[kBinCap];
  __shared__ uint16_t bs[kBinCap], be[kBinCap], np[kBinCap];
  __shared__ uint8_t mixed[kBinCap];
  __shared__ uint32_t sh[16];
  __shared__ unsigned long long s_hi;
  __shared__ int s_first, s_last, s_end;
  constexpr uint32_t kPer = kBinCap / kThreads;
  const uint32_t seg = blockIdx.y;
  const uint32_t bsh = a.bin_shift;
  const uint64_t n = a.n;
  const uint64_t* K = a.keys + (uint64_t)seg * n;
  const uint32_t* V = a.vals + (uint64_t)seg * n;
  uint64_t pk[kPer];
  uint32_t pv[kPer];
  auto window = [&](uint32_t c) -> uint64_t { return c ? (uint64_t)c * a.chunk - 1 : 0ull; };
  auto fetch = [&](uint32_t c) {
    const uint64_t w0 = window(c);
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      const uint64_t p = w0 + q * kThreads + threadIdx.x;
      pk[q] = p < n ? K[p] : 0ull;
      pv[q] = p < n ? V[p] : 0u;
    }
  };
  BucketTotals tot{0ull, 0u, kNoStation, 0u};
  uint32_t c = blockIdx.x;
  if (c < nchunks) fetch(c);
  for (; c < nchunks; c += gridDim.x) {
    const uint64_t c0 = (uint64_t)c * a.chunk;
    const uint64_t c1 = c0 + a.chunk < n ? c0 + a.chunk : n;
    const uint64_t w0 = window(c);
    const uint32_t wn = (uint32_t)(n - w0 < (uint64_t)kBinCap ? n - w0 : (uint64_t)kBinCap);
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      const uint32_t e = q * kThreads + threadIdx.x;
      if (e < wn) {
        sk[e] = pk[q];
        sv[e] = pv[q];
      }
    }
    if (threadIdx.x == 0) {
      s_first = 0x7FFFFFFF;
      s_last = -1;
      s_end = 0x7FFFFFFF;
    }
    __syncthreads();
    if (c + gridDim.x < nchunks) fetch(c + gridDim.x);
    // Bin heads: the first and last inside the chunk, and the first at or
    // after its end (the end of its last bin), as window offsets.
    {
      const uint32_t cb = (uint32_t)(c0 - w0), ce = (uint32_t)(c1 - w0);
      int first = 0x7FFFFFFF, lastp = -1, endp = 0x7FFFFFFF;
#pragma unroll
      for (uint32_t q = 0; q < kPer; ++q) {
        const uint32_t e = q * kThreads + threadIdx.x;
        if (e >= cb && e < wn && (w0 + e == 0 || (sk[e] >> bsh) != (sk[e - 1] >> bsh))) {
          if (e < ce) {
            first = min(first, (int)e);
            lastp = max(lastp, (int)e);
          } else {
            endp = min(endp, (int)e);
          }
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        first = min(first, __shfl_xor(first, o, 64));
        lastp = max(lastp, __shfl_xor(lastp, o, 64));
        endp = min(endp, __shfl_xor(endp, o, 64));
      }
      if ((threadIdx.x & 63) == 0) {
        if (first != 0x7FFFFFFF) atomicMin(&s_first, first);
        if (lastp >= 0) atomicMax(&s_last, lastp);
        if (endp != 0x7FFFFFFF) atomicMin(&s_end, endp);
      }
    }
    __syncthreads();
    const int first = s_first, lastp = s_last, endp = s_end;
    __syncthreads();  // the next chunk's thread 0 resets these
    if (first == 0x7FFFFFFF) continue;  // no bin starts in this chunk
    const uint64_t lo = w0 + (uint64_t)first;
    if (endp != 0x7FFFFFFF || w0 + wn == n) {  // the last bin ends inside the window
      const uint64_t hi = endp != 0x7FFFFFFF ? w0 + (uint64_t)endp : n;
      process_bins(a, seg, lo, (uint32_t)(hi - lo), sk + first, sv + first, bs, be, np, mixed, sh, tot);
      continue;
    }
    // The last bin runs past the window: the bins before it from LDS, then
    // its end from HBM, and the bin itself from HBM or the big-bin list.
    const uint64_t last = w0 + (uint64_t)lastp;
    if (lastp > first)
      process_bins(a, seg, lo, (uint32_t)(last - lo), sk + first, sv + first, bs, be, np, mixed, sh, tot);
    if (threadIdx.x == 0) {
      const uint64_t binlast = sk[lastp] >> bsh;
      uint64_t L = w0 + wn, R = n;  // first p in [L, R) with bin(p) > binlast
      while (L < R) {
        const uint64_t M = (L + R) / 2;
        if ((K[M] >> bsh) > binlast) R = M; else L = M + 1;
      }
      s_hi = L;
    }
    __syncthreads();
    const uint64_t hi = s_hi;
    __syncthreads();
    if (hi - last <= (uint64_t)kBinCap) {
      load_bins(a, seg, last, (uint32_t)(hi - last), sk, sv);
      process_bins(a, seg, last, (uint32_t)(hi - last), sk, sv, bs, be, np, mixed, sh, tot);
    } else if (threadIdx.x == 0) {
      const uint32_t q = atomicAdd(a.bin_count, 1u);
      a.bin_desc[q] = make_uint4((uint32_t)last, (uint32_t)hi, seg, 0);
    }
    __syncthreads();
  }
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
static uint32_t device_cus() {
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

// Persistent: one resident round of workgroups (the LDS of four fits a CU)
// spread over the segments.
void launch_bucket(const BucketArgs& a, uint32_t S, hipStream_t s) {
  if (a.n == 0) return;
  const uint32_t nch = (uint32_t)((a.n + a.chunk - 1) / a.chunk);
  const uint32_t per_seg = std::max<uint32_t>(1u, std::min<uint32_t>(nch, 4 * device_cus() / S));
  hipLaunchKernelGGL(k_bucket, dim3(per_seg, S), dim3(kThreads), 0, s, a, nch);
}

void launch_bigbin(const BucketArgs& a, const uint4* bins, uint32_t grid, uint64_t* tk, uint32_t* tv,
                   hipStream_t s) {
  if (a.n == 0 || grid == 0) return;
  hipLaunchKernelGGL(k_bigbin, dim3(grid), dim3(kThreads), 0, s, a, bins, tk, tv);
}

}  // namespace fl
