// Serving form of the similarity search: stations whose hash tables stay
// resident in HBM, and chunks of new fingerprints that are searched against
// everything the station holds as they arrive, then inserted (the paper's
// query-only use of the tables, section 6.4, on a growing station).
//
// A chunk's result is every pair (i, j) with j in the chunk, i < j anywhere
// in the station (history, earlier chunks, or the chunk itself), j - i at
// least the lag, and at least v shared buckets over the t tables: the union
// over chunks equals the search over the concatenated station.
//
// Resident per station and table: the (mixed key, id) pairs of the history
// sorted by (key, id), and a sorted delta of the chunks inserted since the
// last merge.  Per batch of chunks (one per station at most):
//   1. signatures of the batch's rows (mixed keys, table-major);
//   2. each chunk sorted per table in LDS (bitonic);
//   3. one workgroup per query row: in every table it finds its bucket in
//      the history, the delta and its own chunk by binary search (ids inside
//      a bucket are ascending, so the lag bound is one more binary search),
//      and counts the votes of every earlier member exactly in an LDS hash
//      table; queries with more members than the table holds are counted in
//      id windows, each holding every occurrence of its ids;
//   4. each chunk is merged into its station's delta; a full delta is first
//      merged into the history.
// A host worker thread forms the batches from the chunks waiting (continuous
// batching) and runs them on the server's stream.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "host.hpp"

namespace fl {

constexpr int kChunkMax = 4096;   // rows per chunk (one LDS bitonic sort)
constexpr int kQT = 256;          // threads per query workgroup
constexpr int kHashSlots = 8192;  // LDS vote table
constexpr uint32_t kQueryCap = 4096;  // members counted per pass (load factor <= 1/2)
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kStatSlots = 64;   // spread of the per-chunk counters

struct ServeEntry {
  const uint64_t* hkey;  // history [t][hstride], first nh sorted
  const uint32_t* hid;
  uint64_t hstride, nh;
  const uint64_t* dkey;  // delta [t][dstride], first nd sorted
  const uint32_t* did;
  uint64_t dstride, nd;
  uint32_t cbase, nq;  // the chunk's rows are batch rows [cbase, cbase + nq)
  uint32_t id0, pad;   // station id of the chunk's first row
};

struct QueryArgs {
  const ServeEntry* ent;
  uint32_t nent;
  uint32_t Qtot, t;
  const uint64_t* ckeys;  // [t][Qtot] mixed keys of the batch rows
  const uint64_t* csk;    // [t][Qtot] each chunk sorted per table
  const uint32_t* csid;
  uint32_t min_lag, min_votes;
  uint32_t* out_h;
  uint32_t* out_q;
  uint8_t* out_v;
  uint8_t* out_e;
  unsigned int* out_count;
  uint32_t out_cap;
  unsigned long long* stats;  // [nent][kStatSlots][4]: e_raw, e_voted, n_distinct, max bucket
};

__device__ __forceinline__ bool kv_lt(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb) {
  return ka < kb || (ka == kb && va < vb);
}

// First position in sorted k[0, n) whose key is >= key (upper: > key).
__device__ __forceinline__ uint64_t key_bound(const uint64_t* k, uint64_t n, uint64_t key, bool upper) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t m = (lo + hi) >> 1;
    if (upper ? k[m] <= key : k[m] < key) lo = m + 1; else hi = m;
  }
  return lo;
}

// Number of entries of ascending ids[0, n) below x.
__device__ __forceinline__ uint32_t ids_below(const uint32_t* ids, uint32_t n, uint64_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t m = (lo + hi) >> 1;
    if ((uint64_t)ids[m] < x) lo = m + 1; else hi = m;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// 2. Sort each chunk's (key, id) per table: workgroup (table, entry).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sort_chunk(const ServeEntry* ent, const uint64_t* ckeys, uint64_t* csk,
                                                    uint32_t* csid, uint32_t Qtot) {
  __shared__ uint64_t sk[kChunkMax];
  __shared__ uint32_t sv[kChunkMax];
  const ServeEntry e = ent[blockIdx.y];
  const uint32_t u = blockIdx.x;
  uint32_t P = 1;
  while (P < e.nq) P <<= 1;
  const uint64_t base = (uint64_t)u * Qtot + e.cbase;
  for (uint32_t k = threadIdx.x; k < P; k += 256) {
    const bool ok = k < e.nq;
    sk[k] = ok ? ckeys[base + k] : ~0ull;
    sv[k] = ok ? e.id0 + k : kEmpty;  // padding sorts last (ids are below 2^31)
  }
  __syncthreads();
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < P; i += 256) {
        const uint32_t j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const bool gt = kv_lt(sk[j], sv[j], sk[i], sv[i]);
          if (gt == up) {
            const uint64_t tk = sk[i];
            sk[i] = sk[j];
            sk[j] = tk;
            const uint32_t tv = sv[i];
            sv[i] = sv[j];
            sv[j] = tv;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t k = threadIdx.x; k < e.nq; k += 256) {
    csk[base + k] = sk[k];
    csid[base + k] = sv[k];
  }
}

// ---------------------------------------------------------------------------
// 3. Votes of one query row against everything before it.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  T s = 0;
  for (uint32_t w = 0; w < kQT / 64; ++w) s += scratch[w];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(kQT) void k_query(QueryArgs a) {
  __shared__ uint32_t rbeg[3 * 256];      // member range of (table, source): start in its id array
  __shared__ uint32_t rcnt[3 * 256];      // its length (ids at or below the lag bound)
  __shared__ uint32_t wbeg[3 * 256];      // sub-range inside the current id window
  __shared__ uint32_t wpre[3 * 256 + 1];  // exclusive prefix of the window's lengths
  __shared__ uint32_t hk[kHashSlots];
  __shared__ uint32_t hc[kHashSlots];
  __shared__ unsigned long long red[kQT / 64];
  const uint32_t q = blockIdx.x;
  uint32_t e = 0;
  while (e + 1 < a.nent && a.ent[e + 1].cbase <= q) ++e;
  const ServeEntry E = a.ent[e];
  const uint32_t k = q - E.cbase;
  const uint32_t id = E.id0 + k;
  // members h < id with id - h >= min_lag: h <= id - max(min_lag, 1)
  const uint32_t gap = a.min_lag > 1 ? a.min_lag : 1u;
  const bool any = id >= gap;
  const uint64_t lim = any ? (uint64_t)id - gap : 0;  // allowed member ids: <= lim
  const uint32_t R = 3 * a.t;

  // Ranges of the query's bucket in history, delta and chunk, per table.
  unsigned long long raw = 0, mb = 0;
  for (uint32_t u = threadIdx.x; u < a.t; u += kQT) {
    const uint64_t key = a.ckeys[(uint64_t)u * a.Qtot + q];
    uint64_t bucket = 0;
    {  // history
      const uint64_t* kk = E.hkey + (uint64_t)u * E.hstride;
      const uint32_t* ii = E.hid + (uint64_t)u * E.hstride;
      const uint64_t lo = key_bound(kk, E.nh, key, false), hi = key_bound(kk, E.nh, key, true);
      raw += hi - lo;
      bucket += hi - lo;
      rbeg[3 * u] = (uint32_t)lo;
      rcnt[3 * u] = any ? ids_below(ii + lo, (uint32_t)(hi - lo), lim + 1) : 0u;
    }
    {  // delta
      const uint64_t* kk = E.dkey + (uint64_t)u * E.dstride;
      const uint32_t* ii = E.did + (uint64_t)u * E.dstride;
      const uint64_t lo = key_bound(kk, E.nd, key, false), hi = key_bound(kk, E.nd, key, true);
      raw += hi - lo;
      bucket += hi - lo;
      rbeg[3 * u + 1] = (uint32_t)lo;
      rcnt[3 * u + 1] = any ? ids_below(ii + lo, (uint32_t)(hi - lo), lim + 1) : 0u;
    }
    {  // own chunk: members before the query
      const uint64_t* kk = a.csk + (uint64_t)u * a.Qtot + E.cbase;
      const uint32_t* ii = a.csid + (uint64_t)u * a.Qtot + E.cbase;
      const uint64_t lo = key_bound(kk, E.nq, key, false), hi = key_bound(kk, E.nq, key, true);
      raw += ids_below(ii + lo, (uint32_t)(hi - lo), id);
      bucket += hi - lo;
      rbeg[3 * u + 2] = (uint32_t)lo;
      rcnt[3 * u + 2] = any ? ids_below(ii + lo, (uint32_t)(hi - lo), lim + 1) : 0u;
    }
    mb = bucket > mb ? bucket : mb;
  }
  __syncthreads();

  auto ids_of = [&](uint32_t r) -> const uint32_t* {
    const uint32_t u = r / 3, s = r - 3 * u;
    if (s == 0) return E.hid + (uint64_t)u * E.hstride;
    if (s == 1) return E.did + (uint64_t)u * E.dstride;
    return a.csid + (uint64_t)u * a.Qtot + E.cbase;
  };

  unsigned long long ev = 0, nd = 0;
  uint64_t w_lo = 0;
  const uint64_t w_end = any ? lim + 1 : 0;
  while (w_lo < w_end) {
    // Largest window [w_lo, w_hi) holding at most kQueryCap members.
    uint64_t w_hi = w_end;
    uint32_t total;
    for (;;) {
      uint32_t c = 0;
      for (uint32_t r = threadIdx.x; r < R; r += kQT) {
        const uint32_t* ii = ids_of(r) + rbeg[r];
        const uint32_t n = rcnt[r];
        const uint32_t b0 = w_lo ? ids_below(ii, n, w_lo) : 0u;
        const uint32_t b1 = w_hi == w_end ? n : ids_below(ii, n, w_hi);
        wbeg[r] = rbeg[r] + b0;
        wpre[r] = b1 - b0;
        c += b1 - b0;
      }
      total = (uint32_t)block_sum<unsigned long long>(c, red);
      if (total <= kQueryCap || w_hi - w_lo <= 1) break;
      w_hi = w_lo + (w_hi - w_lo) / 2;
    }
    if (total) {
      // exclusive prefix of the window lengths (one thread: at most 765 entries)
      if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t r = 0; r < R; ++r) {
          const uint32_t n = wpre[r];
          wpre[r] = s;
          s += n;
        }
        wpre[R] = s;
      }
      for (uint32_t x = threadIdx.x; x < kHashSlots; x += kQT) {
        hk[x] = kEmpty;
        hc[x] = 0;
      }
      __syncthreads();
      for (uint32_t m = threadIdx.x; m < total; m += kQT) {
        uint32_t lo = 0, hi = R;  // last r with wpre[r] <= m
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (wpre[mid] <= m) lo = mid; else hi = mid;
        }
        const uint32_t h = ids_of(lo)[wbeg[lo] + (m - wpre[lo])];
        uint32_t slot = (h * 0x9E3779B1u) >> (32 - 13);
        for (;;) {
          const uint32_t prev = atomicCAS(&hk[slot], kEmpty, h);
          if (prev == kEmpty || prev == h) {
            atomicAdd(&hc[slot], 1u);
            break;
          }
          slot = (slot + 1) & (kHashSlots - 1);
        }
      }
      __syncthreads();
      for (uint32_t x = threadIdx.x; x < kHashSlots; x += kQT) {
        const uint32_t h = hk[x];
        if (h == kEmpty) continue;
        const uint32_t c = hc[x];
        ev += c;
        nd += 1;
        if (c >= a.min_votes) {
          const uint32_t p = atomicAdd(a.out_count, 1u);
          if (p < a.out_cap) {
            a.out_h[p] = h;
            a.out_q[p] = id;
            a.out_v[p] = (uint8_t)c;
            a.out_e[p] = (uint8_t)e;
          }
        }
      }
      __syncthreads();
    }
    w_lo = w_hi;
  }

  raw = block_sum<unsigned long long>(raw, red);
  ev = block_sum<unsigned long long>(ev, red);
  nd = block_sum<unsigned long long>(nd, red);
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(mb, o, 64);
    mb = y > mb ? y : mb;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(&a.stats[((uint64_t)e * kStatSlots + q % kStatSlots) * 4 + 3], mb);
  if (threadIdx.x == 0) {
    unsigned long long* s = a.stats + ((uint64_t)e * kStatSlots + q % kStatSlots) * 4;
    atomicAdd(s + 0, raw);
    atomicAdd(s + 1, ev);
    atomicAdd(s + 2, nd);
  }
}

// ---------------------------------------------------------------------------
// 4. Merge of a long sorted (key, id) run A and a short one B per table
// segment (ids are unique, so no two elements compare equal).  Each element
// of B finds its rank in A (the elements of A below it) by bisection and goes
// straight to its place.  The ranks are non-decreasing, so an element of A
// moves up by the number of ranks at or below its index: a block of A reads
// the slice of ranks that fall in its range into LDS once.
// ---------------------------------------------------------------------------
constexpr uint32_t kMergeBlock = 2048;  // elements of A per block
constexpr uint32_t kMergeSlice = 2048;  // ranks a block holds in LDS

__global__ __launch_bounds__(256) void k_merge_rank(const uint64_t* ak, const uint32_t* av, uint64_t as, uint64_t nA,
                                                    const uint64_t* bk, const uint32_t* bv, uint64_t bs, uint64_t nB,
                                                    uint64_t* ok, uint32_t* ov, uint64_t os, uint32_t* rk) {
  const uint64_t u = blockIdx.y;
  const uint64_t* A = ak + u * as;
  const uint32_t* AV = av + u * as;
  const uint64_t* B = bk + u * bs;
  const uint32_t* BV = bv + u * bs;
  for (uint64_t d = (uint64_t)blockIdx.x * 256 + threadIdx.x; d < nB; d += (uint64_t)gridDim.x * 256) {
    const uint64_t key = B[d];
    const uint32_t id = BV[d];
    uint64_t lo = 0, hi = nA;
    while (lo < hi) {
      const uint64_t m = (lo + hi) >> 1;
      if (kv_lt(A[m], AV[m], key, id)) lo = m + 1; else hi = m;
    }
    rk[u * nB + d] = (uint32_t)lo;
    ok[u * os + lo + d] = key;
    ov[u * os + lo + d] = id;
  }
}

// clo[b] = the first rank index d with rk[d] >= b * kMergeBlock, for blocks
// b in [0, nblk] (index d covers the blocks between rank d - 1 and rank d).
__global__ __launch_bounds__(256) void k_merge_blocks(const uint32_t* rk, uint64_t nB, uint32_t nblk,
                                                      uint32_t* clo) {
  const uint64_t u = blockIdx.y;
  const uint32_t* R = rk + u * nB;
  uint32_t* C = clo + u * (uint64_t)(nblk + 1);
  for (uint64_t d = (uint64_t)blockIdx.x * 256 + threadIdx.x; d <= nB; d += (uint64_t)gridDim.x * 256) {
    const uint32_t b0 = d == 0 ? 0u : R[d - 1] / kMergeBlock + 1;
    const uint32_t b1 = d == nB ? nblk : min(R[d] / kMergeBlock, nblk);
    for (uint32_t b = b0; b <= b1; ++b) C[b] = (uint32_t)d;
  }
}

__global__ __launch_bounds__(256) void k_merge_shift(const uint64_t* ak, const uint32_t* av, uint64_t as, uint64_t nA,
                                                     uint64_t nB, uint32_t nblk, const uint32_t* rk,
                                                     const uint32_t* clo, uint64_t* ok, uint32_t* ov, uint64_t os) {
  __shared__ uint32_t slice[kMergeSlice];
  const uint64_t u = blockIdx.y;
  const uint64_t* A = ak + u * as;
  const uint32_t* AV = av + u * as;
  const uint32_t* R = rk + u * nB;
  const uint32_t* C = clo + u * (uint64_t)(nblk + 1);
  for (uint32_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const uint32_t lo = C[b], m = C[b + 1] - lo;
    const bool in_lds = m <= kMergeSlice;
    __syncthreads();  // the previous block's slice is no longer read
    if (in_lds)
      for (uint32_t e = threadIdx.x; e < m; e += 256) slice[e] = R[lo + e];
    __syncthreads();
    const uint64_t x0 = (uint64_t)b * kMergeBlock;
    const uint64_t x1 = x0 + kMergeBlock < nA ? x0 + kMergeBlock : nA;
    for (uint64_t x = x0 + threadIdx.x; x < x1; x += 256) {
      uint32_t l = 0, h = m;  // ranks of the slice at or below x
      while (l < h) {
        const uint32_t mid = (l + h) >> 1;
        if ((in_lds ? slice[mid] : R[lo + mid]) <= x) l = mid + 1; else h = mid;
      }
      const uint64_t dst = u * os + x + lo + l;
      ok[dst] = A[x];
      ov[dst] = AV[x];
    }
  }
}

void launch_sort_chunk(const ServeEntry* ent, uint32_t nent, uint32_t t, const uint64_t* ckeys, uint64_t* csk,
                       uint32_t* csid, uint32_t Qtot, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_chunk, dim3(t, nent), dim3(256), 0, s, ent, ckeys, csk, csid, Qtot);
}

void launch_query(const QueryArgs& a, hipStream_t s) {
  if (a.Qtot) hipLaunchKernelGGL(k_query, dim3(a.Qtot), dim3(kQT), 0, s, a);
}

// Scratch: rk holds t * nB ranks, clo t * (ceil(nA / kMergeBlock) + 1) block starts.
uint64_t merge_scratch(uint64_t nA, uint64_t nB, uint32_t t) {
  return (uint64_t)t * (nB + (nA + kMergeBlock - 1) / kMergeBlock + 1);
}

void launch_merge(const uint64_t* ak, const uint32_t* av, uint64_t as, uint64_t nA, const uint64_t* bk,
                  const uint32_t* bv, uint64_t bs, uint64_t nB, uint64_t* ok, uint32_t* ov, uint64_t os, uint32_t t,
                  uint32_t* scratch, hipStream_t s) {
  if (nA + nB == 0) return;
  uint32_t* rk = scratch;
  uint32_t* clo = scratch + (uint64_t)t * nB;
  const uint32_t nblk = (uint32_t)((nA + kMergeBlock - 1) / kMergeBlock);
  const uint64_t gb = (nB + 256) / 256;
  if (nB)
    hipLaunchKernelGGL(k_merge_rank, dim3((unsigned)std::min<uint64_t>(gb, 4096), t), dim3(256), 0, s, ak, av, as, nA,
                       bk, bv, bs, nB, ok, ov, os, rk);
  hipLaunchKernelGGL(k_merge_blocks, dim3((unsigned)std::min<uint64_t>(gb, 4096), t), dim3(256), 0, s, rk, nB, nblk,
                     clo);
  if (nblk)
    hipLaunchKernelGGL(k_merge_shift, dim3(std::min<uint32_t>(nblk, 8192u), t), dim3(256), 0, s, ak, av, as, nA, nB,
                       nblk, rk, clo, ok, ov, os);
}

}  // namespace fl

using namespace fl;

// ---------------------------------------------------------------------------
// Host side: stations, tickets and the batching worker.
// ---------------------------------------------------------------------------
namespace {

struct Station {
  uint64_t n = 0;         // rows so far (history and inserted chunks)
  uint64_t nh = 0, hcap = 0;  // history rows and row stride per table
  uint64_t hphys = 0;     // rows per table the history buffers hold (>= hcap)
  uint64_t* hkey = nullptr;
  uint32_t* hid = nullptr;
  uint64_t nd = 0, dcap = 0;
  uint64_t* dkey[2] = {nullptr, nullptr};
  uint32_t* did[2] = {nullptr, nullptr};
  int dcur = 0;
  int err = 0;       // an insertion failed: later chunks of the station fail with it
  std::string msg;
};

// What the insertion step after a batch needs: each chunk's station, rows
// and place among the batch's sorted rows (per table: [t][Qtot]).
struct Insertion {
  std::vector<uint32_t> station;
  std::vector<uint32_t> cbase, nq;
  std::vector<bool> valid;
  const uint64_t* csk = nullptr;
  const uint32_t* csid = nullptr;
  uint32_t Qtot = 0;
};

enum { kPending = 0, kRunning = 1, kDone = 2, kFailed = 3 };

struct Ticket {
  uint32_t station = 0;
  fast_lsh_fps chunk{};
  uint64_t arrival_ns = 0, done_ns = 0;
  int state = kPending;
  int err = FAST_LSH_OK;
  std::string msg;
  fast_lsh_stats st{};
  std::vector<uint32_t> oi, oj;
  std::vector<uint8_t> ov;
};

uint64_t now_ns(std::chrono::steady_clock::time_point t0) {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct fast_lsh_server {
  int device = 0;
  hipStream_t stream = nullptr;
  fast_lsh_ctx* ctx = nullptr;  // scratch workspace and helpers, on `stream`
  std::vector<uint32_t> a, b;
  fast_lsh_hash h{};
  fast_lsh_filter flt{};
  fast_lsh_server_config cfg{};
  std::vector<Station> st;
  // per station: rows held plus the rows of its chunks waiting or running
  // (under mu); a chunk is admitted only while this stays within hcap
  std::vector<uint64_t> reserved;
  uint64_t mphys = 0;          // rows per table of the shared history-merge buffer
  uint64_t max_hcap = 0;       // largest history stride of any station (mphys never drops below it)
  uint64_t* mkey = nullptr;
  uint32_t* mid = nullptr;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<uint64_t> pending;
  std::map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  std::thread worker;
  bool started = false, stop = false;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  uint64_t batches = 0, chunks = 0, max_seen = 0;
  // sizes as of the worker's last step (the worker changes the buffers
  // without the lock; fast_lsh_server_info reads these under it)
  uint64_t snap_resident = 0, snap_workspace = 0;
};

// Pick the chunks of the next batch from the waiting ones, oldest first, at
// most one per station (a station's next chunk waits for the one before it
// to be inserted) and at most max_batch.  `stations[k]` is the station of
// the k-th waiting chunk; picked receives indices into that order.
extern "C" int fast_lsh_plan_batch(const uint32_t* stations, uint32_t n_waiting, uint32_t max_batch,
                                   uint32_t* picked, uint32_t* n_picked) {
  if ((!stations && n_waiting) || !picked || !n_picked) return fl_fail(FAST_LSH_E_INVALID, "NULL argument");
  uint32_t np = 0;
  for (uint32_t k = 0; k < n_waiting && np < max_batch; ++k) {
    bool earlier = false;  // an earlier chunk of this station waits (picked or not)
    for (uint32_t q = 0; q < k && !earlier; ++q) earlier = stations[q] == stations[k];
    if (!earlier) picked[np++] = k;
  }
  *n_picked = np;
  return FAST_LSH_OK;
}

// Bytes held by station tables and the shared merge buffer.
static uint64_t resident_bytes(const fast_lsh_server* sv) {
  const uint64_t t = sv->h.num_tables;
  uint64_t r = t * sv->mphys * 12;
  for (const Station& S : sv->st) r += t * (S.hphys + 2 * S.dcap) * 12;
  return r;
}

// Workspace of a full batch (max_batch chunks of max_chunk rows): the
// chunks' keys, sorted keys and ids per table, the output records at their
// initial size (16 per row; a batch with more matches grows them), and the
// scratch of the largest history merge.
static uint64_t batch_bytes(const fast_lsh_server* sv) {
  const uint64_t t = sv->h.num_tables;
  const uint64_t Q = (uint64_t)sv->cfg.max_batch * sv->cfg.max_chunk;
  uint64_t merge = 0;
  for (const Station& S : sv->st) merge = std::max(merge, merge_scratch(S.hcap, S.dcap, (uint32_t)t) * 4);
  return 20 * t * Q + 10 * std::max<uint64_t>(1u << 16, 16 * Q) + merge;
}

static int alloc_dev(void** p, uint64_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fl_fail(FAST_LSH_E_NOMEM, "hipMalloc of %llu bytes failed", (unsigned long long)bytes);
  }
  return FAST_LSH_OK;
}

// Merge a station's delta into its history: the merged run is written to
// the shared buffer (as large as the largest station's history, reserved
// when that station was admitted).  When the station's own history buffers
// are at least that large they swap roles with the shared one (no copy);
// a smaller station's merged run is copied back instead, so that the shared
// buffer never shrinks below the largest station.
static int merge_history(fast_lsh_server* sv, Station& S) {
  const uint32_t t = sv->h.num_tables;
  if (S.nh + S.nd > S.hcap)
    return fl_fail(FAST_LSH_E_NOMEM, "station history is full (%llu rows of %llu)",
                   (unsigned long long)(S.nh + S.nd), (unsigned long long)S.hcap);
  if (sv->mphys < S.hcap) return fl_fail(FAST_LSH_E_DEVICE, "history merge buffer smaller than the station");
  uint32_t* scr;
  RC(ws<uint32_t>(sv->ctx, "sv_merge", merge_scratch(S.nh, S.nd, t), &scr));
  launch_merge(S.hkey, S.hid, S.hcap, S.nh, S.dkey[S.dcur], S.did[S.dcur], S.dcap, S.nd, sv->mkey, sv->mid, S.hcap,
               t, scr, sv->stream);
  LAUNCHCK();
  const uint64_t rows = S.nh + S.nd;
  if (S.hphys >= sv->max_hcap) {
    std::swap(S.hkey, sv->mkey);
    std::swap(S.hid, sv->mid);
    std::swap(S.hphys, sv->mphys);
  } else if (rows) {
    HIPCK(hipMemcpy2DAsync(S.hkey, S.hcap * 8, sv->mkey, S.hcap * 8, rows * 8, t, hipMemcpyDeviceToDevice,
                           sv->stream));
    HIPCK(hipMemcpy2DAsync(S.hid, S.hcap * 4, sv->mid, S.hcap * 4, rows * 4, t, hipMemcpyDeviceToDevice,
                           sv->stream));
  }
  S.nh = rows;
  S.nd = 0;
  return FAST_LSH_OK;
}

// Search one batch (worker thread; the server lock is not held): every
// ticket's result is on the host when this returns; `ins` receives what the
// insertion step needs.
static int run_batch(fast_lsh_server* sv, std::vector<std::pair<uint64_t, Ticket*>>& batch, Insertion& ins) {
  fast_lsh_ctx* c = sv->ctx;
  hipStream_t s = sv->stream;
  const uint32_t t = sv->h.num_tables;
  const uint32_t nent = (uint32_t)batch.size();
  std::vector<ServeEntry> ent(nent);
  std::vector<int> cap(nent);
  std::vector<bool> vec(nent);
  uint32_t Qtot = 0;
  for (uint32_t e = 0; e < nent; ++e) {
    Ticket& T = *batch[e].second;
    Station& S = sv->st[T.station];
    int cp;
    bool vc;
    RC(fl_row_capacity(c, &T.chunk, &cp, &vc));
    cap[e] = cp;
    vec[e] = vc;
    ServeEntry& E = ent[e];
    E.hkey = S.hkey;
    E.hid = S.hid;
    E.hstride = S.hcap;
    E.nh = S.nh;
    E.dkey = S.dkey[S.dcur];
    E.did = S.did[S.dcur];
    E.dstride = S.dcap;
    E.nd = S.nd;
    E.cbase = Qtot;
    E.nq = (uint32_t)T.chunk.n;
    E.id0 = (uint32_t)S.n;
    E.pad = 0;
    Qtot += E.nq;
  }
  uint32_t* dh;
  RC(fl_upload_hash(c, &sv->h, &dh));
  ServeEntry* dent;
  uint64_t *ckeys, *csk;
  uint32_t* csid;
  unsigned long long* stats;
  int* err;  // one flag per chunk
  unsigned int* cnt;
  RC(ws<ServeEntry>(c, "sv_ent", nent, &dent));
  RC(ws<uint64_t>(c, "sv_ckeys", (uint64_t)t * Qtot, &ckeys));
  RC(ws<uint64_t>(c, "sv_csk", (uint64_t)t * Qtot, &csk));
  RC(ws<uint32_t>(c, "sv_csid", (uint64_t)t * Qtot, &csid));
  RC(ws<unsigned long long>(c, "sv_stats", (uint64_t)nent * kStatSlots * 4, &stats));
  RC(ws<int>(c, "sv_errs", nent, &err));
  RC(ws<unsigned int>(c, "sv_cnt", 1, &cnt));
  RC(h2d(c, dent, ent.data(), nent));
  fill_u32(reinterpret_cast<uint32_t*>(err), nent, 0, s);

  // 1. signatures
  for (uint32_t e = 0; e < nent; ++e) {
    SigArgs sa = fl_sig_args(&sv->h, &batch[e].second->chunk, dh, err + e);
    sa.table_begin = 0;
    sa.table_count = t;
    sa.vec_load = vec[e];
    sa.mkeys = ckeys;
    sa.out_stride = Qtot;
    sa.out_base = ent[e].cbase;
    sa.mix = kMixFull;
    prof_begin(c, FAST_LSH_STAGE_SIGNATURES);
    launch_sig(cap[e], sv->h.scheme == FAST_LSH_MINMAX, sa, s);
    prof_end(c);
  }
  LAUNCHCK();
  // 2. chunk sort; 3. votes
  prof_begin(c, FAST_LSH_STAGE_GROUP);
  launch_sort_chunk(dent, nent, t, ckeys, csk, csid, Qtot, s);
  prof_end(c);
  LAUNCHCK();
  QueryArgs qa;
  memset(&qa, 0, sizeof qa);
  qa.ent = dent;
  qa.nent = nent;
  qa.Qtot = Qtot;
  qa.t = t;
  qa.ckeys = ckeys;
  qa.csk = csk;
  qa.csid = csid;
  qa.min_lag = sv->flt.min_lag;
  qa.min_votes = sv->flt.min_votes;
  qa.out_count = cnt;
  qa.stats = stats;
  uint64_t out_cap = std::max<uint64_t>(1u << 16, (uint64_t)Qtot * 16);
  unsigned int hcnt = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    RC(ws<uint32_t>(c, "sv_oh", out_cap, &qa.out_h));
    RC(ws<uint32_t>(c, "sv_oq", out_cap, &qa.out_q));
    RC(ws<uint8_t>(c, "sv_ov", out_cap, &qa.out_v));
    RC(ws<uint8_t>(c, "sv_oe", out_cap, &qa.out_e));
    qa.out_cap = (uint32_t)out_cap;
    fill_u32(cnt, 1, 0, s);
    fill_u64(reinterpret_cast<uint64_t*>(stats), (uint64_t)nent * kStatSlots * 4, 0, s);
    prof_begin(c, FAST_LSH_STAGE_PAIRS);
    launch_query(qa, s);
    prof_end(c);
    LAUNCHCK();
    RC(d2h(c, &hcnt, cnt));
    if (hcnt <= out_cap) break;
    out_cap = (uint64_t)hcnt + 1024;
  }
  std::vector<int> herr(nent);
  RC(d2h(c, herr.data(), err, nent));
  for (uint32_t e = 0; e < nent; ++e) {
    Ticket& T = *batch[e].second;
    T.err = herr[e] ? FAST_LSH_E_INVALID : FAST_LSH_OK;
    if (herr[e]) T.msg = "a chunk row is empty or holds an index >= dim";
  }
  std::vector<uint32_t> oh(hcnt), oq(hcnt);
  std::vector<uint8_t> ov(hcnt), oe(hcnt);
  std::vector<unsigned long long> hst((uint64_t)nent * kStatSlots * 4);
  if (hcnt) {
    RC(d2h(c, oh.data(), qa.out_h, hcnt));
    RC(d2h(c, oq.data(), qa.out_q, hcnt));
    RC(d2h(c, ov.data(), qa.out_v, hcnt));
    RC(d2h(c, oe.data(), qa.out_e, hcnt));
  }
  RC(d2h(c, hst.data(), stats, hst.size()));
  // results per chunk, sorted by (i, j)
  std::vector<std::vector<uint32_t>> per(nent);
  for (uint32_t p = 0; p < hcnt; ++p) per[oe[p]].push_back(p);
  for (uint32_t e = 0; e < nent; ++e) {
    Ticket& T = *batch[e].second;
    auto& v = per[e];
    std::sort(v.begin(), v.end(), [&](uint32_t x, uint32_t y) { return oh[x] < oh[y] || (oh[x] == oh[y] && oq[x] < oq[y]); });
    T.oi.resize(v.size());
    T.oj.resize(v.size());
    T.ov.resize(v.size());
    for (size_t q = 0; q < v.size(); ++q) {
      T.oi[q] = oh[v[q]];
      T.oj[q] = oq[v[q]];
      T.ov[q] = ov[v[q]];
    }
    fast_lsh_stats& o = T.st;
    memset(&o, 0, sizeof o);
    for (uint32_t k = 0; k < kStatSlots; ++k) {
      const unsigned long long* x = &hst[((uint64_t)e * kStatSlots + k) * 4];
      o.e_raw += x[0];
      o.e_voted += x[1];
      o.n_distinct += x[2];
      o.max_bucket = std::max<uint64_t>(o.max_bucket, x[3]);
    }
    o.n_out = v.size();
  }
  ins.station.resize(nent);
  ins.cbase.resize(nent);
  ins.nq.resize(nent);
  ins.valid.resize(nent);
  for (uint32_t e = 0; e < nent; ++e) {
    ins.station[e] = batch[e].second->station;
    ins.cbase[e] = ent[e].cbase;
    ins.nq[e] = ent[e].nq;
    ins.valid[e] = batch[e].second->err == FAST_LSH_OK;
  }
  ins.csk = csk;
  ins.csid = csid;
  ins.Qtot = Qtot;
  return FAST_LSH_OK;
}

// Insert every valid chunk of the last batch into its station's delta (a
// rejected chunk leaves its station unchanged), merging a full delta into
// the history first.  Runs after the batch's tickets are done, so a history
// merge delays only later batches.  A failed insertion marks its station.
static void insert_batch(fast_lsh_server* sv, const Insertion& ins) {
  fast_lsh_ctx* c = sv->ctx;
  hipStream_t s = sv->stream;
  const uint32_t t = sv->h.num_tables;
  for (size_t e = 0; e < ins.station.size(); ++e) {
    Station& S = sv->st[ins.station[e]];
    if (!ins.valid[e] || S.err) continue;
    const uint64_t nq = ins.nq[e];
    int rc = FAST_LSH_OK;
    if (S.nd + nq > S.dcap) rc = merge_history(sv, S);
    uint32_t* scr = nullptr;
    if (rc == FAST_LSH_OK) rc = ws<uint32_t>(c, "sv_merge", merge_scratch(S.nd, nq, t), &scr);
    if (rc == FAST_LSH_OK) {
      const int nx = 1 - S.dcur;
      prof_begin(c, FAST_LSH_STAGE_OUTPUT);
      launch_merge(S.dkey[S.dcur], S.did[S.dcur], S.dcap, S.nd, ins.csk + ins.cbase[e], ins.csid + ins.cbase[e],
                   ins.Qtot, nq, S.dkey[nx], S.did[nx], S.dcap, t, scr, s);
      prof_end(c);
      if (hipGetLastError() != hipSuccess) {
        rc = fl_fail(FAST_LSH_E_DEVICE, "chunk insertion launch failed");
      } else {
        S.dcur = nx;
        S.nd += nq;
        S.n += nq;
      }
    }
    if (rc != FAST_LSH_OK) {
      S.err = rc;
      S.msg = fast_lsh_last_error();
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess)
    for (size_t e = 0; e < ins.station.size(); ++e) {
      Station& S = sv->st[ins.station[e]];
      if (!S.err) {
        S.err = FAST_LSH_E_DEVICE;
        S.msg = "chunk insertion failed on the device";
      }
    }
  prof_collect(c);
}

static void worker_main(fast_lsh_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    sv->cv.wait(lk, [&] { return sv->stop || !sv->pending.empty(); });
    if (sv->stop && sv->pending.empty()) break;
    std::vector<uint32_t> stations;
    for (uint64_t id : sv->pending) stations.push_back(sv->tickets[id].station);
    std::vector<uint32_t> picked(stations.size());
    uint32_t np = 0;
    fast_lsh_plan_batch(stations.data(), (uint32_t)stations.size(), sv->cfg.max_batch, picked.data(), &np);
    std::vector<std::pair<uint64_t, Ticket*>> batch;
    std::vector<uint64_t> ids;
    for (uint32_t q = 0; q < np; ++q) ids.push_back(sv->pending[picked[q]]);
    for (uint64_t id : ids) {
      Ticket& T = sv->tickets[id];
      T.state = kRunning;
      batch.emplace_back(id, &T);
    }
    for (uint64_t id : ids) sv->pending.erase(std::find(sv->pending.begin(), sv->pending.end(), id));
    lk.unlock();
    // chunks of a station whose insertion failed earlier fail with that error
    std::vector<std::pair<uint64_t, Ticket*>> run;
    for (auto& b : batch) {
      const Station& S = sv->st[b.second->station];
      b.second->err = S.err;
      if (S.err) b.second->msg = S.msg; else run.push_back(b);
    }
    Insertion ins;
    const int rc = run.empty() ? FAST_LSH_OK : run_batch(sv, run, ins);
    const std::string msg = rc == FAST_LSH_OK ? std::string() : std::string(fast_lsh_last_error());
    lk.lock();
    const uint64_t done = now_ns(sv->t0);
    for (auto& b : run) {
      if (rc != FAST_LSH_OK) {  // the batch as a whole failed
        b.second->err = rc;
        b.second->msg = msg;
      }
    }
    for (auto& b : batch) {
      b.second->state = b.second->err == FAST_LSH_OK ? kDone : kFailed;
      b.second->done_ns = done;
      // a failed chunk is not inserted: its rows leave the reservation
      if (b.second->err != FAST_LSH_OK) sv->reserved[b.second->station] -= b.second->chunk.n;
    }
    ++sv->batches;
    sv->chunks += batch.size();
    sv->max_seen = std::max<uint64_t>(sv->max_seen, batch.size());
    sv->snap_workspace = sv->ctx->ws_total;
    sv->cv_done.notify_all();
    if (rc == FAST_LSH_OK && !run.empty()) {  // tickets are done; now the insertion
      lk.unlock();
      insert_batch(sv, ins);
      lk.lock();
      sv->snap_resident = resident_bytes(sv);
      sv->snap_workspace = sv->ctx->ws_total;
    }
  }
}

extern "C" {

int fast_lsh_server_create(int device, const fast_lsh_hash* h, const fast_lsh_filter* flt,
                           const fast_lsh_server_config* cfg, fast_lsh_server** out) {
  if (!out) return fl_fail(FAST_LSH_E_INVALID, "out is NULL");
  *out = nullptr;
  RC(fl_check_hash(h));
  if (!flt) return fl_fail(FAST_LSH_E_INVALID, "filter is NULL");
  if (flt->min_votes < 1) return fl_fail(FAST_LSH_E_INVALID, "min_votes must be >= 1");
  if (flt->occ_den) return fl_fail(FAST_LSH_E_INVALID, "the serving form runs without the occurrence filter");
  fast_lsh_server_config c{8, 3600, 262144, 2000000, 0};
  if (cfg) c = *cfg;
  if (c.max_batch < 1 || c.max_batch > 16) return fl_fail(FAST_LSH_E_INVALID, "max_batch %u outside [1, 16]", c.max_batch);
  if (c.max_chunk < 1 || c.max_chunk > (uint32_t)kChunkMax)
    return fl_fail(FAST_LSH_E_INVALID, "max_chunk %u outside [1, %d]", c.max_chunk, kChunkMax);
  if (c.delta_rows < c.max_chunk) return fl_fail(FAST_LSH_E_INVALID, "delta_rows below max_chunk");
  fast_lsh_server* sv = new fast_lsh_server();
  sv->device = device;
  sv->cfg = c;
  sv->flt = *flt;
  const uint32_t F = fl_n_funcs(h);
  sv->a.assign(h->a, h->a + F);
  sv->b.assign(h->b, h->b + F);
  sv->h = *h;
  sv->h.a = sv->a.data();
  sv->h.b = sv->b.data();
  int rc = FAST_LSH_OK;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    delete sv;
    return fl_fail(FAST_LSH_E_DEVICE, "cannot create a stream on device %d", device);
  }
  rc = fast_lsh_ctx_create(device, sv->stream, 0, &sv->ctx);
  if (rc != FAST_LSH_OK) {
    (void)hipStreamDestroy(sv->stream);
    delete sv;
    return rc;
  }
  *out = sv;
  return FAST_LSH_OK;
}

void fast_lsh_server_destroy(fast_lsh_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  (void)hipSetDevice(sv->device);
  (void)hipStreamSynchronize(sv->stream);
  for (Station& S : sv->st) {
    (void)hipFree(S.hkey);
    (void)hipFree(S.hid);
    for (int k = 0; k < 2; ++k) {
      (void)hipFree(S.dkey[k]);
      (void)hipFree(S.did[k]);
    }
  }
  if (sv->mkey) (void)hipFree(sv->mkey);
  if (sv->mid) (void)hipFree(sv->mid);
  fast_lsh_ctx_destroy(sv->ctx);
  (void)hipStreamDestroy(sv->stream);
  delete sv;
}

int fast_lsh_server_add_station(fast_lsh_server* sv, const fast_lsh_fps* hist, uint32_t* station) {
  if (!sv || !station) return fl_fail(FAST_LSH_E_INVALID, "server or station is NULL");
  RC(fl_check_fps(hist));
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->started) return fl_fail(FAST_LSH_E_BUSY, "stations are added before the first chunk is submitted");
  }
  HIPCK(hipSetDevice(sv->device));
  fast_lsh_ctx* c = sv->ctx;
  hipStream_t s = sv->stream;
  const uint32_t t = sv->h.num_tables;
  const uint64_t n = hist->n;
  Station S;
  S.n = S.nh = n;
  S.hcap = n + sv->cfg.slack_rows;
  S.dcap = sv->cfg.delta_rows;
  S.hphys = S.hcap;
  // admission: the station's tables, the growth of the shared merge buffer
  // to its size, and the transient build buffers must fit the budget
  const uint64_t in_use = resident_bytes(sv) + c->ws_total;
  const uint64_t grow = S.hcap > sv->mphys ? (uint64_t)t * (S.hcap - sv->mphys) * 12 : 0;
  const uint64_t build = (uint64_t)std::min<uint32_t>(10, t) * n * 32 + (uint64_t)t * 256 * 8;
  const uint64_t need = (uint64_t)t * (S.hcap + 2 * S.dcap) * 12 + grow;
  if (sv->cfg.hbm_budget && in_use + need + build > sv->cfg.hbm_budget)
    return fl_fail(FAST_LSH_E_NOMEM,
                   "station of %llu rows needs %llu bytes (+%llu while building); %llu of the %llu-byte budget are in use",
                   (unsigned long long)n, (unsigned long long)need, (unsigned long long)build,
                   (unsigned long long)in_use, (unsigned long long)sv->cfg.hbm_budget);
  int rc = FAST_LSH_OK;
  auto cleanup = [&] {
    (void)hipFree(S.hkey);
    (void)hipFree(S.hid);
    for (int k = 0; k < 2; ++k) {
      (void)hipFree(S.dkey[k]);
      (void)hipFree(S.did[k]);
    }
  };
  if ((rc = alloc_dev((void**)&S.hkey, (uint64_t)t * S.hcap * 8)) ||
      (rc = alloc_dev((void**)&S.hid, (uint64_t)t * S.hcap * 4)) ||
      (rc = alloc_dev((void**)&S.dkey[0], (uint64_t)t * S.dcap * 8)) ||
      (rc = alloc_dev((void**)&S.did[0], (uint64_t)t * S.dcap * 4)) ||
      (rc = alloc_dev((void**)&S.dkey[1], (uint64_t)t * S.dcap * 8)) ||
      (rc = alloc_dev((void**)&S.did[1], (uint64_t)t * S.dcap * 4))) {
    cleanup();
    return rc;
  }
  if (grow) {  // the shared merge buffer grows to this station's size
    uint64_t* mk = nullptr;
    uint32_t* mi = nullptr;
    if ((rc = alloc_dev((void**)&mk, (uint64_t)t * S.hcap * 8)) || (rc = alloc_dev((void**)&mi, (uint64_t)t * S.hcap * 4))) {
      (void)hipFree(mk);
      cleanup();
      return rc;
    }
    if (sv->mkey) {
      (void)hipFree(sv->mkey);
      (void)hipFree(sv->mid);
    }
    sv->mkey = mk;
    sv->mid = mi;
    sv->mphys = S.hcap;
  }
  if (n) {
    // build: signatures and a full 64-bit (key, id) sort, ten tables at a time
    uint32_t* dh;
    int cp;
    bool vc;
    if ((rc = fl_upload_hash(c, &sv->h, &dh)) || (rc = fl_row_capacity(c, hist, &cp, &vc))) {
      cleanup();
      return rc;
    }
    const uint32_t TG = std::min<uint32_t>(10, t);
    const uint64_t gn = (uint64_t)TG * n;
    uint64_t *mk, *ak, *bk;
    uint32_t *av, *bv, *hs, *sums;
    int* err;
    const uint32_t nt = radix_tiles(n, 0);
    if ((rc = ws<uint64_t>(c, "sv_build_mk", gn, &mk)) || (rc = ws<uint64_t>(c, "sv_build_ak", gn, &ak)) ||
        (rc = ws<uint64_t>(c, "sv_build_bk", gn, &bk)) || (rc = ws<uint32_t>(c, "sv_build_av", gn, &av)) ||
        (rc = ws<uint32_t>(c, "sv_build_bv", gn, &bv)) ||
        (rc = ws<uint32_t>(c, "sv_build_hist", (uint64_t)256 * nt * TG, &hs)) ||
        (rc = ws<uint32_t>(c, "sv_build_sums", scan_sums_elems((uint64_t)256 * nt, TG), &sums)) ||
        (rc = ws<int>(c, "sv_err", 1, &err))) {
      cleanup();
      return rc;
    }
    fill_u32(reinterpret_cast<uint32_t*>(err), 1, 0, s);
    for (uint32_t tb = 0; tb < t; tb += TG) {
      const uint32_t tc = std::min(TG, t - tb);
      SigArgs sa = fl_sig_args(&sv->h, hist, dh, err);
      sa.table_begin = tb;
      sa.table_count = tc;
      sa.vec_load = vc;
      sa.mkeys = mk;
      sa.mix = kMixFull;
      launch_sig(cp, sv->h.scheme == FAST_LSH_MINMAX, sa, s);
      const uint64_t* kin = mk;
      const uint32_t* vin = nullptr;
      uint64_t *ko = ak, *ko2 = bk;
      uint32_t *vo = av, *vo2 = bv;
      for (uint32_t shift = 0; shift < 64; shift += 8) {
        radix_pass(kin, vin, ko, vo, n, tc, shift, hs, sums, 0, s);
        kin = ko;
        vin = vo;
        std::swap(ko, ko2);
        std::swap(vo, vo2);
      }
      // kin / vin hold the sorted tables, n per table: copy into the station's rows
      if (hipMemcpy2DAsync(S.hkey + (uint64_t)tb * S.hcap, S.hcap * 8, kin, n * 8, n * 8, tc,
                           hipMemcpyDeviceToDevice, s) != hipSuccess ||
          hipMemcpy2DAsync(S.hid + (uint64_t)tb * S.hcap, S.hcap * 4, vin, n * 4, n * 4, tc,
                           hipMemcpyDeviceToDevice, s) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fl_fail(FAST_LSH_E_DEVICE, "copy of the sorted history failed");
      }
    }
    int herr = 0;
    if ((rc = d2h(c, &herr, err))) {
      cleanup();
      return rc;
    }
    if (herr) {
      cleanup();
      return fl_fail(FAST_LSH_E_INVALID, "a history row is empty or holds an index >= dim (%u)", sv->h.dim);
    }
    // release the build buffers (the serving workspace is small)
    for (const char* name : {"sv_build_mk", "sv_build_ak", "sv_build_bk", "sv_build_av", "sv_build_bv",
                             "sv_build_hist", "sv_build_sums"}) {
      Buf& b = c->ws[name];
      if (b.p) {
        (void)hipFree(b.p);
        c->ws_total -= b.cap;
        b = Buf();
      }
    }
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  *station = (uint32_t)sv->st.size();
  sv->max_hcap = std::max(sv->max_hcap, S.hcap);
  sv->st.push_back(S);
  sv->reserved.push_back(S.n);
  return FAST_LSH_OK;
}

int fast_lsh_server_submit(fast_lsh_server* sv, uint32_t station, const fast_lsh_fps* chunk, uint64_t arrival_ns,
                           uint64_t* ticket) {
  if (!sv || !ticket) return fl_fail(FAST_LSH_E_INVALID, "server or ticket is NULL");
  RC(fl_check_fps(chunk));
  if (chunk->n < 1 || chunk->n > sv->cfg.max_chunk)
    return fl_fail(FAST_LSH_E_INVALID, "chunk of %llu rows outside [1, %u]", (unsigned long long)chunk->n,
                   sv->cfg.max_chunk);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (station >= sv->st.size()) return fl_fail(FAST_LSH_E_INVALID, "no station %u", station);
  // admission by footprint: the chunk's rows must fit the tables its station
  // holds once every chunk already queued for it is inserted, and (with a
  // budget) a full batch's workspace must fit beside the resident tables
  if (sv->reserved[station] + chunk->n > sv->st[station].hcap)
    return fl_fail(FAST_LSH_E_NOMEM, "station %u has room for %llu more rows, the chunk has %llu", station,
                   (unsigned long long)(sv->st[station].hcap - sv->reserved[station]),
                   (unsigned long long)chunk->n);
  if (!sv->started && sv->cfg.hbm_budget) {
    const uint64_t need = resident_bytes(sv) + batch_bytes(sv);
    if (need > sv->cfg.hbm_budget)
      return fl_fail(FAST_LSH_E_NOMEM, "resident tables and a full batch need %llu bytes of the %llu-byte budget",
                     (unsigned long long)need, (unsigned long long)sv->cfg.hbm_budget);
  }
  sv->reserved[station] += chunk->n;
  const uint64_t id = sv->next_ticket++;
  Ticket& T = sv->tickets[id];
  T.station = station;
  T.chunk = *chunk;
  T.arrival_ns = arrival_ns;
  sv->pending.push_back(id);
  if (!sv->started) {
    sv->snap_resident = resident_bytes(sv);
    sv->snap_workspace = sv->ctx->ws_total;
    sv->started = true;
    sv->worker = std::thread(worker_main, sv);
  }
  sv->cv.notify_all();
  *ticket = id;
  return FAST_LSH_OK;
}

int fast_lsh_server_poll(fast_lsh_server* sv, uint64_t ticket, int wait, fast_lsh_stats* st, uint64_t* done_ns) {
  if (!sv) return fl_fail(FAST_LSH_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return fl_fail(FAST_LSH_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  if (wait) sv->cv_done.wait(lk, [&] { return it->second.state >= kDone; });
  Ticket& T = it->second;
  if (T.state < kDone) return FAST_LSH_E_BUSY;
  if (T.state == kFailed) return fl_fail(T.err, "%s", T.msg.c_str());
  if (st) *st = T.st;
  if (done_ns) *done_ns = T.done_ns;
  return FAST_LSH_OK;
}

int fast_lsh_server_take(fast_lsh_server* sv, uint64_t ticket, uint32_t* oi, uint32_t* oj, uint8_t* ov,
                         uint64_t capacity) {
  if (!sv) return fl_fail(FAST_LSH_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return fl_fail(FAST_LSH_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Ticket& T = it->second;
  if (T.state < kDone) return FAST_LSH_E_BUSY;
  if (T.state == kFailed) {
    const int e = T.err;
    const std::string m = T.msg;
    sv->tickets.erase(it);
    return fl_fail(e, "%s", m.c_str());
  }
  const uint64_t m = T.oi.size();
  if (m > capacity)
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)m,
                   (unsigned long long)capacity);
  if (m && (!oi || !oj || !ov)) return fl_fail(FAST_LSH_E_INVALID, "output pointer is NULL");
  if (m) {
    memcpy(oi, T.oi.data(), m * 4);
    memcpy(oj, T.oj.data(), m * 4);
    memcpy(ov, T.ov.data(), m);
  }
  sv->tickets.erase(it);
  return FAST_LSH_OK;
}

uint64_t fast_lsh_server_now_ns(fast_lsh_server* sv) { return sv ? now_ns(sv->t0) : 0; }

int fast_lsh_server_info(fast_lsh_server* sv, fast_lsh_server_state* out) {
  if (!sv || !out) return fl_fail(FAST_LSH_E_INVALID, "server or out is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  out->stations = (uint32_t)sv->st.size();
  out->waiting = (uint32_t)sv->pending.size();
  out->resident_bytes = sv->started ? sv->snap_resident : resident_bytes(sv);
  out->workspace_bytes = sv->started ? sv->snap_workspace : sv->ctx->ws_total;
  out->batches = sv->batches;
  out->chunks = sv->chunks;
  out->largest_batch = sv->max_seen;
  return FAST_LSH_OK;
}

}  // extern "C"
