// Spatiotemporal alignment of search outputs (section 7): the channel-level
// merge of a station's channels (section 7.1 "Channel Level", section 7.2
// "Channel": sort by (dt, idx1), merge, sum the similarity of equal entries,
// threshold) and the station-level clustering of the combined entries along
// thin diagonals (section 7.1 "Station Level", section 7.2 "Station": runs
// along each diagonal with bounded gaps, runs of adjacent diagonals merged,
// one summary per cluster, small and wide clusters pruned).
//
// Channel merge on the GPU: every channel's pairs are packed as 64-bit keys
// dt << 32 | idx1 (dt = j - i, idx1 = i) with the votes as values and all
// channels are sorted at once by LSD radix passes over the bits the ids use
// (one sort of the concatenation leaves equal keys adjacent, which is what
// the paper's per-channel sort plus merge achieves); equal keys are summed
// from each run's first element and the survivors compacted by a scan.
//
// Clusters on the GPU: run heads come from comparing each entry with its
// predecessor and are numbered by a scan; a run is linked to the runs of the
// next diagonal whose spans come within the gap, found by bisection in the
// run table (within one diagonal both ends of the runs ascend); links are
// joined by a lock-free union-find that always hooks the larger root under
// the smaller, so every cluster's root is its first run; per-entry summaries
// go to the root with one atomic per wave when a wave lies in one run.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "host.hpp"

using namespace fl;

namespace {

constexpr int kAT = 256;

struct AlignCtrl {
  int err;               // 1: a pair with j <= i or an id >= n; 2: entries out of order; 3: sim >= 2^24
  unsigned int pad;
  uint64_t runs;         // station clusters: runs found
};

__global__ __launch_bounds__(kAT) void k_pack_pairs(const uint32_t* pi, const uint32_t* pj, const uint8_t* pv,
                                                    uint64_t count, uint64_t n, uint64_t* key, uint32_t* val,
                                                    int* err) {
  for (uint64_t e = (uint64_t)blockIdx.x * kAT + threadIdx.x; e < count; e += (uint64_t)gridDim.x * kAT) {
    const uint32_t i = pi[e], j = pj[e];
    if (j <= i || j >= n) {
      *err = 1;
      key[e] = 0;
      val[e] = 0;
      continue;
    }
    key[e] = ((uint64_t)(j - i) << 32) | i;
    val[e] = pv[e];
  }
}

// keep[k] = 1 at the first element of each run of equal keys whose summed
// value reaches min_sim (its sum in sum[k]); 0 elsewhere.
__global__ __launch_bounds__(kAT) void k_merge_heads(const uint64_t* key, const uint32_t* val, uint64_t count,
                                                     uint32_t min_sim, uint64_t* keep, uint32_t* sum) {
  for (uint64_t e = (uint64_t)blockIdx.x * kAT + threadIdx.x; e < count; e += (uint64_t)gridDim.x * kAT) {
    const uint64_t k = key[e];
    uint64_t flag = 0;
    if (e == 0 || key[e - 1] != k) {
      uint32_t s = val[e];
      for (uint64_t q = e + 1; q < count && key[q] == k; ++q) s += val[q];
      sum[e] = s;
      flag = s >= min_sim;
    }
    keep[e] = flag;
  }
}

// pos: exclusive scan of keep (recomputed head test: keep is overwritten).
__global__ __launch_bounds__(kAT) void k_merge_emit(const uint64_t* key, const uint32_t* sum, const uint64_t* pos,
                                                    uint64_t count, uint64_t total, uint32_t* odt, uint32_t* oidx,
                                                    uint32_t* osim) {
  for (uint64_t e = (uint64_t)blockIdx.x * kAT + threadIdx.x; e < count; e += (uint64_t)gridDim.x * kAT) {
    const uint64_t p = pos[e];
    const uint64_t nxt = e + 1 < count ? pos[e + 1] : total;
    if (nxt == p) continue;  // not kept
    const uint64_t k = key[e];
    odt[p] = (uint32_t)(k >> 32);
    oidx[p] = (uint32_t)k;
    osim[p] = sum[e];
  }
}

// ---------------------------------------------------------------------------
// Station clusters
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool run_head(const uint32_t* dt, const uint32_t* x, uint64_t k, uint32_t gap) {
  return k == 0 || dt[k] != dt[k - 1] || x[k] - x[k - 1] > gap;
}

__global__ __launch_bounds__(kAT) void k_run_heads(const uint32_t* dt, const uint32_t* x, const uint32_t* sim,
                                                   uint64_t n, uint32_t gap, uint64_t* head, int* err) {
  for (uint64_t k = (uint64_t)blockIdx.x * kAT + threadIdx.x; k < n; k += (uint64_t)gridDim.x * kAT) {
    if (k > 0 && (dt[k] < dt[k - 1] || (dt[k] == dt[k - 1] && x[k] <= x[k - 1]))) *err = 2;
    if (sim[k] >= (1u << 24)) *err = 3;
    head[k] = run_head(dt, x, k, gap) ? 1 : 0;
  }
}

// Run of entry k: heads in [0, k] minus one (rs = exclusive scan of heads).
__device__ __forceinline__ uint32_t run_of(const uint64_t* rs, const uint32_t* dt, const uint32_t* x, uint64_t k,
                                           uint32_t gap) {
  return (uint32_t)(rs[k] + (run_head(dt, x, k, gap) ? 1 : 0) - 1);
}

__global__ __launch_bounds__(kAT) void k_run_table(const uint32_t* dt, const uint32_t* x, uint64_t n, uint32_t gap,
                                                   const uint64_t* rs, uint32_t* rdt, uint32_t* rlo, uint32_t* rhi,
                                                   uint32_t* parent) {
  for (uint64_t k = (uint64_t)blockIdx.x * kAT + threadIdx.x; k < n; k += (uint64_t)gridDim.x * kAT) {
    const uint32_t r = run_of(rs, dt, x, k, gap);
    if (run_head(dt, x, k, gap)) {
      rdt[r] = dt[k];
      rlo[r] = x[k];
      parent[r] = r;
    }
    if (k + 1 == n || run_head(dt, x, k + 1, gap)) rhi[r] = x[k];
  }
}

__device__ __forceinline__ uint32_t uf_root(uint32_t* p, uint32_t a) {
  while (true) {
    const uint32_t b = __atomic_load_n(&p[a], __ATOMIC_RELAXED);
    if (b == a) return a;
    a = b;
  }
}

// Join the sets of a and b: the larger root is hooked under the smaller one
// (a root only ever changes from itself to a smaller index, so a find always
// ends and every set's root is its smallest member).
__device__ __forceinline__ void uf_union(uint32_t* p, uint32_t a, uint32_t b) {
  while (true) {
    a = uf_root(p, a);
    b = uf_root(p, b);
    if (a == b) return;
    if (a < b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(&p[a], a, b) == a) return;
  }
}

// Run a joins the runs of diagonal dt(a) + 1 whose span [lo, hi] comes
// within gap of its own: the first such run is the first with
// (dt, hi) >= (dt(a) + 1, lo(a) - gap) (runs ascend by (dt, lo) and by
// (dt, hi)); the following ones while lo <= hi(a) + gap.
__global__ __launch_bounds__(kAT) void k_run_links(const uint32_t* rdt, const uint32_t* rlo, const uint32_t* rhi,
                                                   uint32_t R, uint32_t gap, uint32_t* parent) {
  for (uint64_t a = (uint64_t)blockIdx.x * kAT + threadIdx.x; a < R; a += (uint64_t)gridDim.x * kAT) {
    const uint32_t d = rdt[a] + 1;
    if (d == 0) continue;  // dt(a) = 2^32 - 1 has no next diagonal
    const uint64_t lo = rlo[a], hi = rhi[a];
    const uint64_t want = ((uint64_t)d << 32) | (lo > gap ? lo - gap : 0);
    uint32_t L = (uint32_t)a + 1, H = R;  // runs of larger diagonals follow a
    while (L < H) {
      const uint32_t M = L + (H - L) / 2;
      if ((((uint64_t)rdt[M] << 32) | rhi[M]) < want) L = M + 1; else H = M;
    }
    for (uint32_t b = L; b < R && rdt[b] == d && (uint64_t)rlo[b] <= hi + gap; ++b) uf_union(parent, (uint32_t)a, b);
  }
}

__global__ __launch_bounds__(kAT) void k_run_compress(uint32_t* parent, uint32_t R) {
  for (uint64_t a = (uint64_t)blockIdx.x * kAT + threadIdx.x; a < R; a += (uint64_t)gridDim.x * kAT)
    parent[a] = uf_root(parent, (uint32_t)a);
}

struct ClusterAcc {
  uint32_t* dtmax;
  uint32_t* xmin;
  uint32_t* xmax;
  uint32_t* cnt;
  unsigned long long* sum;
  unsigned long long* peak;  // sim << 40 | (2^40 - 1 - entry): the largest is the strongest, earliest entry
};

constexpr uint64_t kPeakIdx = (1ull << 40) - 1;

__global__ __launch_bounds__(kAT) void k_cluster_stats(const uint32_t* dt, const uint32_t* x, const uint32_t* sim,
                                                       uint64_t n, uint32_t gap, const uint64_t* rs,
                                                       const uint32_t* parent, ClusterAcc acc) {
  const uint64_t stride = (uint64_t)gridDim.x * kAT;
  // every lane runs the same number of rounds so that wave votes see all lanes
  const uint64_t rounds = (n + stride - 1) / stride;
  for (uint64_t rd = 0; rd < rounds; ++rd) {
    const uint64_t k = rd * stride + (uint64_t)blockIdx.x * kAT + threadIdx.x;
    const bool live = k < n;
    uint32_t root = 0, d = 0, xv = 0;
    unsigned long long s = 0, pk = 0;
    if (live) {
      root = parent[run_of(rs, dt, x, k, gap)];
      d = dt[k];
      xv = x[k];
      s = sim[k];
      pk = (s << 40) | (kPeakIdx - k);
    }
    const uint64_t act = __ballot(live);
    if (act == 0) continue;
    const uint32_t r0 = __shfl(root, __ffsll((long long)act) - 1, 64);
    if (__all(!live || root == r0)) {
      // one cluster: reduce over the wave, one atomic per field
      uint32_t dmax = live ? d : 0u, xmn = live ? xv : 0xFFFFFFFFu, xmx = live ? xv : 0u, c = live ? 1u : 0u;
      for (int o = 32; o > 0; o >>= 1) {
        dmax = max(dmax, (uint32_t)__shfl_xor(dmax, o, 64));
        xmn = min(xmn, (uint32_t)__shfl_xor(xmn, o, 64));
        xmx = max(xmx, (uint32_t)__shfl_xor(xmx, o, 64));
        c += __shfl_xor(c, o, 64);
        s += __shfl_xor(s, o, 64);
        pk = max(pk, (unsigned long long)__shfl_xor(pk, o, 64));
      }
      if ((threadIdx.x & 63) == (uint32_t)(__ffsll((long long)act) - 1)) {
        atomicMax(acc.dtmax + r0, dmax);
        atomicMin(acc.xmin + r0, xmn);
        atomicMax(acc.xmax + r0, xmx);
        atomicAdd(acc.cnt + r0, c);
        atomicAdd(acc.sum + r0, s);
        atomicMax(acc.peak + r0, pk);
      }
    } else if (live) {
      atomicMax(acc.dtmax + root, d);
      atomicMin(acc.xmin + root, xv);
      atomicMax(acc.xmax + root, xv);
      atomicAdd(acc.cnt + root, 1u);
      atomicAdd(acc.sum + root, s);
      atomicMax(acc.peak + root, pk);
    }
  }
}

__global__ __launch_bounds__(kAT) void k_cluster_init(ClusterAcc acc, uint32_t R) {
  for (uint64_t a = (uint64_t)blockIdx.x * kAT + threadIdx.x; a < R; a += (uint64_t)gridDim.x * kAT) {
    acc.dtmax[a] = 0;
    acc.xmin[a] = 0xFFFFFFFFu;
    acc.xmax[a] = 0;
    acc.cnt[a] = 0;
    acc.sum[a] = 0;
    acc.peak[a] = 0;
  }
}

__global__ __launch_bounds__(kAT) void k_cluster_keep(const uint32_t* parent, const uint32_t* rdt, ClusterAcc acc,
                                                      uint32_t R, uint32_t max_width, uint32_t min_entries,
                                                      uint64_t min_sum, uint64_t* keep) {
  for (uint64_t a = (uint64_t)blockIdx.x * kAT + threadIdx.x; a < R; a += (uint64_t)gridDim.x * kAT) {
    bool k = parent[a] == a;
    if (k) {
      const uint64_t width = (uint64_t)acc.dtmax[a] - rdt[a] + 1;
      k = width <= max_width && acc.cnt[a] >= min_entries && acc.sum[a] >= min_sum;
    }
    keep[a] = k ? 1 : 0;
  }
}

__global__ __launch_bounds__(kAT) void k_cluster_emit(const uint32_t* rdt, ClusterAcc acc, const uint64_t* pos,
                                                      uint32_t R, uint64_t total, const uint32_t* dt,
                                                      const uint32_t* x, fast_lsh_cluster* out) {
  for (uint64_t a = (uint64_t)blockIdx.x * kAT + threadIdx.x; a < R; a += (uint64_t)gridDim.x * kAT) {
    const uint64_t p = pos[a];
    const uint64_t nxt = a + 1 < R ? pos[a + 1] : total;
    if (nxt == p) continue;
    const unsigned long long pk = acc.peak[a];
    const uint64_t e = kPeakIdx - (pk & kPeakIdx);
    fast_lsh_cluster c;
    c.dt_min = rdt[a];
    c.dt_max = acc.dtmax[a];
    c.idx1_min = acc.xmin[a];
    c.idx1_max = acc.xmax[a];
    c.n_entries = acc.cnt[a];
    c.peak_sim = (uint32_t)(pk >> 40);
    c.peak_dt = dt[e];
    c.peak_idx1 = x[e];
    c.sim_sum = acc.sum[a];
    out[p] = c;
  }
}

unsigned grid_of(uint64_t n) {
  const uint64_t b = (n + kAT - 1) / kAT;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 8u * device_cus()));
}

// ---------------------------------------------------------------------------
// Channel merge host side: buffers, checks, the launch sequence
// ---------------------------------------------------------------------------
struct MergeBufs {
  uint64_t *k0, *k1, *keep, *sums64;
  uint32_t *v0, *v1, *hist, *sums, *tot;
  AlignCtrl* ctl;
};

// The merge's buffers for `total` pairs laid out one after another from
// base (256-byte aligned pieces); returns the bytes they span.  base ==
// nullptr only measures.
uint64_t merge_layout(uint64_t total, uint8_t* base, MergeBufs* b) {
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += (std::max<uint64_t>(bytes, 1) + 255) & ~255ull;
    return p;
  };
  const uint32_t nt = radix_tiles(total, 0);
  b->k0 = static_cast<uint64_t*>(take(8 * total));
  b->k1 = static_cast<uint64_t*>(take(8 * total));
  b->v0 = static_cast<uint32_t*>(take(4 * total));
  b->v1 = static_cast<uint32_t*>(take(4 * total));
  b->hist = static_cast<uint32_t*>(take(4ull * 256 * nt));
  b->sums = static_cast<uint32_t*>(take(4 * scan_sums_elems((uint64_t)256 * nt, 1)));
  b->keep = static_cast<uint64_t*>(take(8 * total));
  b->sums64 = static_cast<uint64_t*>(take(8 * (scan_sums_elems(total, 1) + 1)));
  b->tot = static_cast<uint32_t*>(take(4 * total));
  b->ctl = static_cast<AlignCtrl*>(take(sizeof(AlignCtrl)));
  return off;
}

int merge_check(fast_lsh_ctx* c, uint32_t n_channels, const fast_lsh_pairs* ch, uint64_t n_fps, uint64_t* n_out,
                uint64_t* total) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  if (!n_out) return fl_fail(FAST_LSH_E_INVALID, "n_out is NULL");
  *n_out = 0;
  if (n_channels > 0 && !ch) return fl_fail(FAST_LSH_E_INVALID, "channels is NULL");
  if (n_fps >= (1ull << 32))
    return fl_fail(FAST_LSH_E_INVALID, "n_fingerprints %llu must be below 2^32", (unsigned long long)n_fps);
  *total = 0;
  for (uint32_t q = 0; q < n_channels; ++q) {
    if (ch[q].count && (!ch[q].i || !ch[q].j || !ch[q].votes))
      return fl_fail(FAST_LSH_E_INVALID, "channel %u has a NULL array", q);
    *total += ch[q].count;
  }
  return FAST_LSH_OK;
}

// Pack, sort, sum and compact (total > 0 pairs) with the buffers in b.
int merge_run(fast_lsh_ctx* c, uint32_t n_channels, const fast_lsh_pairs* ch, uint64_t n_fps, uint32_t min_sim,
              uint64_t total, const MergeBufs& b, bool prof, uint32_t* odt, uint32_t* oidx, uint32_t* osim,
              uint64_t capacity, uint64_t* n_out) {
  hipStream_t s = c->stream;
  uint64_t *k0 = b.k0, *k1 = b.k1;
  uint32_t *v0 = b.v0, *v1 = b.v1;
  fill_u8(reinterpret_cast<uint8_t*>(b.ctl), sizeof(AlignCtrl), 0, s);
  if (prof) prof_begin(c, FAST_LSH_STAGE_CHANNEL_MERGE);
  uint64_t off = 0;
  for (uint32_t q = 0; q < n_channels; ++q) {
    if (ch[q].count == 0) continue;
    hipLaunchKernelGGL(k_pack_pairs, dim3(grid_of(ch[q].count)), dim3(kAT), 0, s, ch[q].i, ch[q].j, ch[q].votes,
                       ch[q].count, n_fps, k0 + off, v0 + off, &b.ctl->err);
    off += ch[q].count;
  }
  // LSD passes: the idx1 bits, then the dt bits (both below n_fps)
  const uint32_t nb = fl_key_bits((uint32_t)std::max<uint64_t>(n_fps, 2));
  for (uint32_t base : {0u, 32u})
    for (uint32_t sh = 0; sh < nb; sh += 8) {
      radix_pass(k0, v0, k1, v1, total, 1, base + sh, b.hist, b.sums, 0, s);
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
  hipLaunchKernelGGL(k_merge_heads, dim3(grid_of(total)), dim3(kAT), 0, s, k0, v0, total, min_sim, b.keep, b.tot);
  uint64_t* count = b.sums64 + scan_sums_elems(total, 1);
  scan_u64(b.keep, total, 1, b.sums64, count, s);
  if (prof) prof_end(c);
  LAUNCHCK();
  uint64_t m = 0;
  RC(d2h(c, &m, count));
  AlignCtrl hc;
  RC(d2h(c, &hc, b.ctl));
  if (hc.err) {
    if (prof) prof_collect(c);
    return fl_fail(FAST_LSH_E_INVALID, "a channel holds a pair with j <= i or an id >= %llu",
                   (unsigned long long)n_fps);
  }
  *n_out = m;
  if (m > capacity) {
    if (prof) prof_collect(c);
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu merged entries do not fit capacity %llu", (unsigned long long)m,
                   (unsigned long long)capacity);
  }
  if (m && (!odt || !oidx || !osim)) return fl_fail(FAST_LSH_E_INVALID, "output pointer is NULL");
  if (prof) prof_begin(c, FAST_LSH_STAGE_CHANNEL_MERGE);
  if (m)
    hipLaunchKernelGGL(k_merge_emit, dim3(grid_of(total)), dim3(kAT), 0, s, k0, b.tot, b.keep, total, m, odt, oidx,
                       osim);
  if (prof) prof_end(c);
  LAUNCHCK();
  HIPCK(hipStreamSynchronize(s));
  if (prof) prof_collect(c);
  return FAST_LSH_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free merge: one array per device, held by the
// code object until the process ends.  Host code never passes the array's
// name to a kernel: it passes the device address hipGetSymbolAddress gives
// for the current device, taken once per device.
// ---------------------------------------------------------------------------
constexpr uint64_t kScratchBytes = FAST_LSH_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxScratchDevices = 64;
__device__ __align__(256) uint8_t scratch[kScratchBytes];
void* g_scratch_ptr[kMaxScratchDevices];
std::mutex g_scratch_mu;

int scratch_ptr(int device, uint8_t** out) {
  if (device < 0 || device >= kMaxScratchDevices)
    return fl_fail(FAST_LSH_E_INVALID, "device %d: the allocation-free calls serve devices 0-%d", device,
                   kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the current device's copy
    if (e != hipSuccess || !p)
      return fl_fail(FAST_LSH_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                     hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = static_cast<uint8_t*>(g_scratch_ptr[device]);
  return FAST_LSH_OK;
}

// Largest pair count whose merge layout fits the scratch array.
uint64_t noalloc_max_pairs() {
  // largest total whose layout fits the scratch array (the layout grows with total)
  uint64_t lo = 0, hi = kScratchBytes / 36 + 1;
  MergeBufs b;
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (merge_layout(mid, nullptr, &b) <= kScratchBytes) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace

// Taken at context creation, with the context's device current.
int fl_scratch_init(int device) {
  uint8_t* p = nullptr;
  return scratch_ptr(device, &p);
}

extern "C" {

int fast_lsh_channel_merge(fast_lsh_ctx* c, uint32_t n_channels, const fast_lsh_pairs* ch, uint64_t n_fps,
                           uint32_t min_sim, uint32_t* odt, uint32_t* oidx, uint32_t* osim, uint64_t capacity,
                           uint64_t* n_out) {
  uint64_t total = 0;
  RC(merge_check(c, n_channels, ch, n_fps, n_out, &total));
  HIPCK(hipSetDevice(c->device));
  if (total == 0) return FAST_LSH_OK;
  MergeBufs b;
  const uint64_t bytes = merge_layout(total, nullptr, &b);
  uint8_t* base;
  RC(ws<uint8_t>(c, "cm_arena", bytes, &base));
  merge_layout(total, base, &b);
  return merge_run(c, n_channels, ch, n_fps, min_sim, total, b, true, odt, oidx, osim, capacity, n_out);
}

int fast_lsh_channel_merge_noalloc(fast_lsh_ctx* c, uint32_t n_channels, const fast_lsh_pairs* ch, uint64_t n_fps,
                                   uint32_t min_sim, uint32_t* odt, uint32_t* oidx, uint32_t* osim,
                                   uint64_t capacity, uint64_t* n_out) {
  uint64_t total = 0;
  RC(merge_check(c, n_channels, ch, n_fps, n_out, &total));
  HIPCK(hipSetDevice(c->device));
  if (total == 0) return FAST_LSH_OK;
  MergeBufs b;
  const uint64_t bytes = merge_layout(total, nullptr, &b);
  if (bytes > kScratchBytes)
    return fl_fail(FAST_LSH_E_NOMEM, "%llu pairs need %llu bytes of scratch; the allocation-free merge holds %llu "
                   "(at most %llu pairs)", (unsigned long long)total, (unsigned long long)bytes,
                   (unsigned long long)kScratchBytes, (unsigned long long)noalloc_max_pairs());
  uint8_t* base = nullptr;
  RC(scratch_ptr(c->device, &base));
  merge_layout(total, base, &b);
  return merge_run(c, n_channels, ch, n_fps, min_sim, total, b, false, odt, oidx, osim, capacity, n_out);
}

int fast_lsh_station_clusters(fast_lsh_ctx* c, const uint32_t* dt, const uint32_t* idx1, const uint32_t* sim,
                              uint64_t n, const fast_lsh_cluster_params* prm, fast_lsh_cluster* out,
                              uint64_t capacity, uint64_t* n_out) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  if (!prm || !n_out) return fl_fail(FAST_LSH_E_INVALID, "params or n_out is NULL");
  *n_out = 0;
  if (n >= (1ull << 32)) return fl_fail(FAST_LSH_E_INVALID, "n = %llu entries must be below 2^32", (unsigned long long)n);
  if (n && (!dt || !idx1 || !sim)) return fl_fail(FAST_LSH_E_INVALID, "an entry array is NULL");
  HIPCK(hipSetDevice(c->device));
  if (n == 0) return FAST_LSH_OK;
  hipStream_t s = c->stream;
  const uint32_t gap = prm->max_gap;
  uint64_t *rs, *ssum, *keep, *ksum;
  uint32_t *rdt, *rlo, *rhi, *parent;
  AlignCtrl* ctl;
  RC(ws<uint64_t>(c, "sc_rs", n, &rs));
  RC(ws<uint64_t>(c, "sc_ssum", scan_sums_elems(n, 1) + 1, &ssum));
  RC(ws<AlignCtrl>(c, "al_ctrl", 1, &ctl));
  fill_u8(reinterpret_cast<uint8_t*>(ctl), sizeof(AlignCtrl), 0, s);
  prof_begin(c, FAST_LSH_STAGE_CLUSTERS);
  hipLaunchKernelGGL(k_run_heads, dim3(grid_of(n)), dim3(kAT), 0, s, dt, idx1, sim, n, gap, rs, &ctl->err);
  scan_u64(rs, n, 1, ssum, &ctl->runs, s);
  prof_end(c);
  LAUNCHCK();
  AlignCtrl hc;
  RC(d2h(c, &hc, ctl));
  if (hc.err) {
    prof_collect(c);
    return fl_fail(FAST_LSH_E_INVALID, hc.err == 3 ? "a similarity is 2^24 or more"
                                                    : "entries are not strictly ordered by (dt, idx1)");
  }
  const uint32_t R = (uint32_t)hc.runs;
  RC(ws<uint32_t>(c, "sc_rdt", R, &rdt));
  RC(ws<uint32_t>(c, "sc_rlo", R, &rlo));
  RC(ws<uint32_t>(c, "sc_rhi", R, &rhi));
  RC(ws<uint32_t>(c, "sc_parent", R, &parent));
  ClusterAcc acc;
  RC(ws<uint32_t>(c, "sc_dtmax", R, &acc.dtmax));
  RC(ws<uint32_t>(c, "sc_xmin", R, &acc.xmin));
  RC(ws<uint32_t>(c, "sc_xmax", R, &acc.xmax));
  RC(ws<uint32_t>(c, "sc_cnt", R, &acc.cnt));
  RC(ws<unsigned long long>(c, "sc_sum", R, &acc.sum));
  RC(ws<unsigned long long>(c, "sc_peak", R, &acc.peak));
  RC(ws<uint64_t>(c, "sc_keep", R, &keep));
  RC(ws<uint64_t>(c, "sc_ksum", scan_sums_elems(R, 1) + 1, &ksum));
  prof_begin(c, FAST_LSH_STAGE_CLUSTERS);
  hipLaunchKernelGGL(k_run_table, dim3(grid_of(n)), dim3(kAT), 0, s, dt, idx1, n, gap, rs, rdt, rlo, rhi, parent);
  hipLaunchKernelGGL(k_run_links, dim3(grid_of(R)), dim3(kAT), 0, s, rdt, rlo, rhi, R, gap, parent);
  hipLaunchKernelGGL(k_run_compress, dim3(grid_of(R)), dim3(kAT), 0, s, parent, R);
  hipLaunchKernelGGL(k_cluster_init, dim3(grid_of(R)), dim3(kAT), 0, s, acc, R);
  hipLaunchKernelGGL(k_cluster_stats, dim3(grid_of(n)), dim3(kAT), 0, s, dt, idx1, sim, n, gap, rs, parent, acc);
  hipLaunchKernelGGL(k_cluster_keep, dim3(grid_of(R)), dim3(kAT), 0, s, parent, rdt, acc, R, prm->max_width,
                     prm->min_entries, prm->min_sum, keep);
  scan_u64(keep, R, 1, ksum, ksum + scan_sums_elems(R, 1), s);
  prof_end(c);
  LAUNCHCK();
  uint64_t m = 0;
  RC(d2h(c, &m, ksum + scan_sums_elems(R, 1)));
  *n_out = m;
  if (m > capacity) {
    prof_collect(c);
    return fl_fail(FAST_LSH_E_CAPACITY, "%llu clusters do not fit capacity %llu", (unsigned long long)m,
                   (unsigned long long)capacity);
  }
  if (m && !out) return fl_fail(FAST_LSH_E_INVALID, "out is NULL");
  prof_begin(c, FAST_LSH_STAGE_CLUSTERS);
  if (m) hipLaunchKernelGGL(k_cluster_emit, dim3(grid_of(R)), dim3(kAT), 0, s, rdt, acc, keep, R, m, dt, idx1, out);
  prof_end(c);
  LAUNCHCK();
  HIPCK(hipStreamSynchronize(s));
  prof_collect(c);
  return FAST_LSH_OK;
}

}  // extern "C"
