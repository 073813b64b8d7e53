// Signature kernels: MinHash (section 6.1) and Min-Max (section 6.2) values
// over sparse binary fingerprints and the band key of every table.
//
// Layout choice for gfx950: one fingerprint per lane.  The lane keeps the
// fingerprint's element indices in VGPRs (two 16-bit indices per register),
// so the inner loop is pure integer VALU work: the hash parameters of the
// current function are wave-uniform (scalar loads), no reductions across
// lanes are needed, and the 64 keys a wave produces for one table are 64
// consecutive 8-byte words (one coalesced store).  Every function's
// arguments are recovered after the loop from its min/max values by the
// inverse of the hash (x = (v - b) a^-1 mod p), so the loop carries only the
// 32-bit extremes.  This keeps the paper's dimension-major loop order
// (Appendix D, Algorithm 1): each set element is read once per function
// pair, here from registers.
#include "common.hpp"

namespace fl {

// Running extremes of two functions over the set elements, kept on
// t = hash_fold2 (twice the folded value s, wrapped): one multiply-add and
// one shift-add per evaluation, then three-input min and max (two elements
// per instruction).  While every s is below p, s is the hash value and the
// extremes of t are twice the exact extremes.  An element with s >= p shows
// up as a maximum of 2p (s = p) or as a minimum below 2 dim (s >= 2^31
// wraps there); then (about 4e-4 of the functions at d = 4,096, counting the
// genuine minima that small) the function's extremes are recomputed from the
// canonical values (exact()).  The maximum is kept for MinHash too, as that
// check.
template <bool MINMAX>
struct PairAcc {
  uint32_t mnA, mxA, mnB, mxB;
  __device__ __forceinline__ void init() {
    mnA = mnB = 0xFFFFFFFFu;
    mxA = mxB = 0u;
  }
  __device__ __forceinline__ void add(uint32_t a2A, uint32_t b2A, uint32_t a2B, uint32_t b2B, uint32_t v) {
    const uint32_t x0 = v & 0xFFFFu, x1 = v >> 16;
    const uint32_t tA0 = hash_fold2(a2A, b2A, x0), tA1 = hash_fold2(a2A, b2A, x1);
    const uint32_t tB0 = hash_fold2(a2B, b2B, x0), tB1 = hash_fold2(a2B, b2B, x1);
    mnA = min(mnA, min(tA0, tA1));
    mnB = min(mnB, min(tB0, tB1));
    mxA = max(mxA, max(tA0, tA1));
    mxB = max(mxB, max(tB0, tB1));
    // Serialise the running extremes: otherwise the compiler regroups the
    // min and max reductions into separate trees and keeps every hash value
    // of the row alive in registers.
    asm volatile("" : "+v"(mnA), "+v"(mxA), "+v"(mnB), "+v"(mxB));
  }
  // Canonical extremes of one function, from every packed element pair that
  // `each` hands to the callback.
  template <typename Each>
  __device__ __forceinline__ static void exact(uint32_t a2, uint32_t b2, Each each, uint32_t& mn, uint32_t& mx) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    each([&](uint32_t v) {
      const uint32_t h0 = hash_mod(a2, b2, v & 0xFFFFu), h1 = hash_mod(a2, b2, v >> 16);
      lo = min(lo, min(h0, h1));
      hi = max(hi, max(h0, h1));
    });
    mn = lo;
    mx = hi;
  }
  // Hash values of the extremes (canonical), with dim the index bound.
  template <typename Each>
  __device__ __forceinline__ void finish(uint32_t a2A, uint32_t b2A, uint32_t a2B, uint32_t b2B, uint32_t dim,
                                         Each each) {
    const uint32_t wrap = 2u * dim;
    if (mxA >= 2u * kP || mnA < wrap) exact(a2A, b2A, each, mnA, mxA); else { mnA >>= 1; mxA >>= 1; }
    if (mxB >= 2u * kP || mnB < wrap) exact(a2B, b2B, each, mnB, mxB); else { mnB >>= 1; mxB >>= 1; }
  }
};

struct KeyBuilder {
  uint64_t key;
  uint32_t row;
  __device__ __forceinline__ void put(const SigArgs& a, uint32_t f, uint32_t v, uint64_t i, uint32_t u, bool live) {
    const uint32_t bf = a.b[f];
    const uint32_t d = v >= bf ? v - bf : v + kP - bf;
    const uint32_t x = mul_mod(d, a.ainv[f]);
    if (a.packed)
      key |= (uint64_t)x << (a.kbits * row);
    else
      key = fmix64(key + x + 1);
    if (a.sigs && live) a.sigs[(i * a.table_count + u) * a.r + row] = v;
    ++row;
  }
};

// Keys of table u for this lane's fingerprint; the sub-key goes into the
// lane's row under construction in LDS (`my`, row_dw dwords).
__device__ __forceinline__ void store_table(const SigArgs& a, uint64_t key, uint64_t i, uint32_t u, bool live,
                                            uint32_t* my) {
  const uint32_t tab = a.table_begin + u;
  if (live && a.keys) a.keys[(uint64_t)u * a.n + i] = key;
  if (a.mkeys || a.rows || a.hi32) {
    const uint64_t m = a.mix == kMixSplit ? mix48(key) << 16
                                          : (a.mix == kMixStation ? (a.tag | mix60(key)) : fmix64(key));
    if (live && a.mkeys) a.mkeys[(uint64_t)u * a.out_stride + a.out_base + i] = m;
    if (live && a.hi32) a.hi32[(uint64_t)tab * a.out_stride + a.out_base + i] = (uint32_t)(m >> 32);
    if (a.rows) {
      const uint32_t slot = tab % a.tables_per_group;
      if (slot == 0)
        for (uint32_t w = 0; w < a.row_dw; ++w) my[w] = 0;
      const uint32_t sub = (uint32_t)(m >> (a.mix == kMixSplit ? 16 : 0)) & kSubMask;
      my[slot >> 1] |= sub << (16 * (slot & 1));
    }
  }
}

// A launch that starts inside a group of tables continues the rows an
// earlier launch began: the lane's row of that group is loaded first.
__device__ __forceinline__ void resume_row(const SigArgs& a, uint64_t i, bool live, uint32_t* my) {
  if (!a.rows || a.table_begin % a.tables_per_group == 0) return;
  const uint32_t g = a.table_begin / a.tables_per_group;
  const uint32_t* src = a.rows + ((uint64_t)g * a.out_stride + a.out_base + i) * a.row_pitch;
  for (uint32_t w = 0; w < a.row_dw; ++w) my[w] = live ? src[w] : 0u;
}

// After the last table of a group: the workgroup's 256 rows of that group
// are contiguous in HBM; copy them out with consecutive lanes on
// consecutive dwords.
__device__ __forceinline__ void flush_rows(const SigArgs& a, uint32_t u, const uint32_t* srow) {
  const uint32_t tab = a.table_begin + u;
  const uint32_t slot = tab % a.tables_per_group;
  if (!a.rows || (slot + 1 != a.tables_per_group && u + 1 != a.table_count)) return;
  __syncthreads();
  const uint32_t g = tab / a.tables_per_group;
  const uint64_t i0 = (uint64_t)blockIdx.x * 256;
  const uint32_t live = (uint32_t)min((uint64_t)256, a.n - i0);
  uint32_t* dst = a.rows + ((uint64_t)g * a.out_stride + a.out_base + i0) * a.row_pitch;
  for (uint32_t idx = threadIdx.x; idx < live * a.row_dw; idx += 256) {
    const uint32_t r = idx / a.row_dw, w = idx - r * a.row_dw;
    dst[r * a.row_pitch + w] = srow[r * (a.row_dw + 1) + w];
  }
  __syncthreads();
}

// One pass over the register-resident row: functions [F, F + KP) of the
// launch (those past Fn are repeats of its last function and are not
// placed), their values placed into the key under construction, and each
// table stored when its last function is placed.
template <int KP, int W, bool MINMAX, typename Each>
__device__ __forceinline__ void sig_pass(const SigArgs& a, uint32_t F, uint32_t F0, uint32_t Fn, uint32_t (&xs)[W],
                                         Each each_pair, KeyBuilder& kb, uint64_t i, bool live, uint32_t* my,
                                         uint32_t* srow) {
  uint32_t f[KP], a2[KP], b2[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    f[k] = min(F + k, Fn - 1);
    a2[k] = a.a2[f[k]];
    b2[k] = a.b2[f[k]];
  }
  PairAcc<MINMAX> acc[KP / 2];
#pragma unroll
  for (int k = 0; k < KP / 2; ++k) acc[k].init();
#pragma unroll
  for (int w = 0; w < W; ++w) asm volatile("" : "+v"(xs[w]));
#pragma clang loop unroll(full)
  for (int w = 0; w < W; ++w) {
#pragma unroll
    for (int k = 0; k < KP / 2; ++k) acc[k].add(a2[2 * k], b2[2 * k], a2[2 * k + 1], b2[2 * k + 1], xs[w]);
  }
#pragma unroll
  for (int k = 0; k < KP / 2; ++k) acc[k].finish(a2[2 * k], b2[2 * k], a2[2 * k + 1], b2[2 * k + 1], a.dim, each_pair);
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (F + k >= Fn) break;
    const uint32_t u = (F + k - F0) / a.fpt;
    const PairAcc<MINMAX>& c = acc[k / 2];
    kb.put(a, f[k], (k & 1) ? c.mnB : c.mnA, i, u, live);
    if (MINMAX) kb.put(a, f[k], (k & 1) ? c.mxB : c.mxA, i, u, live);
    if ((F + k + 1 - F0) % a.fpt == 0) {
      store_table(a, kb.key, i, u, live, my);
      flush_rows(a, u, srow);
      kb = KeyBuilder{0ull, 0u};
    }
  }
}

// CAP: most indices a row may hold (rows shorter than CAP are padded with
// their first index, which leaves every min and max unchanged).  Rows are
// fixed-length with an even length and 4-byte aligned (other layouts take
// k_sig_long).  Each pass over the register-resident row evaluates eight
// functions (four in a short last pass), so the 16-bit unpacking of an index
// pair is shared by eight.
template <int CAP, bool MINMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CAP <= 200 ? 3 : 1))) void k_sig(SigArgs a) {
  extern __shared__ uint32_t srow[];  // 256 rows of row_dw + 1 dwords (odd stride)
  uint32_t* my = srow + threadIdx.x * (a.row_dw + 1);
  constexpr int W = CAP / 2;
  const uint64_t gi = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = gi < a.n;
  const uint64_t i = live ? gi : a.n - 1;
  uint64_t lo, len;
  if (a.off) {
    lo = a.off[i];
    len = a.off[i + 1] - lo;
  } else {
    lo = i * a.nnz;
    len = a.nnz;
  }
  bool bad = (len == 0) || (len > (uint64_t)CAP);
  uint32_t xs[W];
  if (a.vec_load) {
    const uint4* p = reinterpret_cast<const uint4*>(a.ind + lo);
#pragma unroll
    for (int q = 0; q < CAP / 8; ++q) {
      const uint4 v = p[q];
      xs[4 * q + 0] = v.x;
      xs[4 * q + 1] = v.y;
      xs[4 * q + 2] = v.z;
      xs[4 * q + 3] = v.w;
    }
  } else {
    // Fixed even row length below CAP, 4-byte aligned rows: dword loads,
    // the tail padded with the row's first index.
    const uint32_t* p = reinterpret_cast<const uint32_t*>(a.ind + lo);
    const uint32_t half = (uint32_t)(len / 2);
    const uint32_t first = len ? (uint32_t)a.ind[lo] * 0x10001u : 0u;
#pragma unroll
    for (int w = 0; w < W; ++w) xs[w] = (uint32_t)w < half ? p[w] : first;
  }
  uint32_t top = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) top = max(top, max(xs[w] & 0xFFFFu, xs[w] >> 16));
  if (top >= a.dim) bad = true;
  if (live && bad) *a.err = 1;
  resume_row(a, i, live, my);

  // the rare exact recomputation reads the row from memory (indexing the
  // registers would move them to scratch)
  auto each_pair = [&](auto&& f) {
    for (uint64_t k = 0; k < len; k += 2) {
      const uint32_t x0 = a.ind[lo + k];
      const uint32_t x1 = k + 1 < len ? a.ind[lo + k + 1] : x0;
      f(x0 | (x1 << 16));
    }
  };
  // Functions of the launch's tables in order (table-major), eight per pass;
  // a remainder of at most four takes a four-function pass, so a launch of
  // 4 (mod 8) functions evaluates no repeats.  A table's key is complete
  // after its last function's values are placed.
  const uint32_t F0 = a.table_begin * a.fpt, Fn = F0 + a.table_count * a.fpt;
  KeyBuilder kb{0ull, 0u};
  // (F + 4 < Fn, not Fn - F > 4: a pass over a remainder of five to seven
  // functions leaves F past Fn)
  uint32_t F = F0;
  for (; F + 4 < Fn; F += 8) sig_pass<8, W, MINMAX>(a, F, F0, Fn, xs, each_pair, kb, i, live, my, srow);
  if (F < Fn) sig_pass<4, W, MINMAX>(a, F, F0, Fn, xs, each_pair, kb, i, live, my, srow);
}

// Rows longer than the largest register-resident capacity: indices are read
// from memory once per function pair.
template <bool MINMAX>
__global__ __launch_bounds__(256) void k_sig_long(SigArgs a) {
  extern __shared__ uint32_t srow[];
  uint32_t* my = srow + threadIdx.x * (a.row_dw + 1);
  const uint64_t gi = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = gi < a.n;
  const uint64_t i = live ? gi : a.n - 1;
  uint64_t lo, len;
  if (a.off) {
    lo = a.off[i];
    len = a.off[i + 1] - lo;
  } else {
    lo = i * a.nnz;
    len = a.nnz;
  }
  bool bad = len == 0;
  for (uint64_t k = 0; k < len; ++k)
    if (a.ind[lo + k] >= a.dim) bad = true;
  if (live && bad) *a.err = 1;  // (empty rows never reach this kernel: the host rejects them)
  resume_row(a, i, live, my);

  for (uint32_t u = 0; u < a.table_count; ++u) {
    const uint32_t f0 = (a.table_begin + u) * a.fpt;
    KeyBuilder kb{0ull, 0u};
    for (uint32_t q = 0; q < a.fpt; q += 2) {
      const uint32_t fA = f0 + q;
      const bool two = q + 1 < a.fpt;
      const uint32_t fB = two ? fA + 1 : fA;
      const uint32_t a2A = a.a2[fA], b2A = a.b2[fA], a2B = a.a2[fB], b2B = a.b2[fB];
      PairAcc<MINMAX> acc;
      acc.init();
      auto each = [&](auto&& f) {
        for (uint64_t k = 0; k < len; k += 2) {
          const uint32_t x0 = a.ind[lo + k];
          const uint32_t x1 = k + 1 < len ? a.ind[lo + k + 1] : x0;
          f(x0 | (x1 << 16));
        }
      };
      each([&](uint32_t v) { acc.add(a2A, b2A, a2B, b2B, v); });
      acc.finish(a2A, b2A, a2B, b2B, a.dim, each);
      kb.put(a, fA, acc.mnA, i, u, live);
      if (MINMAX) kb.put(a, fA, acc.mxA, i, u, live);
      if (two) {
        kb.put(a, fB, acc.mnB, i, u, live);
        if (MINMAX) kb.put(a, fB, acc.mxB, i, u, live);
      }
    }
    store_table(a, kb.key, i, u, live, my);
    flush_rows(a, u, srow);
  }
}

// Largest and smallest row length of a ragged set (for kernel selection and
// the empty-row check).
__global__ __launch_bounds__(256) void k_row_len_range(const uint64_t* off, uint64_t n, unsigned long long* out) {
  uint64_t mx = 0, mn = ~0ull;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint64_t L = off[i + 1] - off[i];
    mx = L > mx ? L : mx;
    mn = L < mn ? L : mn;
  }
  for (int s = 32; s > 0; s >>= 1) {
    const uint64_t omx = __shfl_xor(mx, s, 64), omn = __shfl_xor(mn, s, 64);
    mx = omx > mx ? omx : mx;
    mn = omn < mn ? omn : mn;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out + 0, (unsigned long long)mx);
    atomicMin(out + 1, (unsigned long long)mn);
  }
}

// ---------------------------------------------------------------------------
// Host-side launcher
// ---------------------------------------------------------------------------
static const int kCaps[] = {16, 32, 64, 128, 200, 256};

int sig_capacity_for(uint64_t max_len) {
  for (int c : kCaps)
    if ((uint64_t)c >= max_len) return c;
  return 0;  // long-row kernel
}

template <bool MM>
static void launch_cap(int cap, dim3 g, dim3 b, hipStream_t s, const SigArgs& a) {
  const size_t sm = a.rows ? (size_t)256 * (a.row_dw + 1) * 4 : 0;
  switch (cap) {
    case 16: hipLaunchKernelGGL((k_sig<16, MM>), g, b, sm, s, a); break;
    case 32: hipLaunchKernelGGL((k_sig<32, MM>), g, b, sm, s, a); break;
    case 64: hipLaunchKernelGGL((k_sig<64, MM>), g, b, sm, s, a); break;
    case 128: hipLaunchKernelGGL((k_sig<128, MM>), g, b, sm, s, a); break;
    case 200: hipLaunchKernelGGL((k_sig<200, MM>), g, b, sm, s, a); break;
    case 256: hipLaunchKernelGGL((k_sig<256, MM>), g, b, sm, s, a); break;
    default: hipLaunchKernelGGL((k_sig_long<MM>), g, b, sm, s, a); break;
  }
}

void launch_sig(int cap, bool minmax, const SigArgs& a, hipStream_t s) {
  if (a.n == 0) return;
  const dim3 g((unsigned)((a.n + 255) / 256)), b(256);
  if (minmax)
    launch_cap<true>(cap, g, b, s, a);
  else
    launch_cap<false>(cap, g, b, s, a);
}

void launch_row_len_range(const uint64_t* off, uint64_t n, unsigned long long* out, hipStream_t s) {
  const uint64_t blocks = (n + 255) / 256;
  const unsigned g = (unsigned)(blocks < 4096 ? (blocks ? blocks : 1) : 4096);
  hipLaunchKernelGGL(k_row_len_range, dim3(g), dim3(256), 0, s, off, n, out);
}

}  // namespace fl
