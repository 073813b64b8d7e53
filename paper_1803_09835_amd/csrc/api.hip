// C-ABI entry points and host orchestration of the fast_lsh library.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "common.hpp"
#include "fast_lsh.h"

namespace fl {
// sig.hip
int sig_capacity_for(uint64_t max_len);
void launch_sig(int cap, bool minmax, const SigArgs& a, hipStream_t s);
void launch_row_len_range(const uint64_t* off, uint64_t n, unsigned long long* out, hipStream_t s);
// sort.hip
uint32_t radix_tiles(uint64_t n);
uint64_t scan_sums_elems(uint64_t len, uint32_t S);
void scan_u64(uint64_t* data, uint64_t len, uint32_t S, uint64_t* sums, uint64_t* seg_total, hipStream_t s);
void radix_pass(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, uint64_t n, uint32_t S,
                uint32_t shift, uint32_t* hist, uint32_t* sums, hipStream_t s);
void launch_bucket(const BucketArgs& a, uint32_t S, hipStream_t s);
void launch_bigbin(const BucketArgs& a, const uint4* bins, uint32_t nbins, uint64_t* tk, uint32_t* tv,
                   hipStream_t s);
// pairs.hip
void launch_pairs_wave(const PairArgs& a, const uint8_t* marks, uint32_t S, uint32_t rswl, uint32_t use_flags,
                       hipStream_t s);
void launch_compact_big(const PairArgs& a, const uint4* big, uint32_t nbig, const uint64_t* cofs, uint32_t* ids,
                        uint32_t* cnt, hipStream_t s);
void launch_pairs_tile(const PairArgs& a, const TileUnit* units, uint32_t nunits, const uint4* big,
                       const uint64_t* cofs, const uint32_t* ids, const uint32_t* cnt, uint32_t tb_size,
                       uint32_t rswl, hipStream_t s);
void launch_split_out(const uint64_t* key, const uint32_t* val, uint64_t count, uint32_t* oi, uint32_t* oj,
                      uint8_t* ov, hipStream_t s);
void launch_pack_out(const uint32_t* oi, const uint32_t* oj, const uint8_t* ov, uint64_t count, uint64_t* key,
                     uint32_t* val, hipStream_t s);
void launch_count_flags(const uint8_t* flags, uint64_t n, unsigned long long* out, hipStream_t s);
void fill_u8(uint8_t* p, uint64_t count, uint8_t v, hipStream_t s);
void fill_u32(uint32_t* p, uint64_t count, uint32_t v, hipStream_t s);
void fill_u64(uint64_t* p, uint64_t count, uint64_t v, hipStream_t s);
}  // namespace fl

using namespace fl;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCK(expr)                                                                              \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return fail(FAST_LSH_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCK()                                                                                     \
  do {                                                                                                 \
    hipError_t e_ = hipGetLastError();                                                                 \
    if (e_ != hipSuccess) return fail(FAST_LSH_E_DEVICE, "kernel launch (line %d): %s", __LINE__, \
                                      hipGetErrorString(e_));                                         \
  } while (0)

#define RC(expr)                    \
  do {                              \
    int rc_ = (expr);               \
    if (rc_ != FAST_LSH_OK) return rc_; \
  } while (0)

// ---------------------------------------------------------------------------
// Context and workspace
// ---------------------------------------------------------------------------
struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

struct fast_lsh_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t budget = 0;
  std::map<std::string, Buf> ws;
  uint64_t ws_total = 0;
  std::vector<uint32_t> hparams;  // host staging for hash parameters
  std::vector<uint64_t> hstage;   // host staging for small uploads
  uint64_t res_count = 0;
  bool res_valid = false;
  // stage timing (HIP events on the context stream around each launch)
  static constexpr int kMaxRec = 256;
  bool prof = false;
  std::vector<hipEvent_t> ev;
  int rec_stage[kMaxRec];
  int nrec = 0;
  double prof_ms[FAST_LSH_PROFILE_STAGES] = {0};
  uint64_t prof_launches[FAST_LSH_PROFILE_STAGES] = {0};
};

static void prof_begin(fast_lsh_ctx* c, int stage) {
  if (!c->prof || c->nrec >= fast_lsh_ctx::kMaxRec) return;
  if (c->ev.empty()) {
    c->ev.resize(2 * fast_lsh_ctx::kMaxRec);
    for (auto& e : c->ev) (void)hipEventCreate(&e);
  }
  c->rec_stage[c->nrec] = stage;
  (void)hipEventRecord(c->ev[2 * c->nrec], c->stream);
}

static void prof_end(fast_lsh_ctx* c) {
  if (!c->prof || c->nrec >= fast_lsh_ctx::kMaxRec) return;
  (void)hipEventRecord(c->ev[2 * c->nrec + 1], c->stream);
  ++c->nrec;
}

// Accumulate recorded intervals (the caller has synchronised the stream).
static void prof_collect(fast_lsh_ctx* c) {
  for (int k = 0; k < c->nrec; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]) == hipSuccess) {
      c->prof_ms[c->rec_stage[k]] += ms;
      c->prof_launches[c->rec_stage[k]] += 1;
    }
  }
  c->nrec = 0;
}

static int ws_get(fast_lsh_ctx* c, const char* name, size_t bytes, void** out) {
  Buf& b = c->ws[name];
  const size_t want = bytes ? (bytes + 255) & ~(size_t)255 : 256;
  if (b.p && b.cap >= want) {
    *out = b.p;
    return FAST_LSH_OK;
  }
  if (b.p) {
    HIPCK(hipStreamSynchronize(c->stream));
    HIPCK(hipFree(b.p));
    c->ws_total -= b.cap;
    b = Buf();
  }
  if (c->budget && c->ws_total + want > c->budget)
    return fail(FAST_LSH_E_NOMEM, "workspace '%s' (%zu bytes) exceeds the HBM budget (%llu in use of %llu)", name,
                want, (unsigned long long)c->ws_total, (unsigned long long)c->budget);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(FAST_LSH_E_NOMEM, "hipMalloc of workspace '%s' (%zu bytes) failed", name, want);
  }
  b.cap = want;
  c->ws_total += want;
  *out = b.p;
  return FAST_LSH_OK;
}

template <typename T>
static int ws(fast_lsh_ctx* c, const char* name, uint64_t count, T** out) {
  void* p = nullptr;
  RC(ws_get(c, name, count * sizeof(T), &p));
  *out = static_cast<T*>(p);
  return FAST_LSH_OK;
}

template <typename T>
static int d2h(fast_lsh_ctx* c, T* host, const T* dev, uint64_t count = 1) {
  HIPCK(hipMemcpyAsync(host, dev, count * sizeof(T), hipMemcpyDeviceToHost, c->stream));
  HIPCK(hipStreamSynchronize(c->stream));
  return FAST_LSH_OK;
}

template <typename T>
static int h2d(fast_lsh_ctx* c, T* dev, const T* host, uint64_t count) {
  if (count == 0) return FAST_LSH_OK;
  HIPCK(hipMemcpyAsync(dev, host, count * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HIPCK(hipStreamSynchronize(c->stream));
  return FAST_LSH_OK;
}

// ---------------------------------------------------------------------------
// Hash parameters
// ---------------------------------------------------------------------------
static uint64_t splitmix64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint32_t pow_mod(uint32_t a, uint32_t e) {
  uint64_t r = 1, x = a;
  while (e) {
    if (e & 1) r = r * x % kP;
    x = x * x % kP;
    e >>= 1;
  }
  return (uint32_t)r;
}

static uint32_t n_funcs(const fast_lsh_hash* h) {
  return h->scheme == FAST_LSH_MINHASH ? h->num_tables * h->band_rows : h->num_tables * (h->band_rows / 2);
}

static uint32_t key_bits(uint32_t dim) {
  uint32_t b = 0;
  while ((1ull << b) < dim) ++b;
  return b;
}

static int check_hash(const fast_lsh_hash* h) {
  if (!h) return fail(FAST_LSH_E_INVALID, "hash is NULL");
  if (h->dim < 2 || h->dim > 65536) return fail(FAST_LSH_E_INVALID, "dim %u outside [2, 65536]", h->dim);
  if (h->num_tables < 1 || h->num_tables > 255)
    return fail(FAST_LSH_E_INVALID, "num_tables %u outside [1, 255]", h->num_tables);
  if (h->band_rows < 1 || h->band_rows > 64)
    return fail(FAST_LSH_E_INVALID, "band_rows %u outside [1, 64]", h->band_rows);
  if (h->scheme != FAST_LSH_MINHASH && h->scheme != FAST_LSH_MINMAX)
    return fail(FAST_LSH_E_INVALID, "unknown scheme %u", h->scheme);
  if (h->scheme == FAST_LSH_MINMAX && (h->band_rows & 1))
    return fail(FAST_LSH_E_INVALID, "Min-Max needs an even band_rows (got %u)", h->band_rows);
  if (!h->a || !h->b) return fail(FAST_LSH_E_INVALID, "hash a/b is NULL");
  const uint32_t F = n_funcs(h);
  for (uint32_t f = 0; f < F; ++f) {
    if (h->a[f] < 1 || h->a[f] >= kP) return fail(FAST_LSH_E_INVALID, "a[%u] = %u outside [1, p-1]", f, h->a[f]);
    if (h->b[f] >= kP) return fail(FAST_LSH_E_INVALID, "b[%u] = %u outside [0, p-1]", f, h->b[f]);
  }
  return FAST_LSH_OK;
}

static int check_fps(const fast_lsh_fps* f) {
  if (!f) return fail(FAST_LSH_E_INVALID, "fps is NULL");
  if (f->n >= (1ull << 31)) return fail(FAST_LSH_E_INVALID, "n = %llu must be below 2^31", (unsigned long long)f->n);
  if (f->n && !f->indices) return fail(FAST_LSH_E_INVALID, "fps indices is NULL");
  if (f->n && !f->offsets && f->fixed_nnz == 0) return fail(FAST_LSH_E_INVALID, "fixed_nnz is 0");
  return FAST_LSH_OK;
}

// Upload (2a, 2b, a^-1, b) per function: 4F words.
static int upload_hash(fast_lsh_ctx* c, const fast_lsh_hash* h, uint32_t** dev) {
  const uint32_t F = n_funcs(h);
  c->hparams.assign(4 * (size_t)F, 0);
  for (uint32_t f = 0; f < F; ++f) {
    c->hparams[f] = 2u * h->a[f];
    c->hparams[F + f] = 2u * h->b[f];
    c->hparams[2 * F + f] = pow_mod(h->a[f], kP - 2);
    c->hparams[3 * F + f] = h->b[f];
  }
  RC(ws<uint32_t>(c, "hash", 4 * (uint64_t)F, dev));
  RC(h2d(c, *dev, c->hparams.data(), 4 * (uint64_t)F));
  return FAST_LSH_OK;
}

// Register capacity for the rows of fps (and the empty-row check).
static int row_capacity(fast_lsh_ctx* c, const fast_lsh_fps* f, int* cap, bool* vec) {
  uint64_t mx;
  if (f->offsets) {
    unsigned long long* rng;
    RC(ws<unsigned long long>(c, "rowlen", 2, &rng));
    fill_u64(reinterpret_cast<uint64_t*>(rng), 1, 0, c->stream);
    fill_u64(reinterpret_cast<uint64_t*>(rng) + 1, 1, ~0ull, c->stream);
    launch_row_len_range(f->offsets, f->n, rng, c->stream);
    LAUNCHCK();
    unsigned long long h[2];
    RC(d2h(c, h, rng, 2));
    if (h[1] == 0) return fail(FAST_LSH_E_INVALID, "a fingerprint has no set element");
    mx = h[0];
  } else {
    mx = f->fixed_nnz;
  }
  // Register-resident kernels need fixed, even-length, 4-byte aligned rows;
  // everything else reads its indices from memory (k_sig_long).
  const bool regular = !f->offsets && (mx % 2) == 0 && ((uintptr_t)f->indices % 4) == 0;
  *cap = regular ? sig_capacity_for(mx) : 0;
  *vec = *cap && (uint64_t)*cap == mx && ((uintptr_t)f->indices % 16) == 0;
  return FAST_LSH_OK;
}

static SigArgs sig_args(const fast_lsh_hash* h, const fast_lsh_fps* f, const uint32_t* dhash, int* err) {
  const uint32_t F = n_funcs(h);
  SigArgs a;
  memset(&a, 0, sizeof a);
  a.ind = f->indices;
  a.off = f->offsets;
  a.n = f->n;
  a.nnz = f->fixed_nnz;
  a.dim = h->dim;
  a.r = h->band_rows;
  a.fpt = h->scheme == FAST_LSH_MINHASH ? h->band_rows : h->band_rows / 2;
  a.kbits = key_bits(h->dim);
  a.packed = (uint64_t)a.kbits * h->band_rows <= 64;
  a.a2 = dhash;
  a.b2 = dhash + F;
  a.ainv = dhash + 2 * F;
  a.b = dhash + 3 * F;
  a.err = err;
  a.tables_per_group = 1;
  a.row_dw = 4;
  return a;
}

// ---------------------------------------------------------------------------
// Public API
// ---------------------------------------------------------------------------
extern "C" {

int fast_lsh_version(void) { return 10000; }

const char* fast_lsh_last_error(void) { return g_err.c_str(); }

int fast_lsh_ctx_create(int device, void* hip_stream, uint64_t hbm_budget, fast_lsh_ctx** out) {
  if (!out) return fail(FAST_LSH_E_INVALID, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIPCK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(FAST_LSH_E_INVALID, "device %d not present (%d devices)", device, ndev);
  HIPCK(hipSetDevice(device));
  fast_lsh_ctx* c = new fast_lsh_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->budget = hbm_budget;
  *out = c;
  g_err.clear();
  return FAST_LSH_OK;
}

void fast_lsh_ctx_destroy(fast_lsh_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev) (void)hipEventDestroy(e);
  for (auto& kv : c->ws)
    if (kv.second.p) (void)hipFree(kv.second.p);
  delete c;
}

int fast_lsh_make_hash(uint64_t seed, uint32_t n_funcs_, uint32_t* a, uint32_t* b) {
  if ((!a || !b) && n_funcs_) return fail(FAST_LSH_E_INVALID, "a/b is NULL");
  uint64_t s = seed;
  for (uint32_t f = 0; f < n_funcs_; ++f) {
    a[f] = (uint32_t)(1 + splitmix64(&s) % (kP - 1));
    b[f] = (uint32_t)(splitmix64(&s) % kP);
  }
  return FAST_LSH_OK;
}

int fast_lsh_signatures(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f, uint32_t table_begin,
                        uint32_t table_count, uint64_t* keys, uint32_t* sigs) {
  if (!c) return fail(FAST_LSH_E_INVALID, "ctx is NULL");
  RC(check_hash(h));
  RC(check_fps(f));
  if (table_count == 0 || table_begin + (uint64_t)table_count > h->num_tables)
    return fail(FAST_LSH_E_INVALID, "table range [%u, %u+%u) outside [0, %u)", table_begin, table_begin,
                table_count, h->num_tables);
  if (!keys && !sigs) return fail(FAST_LSH_E_INVALID, "keys and sigs are both NULL");
  if (f->n == 0) return FAST_LSH_OK;
  HIPCK(hipSetDevice(c->device));
  uint32_t* dh;
  RC(upload_hash(c, h, &dh));
  int cap;
  bool vec;
  RC(row_capacity(c, f, &cap, &vec));
  int* err;
  RC(ws<int>(c, "err", 1, &err));
  fill_u32(reinterpret_cast<uint32_t*>(err), 1, 0, c->stream);
  SigArgs a = sig_args(h, f, dh, err);
  a.table_begin = table_begin;
  a.table_count = table_count;
  a.vec_load = vec;
  a.keys = keys;
  a.sigs = sigs;
  prof_begin(c, FAST_LSH_STAGE_SIGNATURES);
  launch_sig(cap, h->scheme == FAST_LSH_MINMAX, a, c->stream);
  prof_end(c);
  LAUNCHCK();
  int herr = 0;
  RC(d2h(c, &herr, err));
  prof_collect(c);
  if (herr) return fail(FAST_LSH_E_INVALID, "a fingerprint is empty or holds an index >= dim (%u)", h->dim);
  return FAST_LSH_OK;
}

int fast_lsh_search(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f, const fast_lsh_filter* flt,
                    uint32_t* oi, uint32_t* oj, uint8_t* ov, uint64_t capacity, fast_lsh_stats* st) {
  return fast_lsh_search_ex(c, h, f, flt, 0, oi, oj, ov, capacity, st);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Search
// ---------------------------------------------------------------------------
struct Plan {
  uint32_t t, G, TG, row_dw, rsw, need;
};

// Bits of the mixed key the radix passes bin on: a multiple of 8 large enough
// that an average bin holds at most about 32 elements.
static uint32_t bin_bits(uint64_t n) {
  uint32_t need = 0;
  while ((32ull << need) < n) ++need;
  uint32_t B = (need + 7) / 8 * 8;
  return std::min<uint32_t>(32, std::max<uint32_t>(8, B));
}

static Plan make_plan(uint32_t t, uint32_t v, bool distinct) {
  Plan p;
  p.t = t;
  uint32_t G = (distinct || v <= 2) ? 1u : std::min(v - 1, t);
  p.TG = (t + G - 1) / G;
  p.G = (t + p.TG - 1) / p.TG;
  p.need = (v + p.G - 1) / p.G;
  p.row_dw = row_dwords(p.TG);
  p.rsw = p.row_dw;
  return p;
}

// Counters kept on the device during one search.  Sums taken by many
// workgroups live in kSpread slots each (see spread_slot) and are added up
// on the host.
struct DevCounters {
  unsigned long long e_raw[kSpread];
  unsigned long long e_voted[kSpread];
  unsigned long long n_distinct[kSpread];
  unsigned int max_bucket[kSpread];
  unsigned long long n_flagged;
  unsigned int big_count;
  unsigned int bin_count;
  unsigned int out_count;
  int err;
};

template <typename T>
static T spread_sum(const T* v) {
  T s = 0;
  for (uint32_t k = 0; k < kSpread; ++k) s += v[k];
  return s;
}

static int search_impl(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f, const fast_lsh_filter* flt,
                       uint32_t flags, fast_lsh_stats* out_stats) {
  const uint64_t n = f->n;
  const uint32_t t = h->num_tables;
  const bool distinct = (flags & FAST_LSH_WANT_DISTINCT) != 0;
  const Plan pl = make_plan(t, flt->min_votes, distinct);
  hipStream_t s = c->stream;
  const uint64_t tn = (uint64_t)t * n;

  uint32_t* dh;
  RC(upload_hash(c, h, &dh));
  int cap;
  bool vec;
  RC(row_capacity(c, f, &cap, &vec));

  DevCounters* dc;
  RC(ws<DevCounters>(c, "counters", 1, &dc));
  fill_u8(reinterpret_cast<uint8_t*>(dc), sizeof(DevCounters), 0, s);

  uint64_t *mkeys, *ak, *bk;
  uint32_t *av, *bv;
  uint32_t* rows;
  RC(ws<uint64_t>(c, "mkeys", tn, &mkeys));
  RC(ws<uint32_t>(c, "rows", (uint64_t)pl.G * n * pl.row_dw, &rows));
  RC(ws<uint64_t>(c, "ak", tn, &ak));
  RC(ws<uint32_t>(c, "av", tn, &av));
  RC(ws<uint64_t>(c, "bk", tn, &bk));
  RC(ws<uint32_t>(c, "bv", tn, &bv));

  // 1. signatures -> mixed keys (table-major) and sub-key rows
  SigArgs sa = sig_args(h, f, dh, &dc->err);
  sa.table_begin = 0;
  sa.table_count = t;
  sa.vec_load = vec;
  sa.mkeys = mkeys;
  sa.rows = rows;
  sa.tables_per_group = pl.TG;
  sa.row_dw = pl.row_dw;
  prof_begin(c, FAST_LSH_STAGE_SIGNATURES);
  launch_sig(cap, h->scheme == FAST_LSH_MINMAX, sa, s);
  prof_end(c);
  LAUNCHCK();

  // 2. stable radix passes on the top B bits, all tables at once
  const uint32_t nt = radix_tiles(n);
  uint32_t *hist, *sums;
  RC(ws<uint32_t>(c, "hist", (uint64_t)256 * nt * t, &hist));
  RC(ws<uint32_t>(c, "sums", scan_sums_elems((uint64_t)256 * nt, t), &sums));
  const uint32_t B = bin_bits(n);
  uint64_t *gk = ak, *gk2 = bk;
  uint32_t *gv = av, *gv2 = bv;
  prof_begin(c, FAST_LSH_STAGE_GROUP);
  for (uint32_t pass = 0; pass < B / 8; ++pass) {
    const uint32_t shift = 64 - B + 8 * pass;
    radix_pass(pass == 0 ? mkeys : gk2, pass == 0 ? nullptr : gv2, gk, gv, n, t, shift, hist, sums, s);
    LAUNCHCK();
    std::swap(gk, gk2);
    std::swap(gv, gv2);
  }
  prof_end(c);
  // the sorted keys and ids are in (gk2, gv2); the other pair is scratch
  uint64_t* sorted_k = gk2;
  uint32_t* sorted_v = gv2;
  uint64_t* scratch_k = gk;
  uint32_t* scratch_v = gv;

  // 3. buckets
  uint8_t* fl8;
  uint64_t* sbase;
  RC(ws<uint8_t>(c, "flags", n, &fl8));
  RC(ws<uint64_t>(c, "station_base", 2, &sbase));
  fill_u8(fl8, n, 0, s);
  c->hstage.assign({0ull, n});
  RC(h2d(c, sbase, c->hstage.data(), 2));

  // Pair stage: buckets of at most smax members are marked in place and
  // handled by chunks of positions; larger ones go to the tiled kernel.
  // Buckets of at most smax members are marked in place and handled by the
  // wave-per-chunk kernel; larger ones go to the tiled kernel.
  const uint32_t smax = 64;
  const uint32_t rswl = pl.rsw | 1u;
  const uint64_t cap_big = tn / (smax + 1) + 1, cap_bin = tn / 129 + t + 1;  // oversized bins and mixed bins above 128 elements
  uint4 *bdesc, *bins;
  uint8_t* marks;
  RC(ws<uint4>(c, "bdesc", cap_big, &bdesc));
  RC(ws<uint4>(c, "bins", cap_bin, &bins));
  RC(ws<uint8_t>(c, "marks", tn, &marks));
  BucketArgs ba;
  ba.keys = sorted_k;
  ba.vals = sorted_v;
  ba.n = n;
  ba.chunk = 1536;
  ba.bin_shift = 64 - B;
  ba.station_base = sbase;
  ba.nstation = 1;
  ba.occ_num = flt->occ_num;
  ba.occ_den = flt->occ_den;
  ba.min_lag = flt->min_lag;
  ba.flags = fl8;
  ba.small_max = smax;
  ba.marks = marks;
  ba.big_desc = bdesc;
  ba.big_count = &dc->big_count;
  ba.bin_desc = bins;
  ba.bin_count = &dc->bin_count;
  ba.e_raw = dc->e_raw;
  ba.max_bucket = dc->max_bucket;
  prof_begin(c, FAST_LSH_STAGE_BUCKETS);
  launch_bucket(ba, t, s);
  prof_end(c);
  LAUNCHCK();
  DevCounters hc;
  RC(d2h(c, &hc, dc));
  if (hc.err) return fail(FAST_LSH_E_INVALID, "a fingerprint is empty or holds an index >= dim (%u)", h->dim);
  if (hc.bin_count) {
    prof_begin(c, FAST_LSH_STAGE_BIG_BINS);
    launch_bigbin(ba, bins, hc.bin_count, scratch_k, scratch_v, s);
    prof_end(c);
    LAUNCHCK();
  }
  launch_count_flags(fl8, n, &dc->n_flagged, s);
  LAUNCHCK();
  RC(d2h(c, &hc, dc));

  // 4. pairs
  PairArgs pa;
  pa.order = sorted_v;
  pa.flags = fl8;
  pa.rows = rows;
  pa.mkeys = mkeys;
  pa.n = n;
  pa.t = t;
  pa.G = pl.G;
  pa.tables_per_group = pl.TG;
  pa.row_dw = pl.row_dw;
  pa.min_lag = flt->min_lag;
  pa.min_votes = flt->min_votes;
  pa.need = pl.need;
  pa.want_distinct = distinct;
  pa.out_count = &dc->out_count;
  pa.e_voted = dc->e_voted;
  pa.n_distinct = dc->n_distinct;

  uint64_t out_cap = std::max<uint64_t>(1u << 20, n / 8);
  std::vector<uint4> hbig(hc.big_count);
  if (hc.big_count) {
    HIPCK(hipMemcpyAsync(hbig.data(), bdesc, hc.big_count * sizeof(uint4), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
  }
  for (int attempt = 0; attempt < 2; ++attempt) {
    uint32_t *oi, *oj;
    uint8_t* ov;
    RC(ws<uint32_t>(c, "out_i", out_cap, &oi));
    RC(ws<uint32_t>(c, "out_j", out_cap, &oj));
    RC(ws<uint8_t>(c, "out_v", out_cap, &ov));
    pa.out_i = oi;
    pa.out_j = oj;
    pa.out_v = ov;
    pa.out_cap = (uint32_t)std::min<uint64_t>(out_cap, 0xFFFFFFFFull);
    fill_u8(reinterpret_cast<uint8_t*>(dc->e_voted), sizeof(dc->e_voted) + sizeof(dc->n_distinct), 0, s);
    fill_u32(&dc->out_count, 1, 0, s);
    prof_begin(c, FAST_LSH_STAGE_PAIRS);
    launch_pairs_wave(pa, marks, t, rswl, hc.n_flagged != 0, s);
    prof_end(c);
    LAUNCHCK();
    if (hc.big_count) {
      std::vector<uint64_t> cofs(hc.big_count + 1, 0);
      for (uint32_t b = 0; b < hc.big_count; ++b) cofs[b + 1] = cofs[b] + hbig[b].z;
      uint64_t* dcofs;
      uint32_t *bids, *bcnt;
      RC(ws<uint64_t>(c, "big_cofs", hc.big_count + 1, &dcofs));
      RC(ws<uint32_t>(c, "big_ids", cofs.back() + 1, &bids));
      RC(ws<uint32_t>(c, "big_cnt", hc.big_count, &bcnt));
      RC(h2d(c, dcofs, cofs.data(), hc.big_count + 1));
      launch_compact_big(pa, bdesc, hc.big_count, dcofs, bids, bcnt, s);
      LAUNCHCK();
      std::vector<uint32_t> hcnt(hc.big_count);
      RC(d2h(c, hcnt.data(), bcnt, hc.big_count));
      // tile edge: a power of two with two tiles of rows and ids within 64 KB of LDS
      const uint32_t fit = 65536 / (8 * rswl + 8);
      uint32_t tb = 256;
      while (tb > 16 && tb > fit) tb >>= 1;
      std::vector<TileUnit> units;
      for (uint32_t b = 0; b < hc.big_count; ++b) {
        const uint32_t m = hcnt[b];
        if (m < 2) continue;
        const uint32_t ntl = (m + tb - 1) / tb;
        for (uint32_t x = 0; x < ntl; ++x)
          for (uint32_t y = x; y < ntl; ++y) units.push_back(TileUnit{b, x, y, 0});
      }
      if (!units.empty()) {
        TileUnit* du;
        RC(ws<TileUnit>(c, "units", units.size(), &du));
        RC(h2d(c, du, units.data(), units.size()));
        for (size_t u0 = 0; u0 < units.size(); u0 += 1u << 20) {
          const uint32_t cnt = (uint32_t)std::min<size_t>(1u << 20, units.size() - u0);
          prof_begin(c, FAST_LSH_STAGE_BIG_PAIRS);
          launch_pairs_tile(pa, du + u0, cnt, bdesc, dcofs, bids, bcnt, tb, rswl, s);
          prof_end(c);
          LAUNCHCK();
        }
      }
    }
    RC(d2h(c, &hc, dc));
    if (hc.out_count <= out_cap) break;
    out_cap = (uint64_t)hc.out_count + 1024;
  }

  // 5. canonical order: sort (i << 32 | j) by LSD radix over the bits in use
  const uint64_t cnt = hc.out_count;
  uint64_t *rk0, *rk1;
  uint32_t *rv0, *rv1;
  RC(ws<uint64_t>(c, "res_k0", cnt + 1, &rk0));
  RC(ws<uint64_t>(c, "res_k1", cnt + 1, &rk1));
  RC(ws<uint32_t>(c, "res_v0", cnt + 1, &rv0));
  RC(ws<uint32_t>(c, "res_v1", cnt + 1, &rv1));
  {
    uint32_t *oi, *oj;
    uint8_t* ov;
    RC(ws<uint32_t>(c, "out_i", out_cap, &oi));
    RC(ws<uint32_t>(c, "out_j", out_cap, &oj));
    RC(ws<uint8_t>(c, "out_v", out_cap, &ov));
    launch_pack_out(oi, oj, ov, cnt, rk0, rv0, s);
    LAUNCHCK();
  }
  if (cnt > 1) {
    const uint32_t nb = key_bits((uint32_t)std::max<uint64_t>(n, 2));
    const uint32_t ont = radix_tiles(cnt);
    uint32_t *ohist, *osums;
    RC(ws<uint32_t>(c, "ohist", (uint64_t)256 * ont, &ohist));
    RC(ws<uint32_t>(c, "osums", scan_sums_elems((uint64_t)256 * ont, 1), &osums));
    std::vector<uint32_t> shifts;
    for (uint32_t sh = 0; sh < nb; sh += 8) shifts.push_back(sh);
    for (uint32_t sh = 0; sh < nb; sh += 8) shifts.push_back(32 + sh);
    for (uint32_t sh : shifts) {
      prof_begin(c, FAST_LSH_STAGE_OUTPUT);
      radix_pass(rk0, rv0, rk1, rv1, cnt, 1, sh, ohist, osums, s);
      prof_end(c);
      LAUNCHCK();
      std::swap(rk0, rk1);
      std::swap(rv0, rv1);
    }
  }
  // The sorted result lives in "res_k0"/"res_v0" or "res_k1"/"res_v1"; remember which.
  c->res_count = cnt;
  c->res_valid = true;
  {
    // Keep the result under fixed names for fast_lsh_copy_result.
    Buf& k0 = c->ws["res_k0"];
    Buf& v0 = c->ws["res_v0"];
    if (k0.p != rk0) {
      std::swap(c->ws["res_k0"], c->ws["res_k1"]);
      std::swap(c->ws["res_v0"], c->ws["res_v1"]);
    }
    (void)v0;
  }

  HIPCK(hipStreamSynchronize(s));
  prof_collect(c);
  fast_lsh_stats stv;
  stv.n_out = cnt;
  stv.e_raw = spread_sum(hc.e_raw);
  stv.e_voted = spread_sum(hc.e_voted);
  stv.n_distinct = distinct ? spread_sum(hc.n_distinct) : ~0ull;
  stv.n_flagged = hc.n_flagged;
  stv.max_bucket = *std::max_element(hc.max_bucket, hc.max_bucket + kSpread);
  *out_stats = stv;
  return FAST_LSH_OK;
}

extern "C" {

int fast_lsh_profile_enable(fast_lsh_ctx* c, int enable) {
  if (!c) return fail(FAST_LSH_E_INVALID, "ctx is NULL");
  c->prof = enable != 0;
  c->nrec = 0;
  for (int k = 0; k < FAST_LSH_PROFILE_STAGES; ++k) {
    c->prof_ms[k] = 0;
    c->prof_launches[k] = 0;
  }
  return FAST_LSH_OK;
}

int fast_lsh_profile_read(fast_lsh_ctx* c, fast_lsh_profile* out) {
  if (!c || !out) return fail(FAST_LSH_E_INVALID, "ctx or out is NULL");
  for (int k = 0; k < FAST_LSH_PROFILE_STAGES; ++k) {
    out->ms[k] = c->prof_ms[k];
    out->launches[k] = c->prof_launches[k];
  }
  return FAST_LSH_OK;
}

int fast_lsh_copy_result(fast_lsh_ctx* c, uint32_t* oi, uint32_t* oj, uint8_t* ov, uint64_t capacity) {
  if (!c) return fail(FAST_LSH_E_INVALID, "ctx is NULL");
  if (!c->res_valid) return fail(FAST_LSH_E_INVALID, "no search result in this context");
  if (c->res_count > capacity)
    return fail(FAST_LSH_E_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)c->res_count,
                (unsigned long long)capacity);
  if (c->res_count == 0) return FAST_LSH_OK;
  if (!oi || !oj || !ov) return fail(FAST_LSH_E_INVALID, "output pointer is NULL");
  HIPCK(hipSetDevice(c->device));
  launch_split_out(static_cast<uint64_t*>(c->ws["res_k0"].p), static_cast<uint32_t*>(c->ws["res_v0"].p),
                   c->res_count, oi, oj, ov, c->stream);
  LAUNCHCK();
  HIPCK(hipStreamSynchronize(c->stream));
  return FAST_LSH_OK;
}

int fast_lsh_search_ex(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f, const fast_lsh_filter* flt,
                       uint32_t flags, uint32_t* oi, uint32_t* oj, uint8_t* ov, uint64_t capacity,
                       fast_lsh_stats* st) {
  if (!c) return fail(FAST_LSH_E_INVALID, "ctx is NULL");
  RC(check_hash(h));
  RC(check_fps(f));
  if (!flt) return fail(FAST_LSH_E_INVALID, "filter is NULL");
  if (flt->min_votes < 1) return fail(FAST_LSH_E_INVALID, "min_votes must be >= 1");
  if (flt->occ_den && flt->occ_num > flt->occ_den)
    return fail(FAST_LSH_E_INVALID, "occurrence filter fraction %u/%u above 1", flt->occ_num, flt->occ_den);
  if (flags & ~(uint32_t)FAST_LSH_WANT_DISTINCT) return fail(FAST_LSH_E_INVALID, "unknown flags 0x%x", flags);
  HIPCK(hipSetDevice(c->device));
  c->res_valid = false;
  fast_lsh_stats local;
  if (f->n == 0) {
    memset(&local, 0, sizeof local);
    c->res_count = 0;
    c->res_valid = true;
  } else {
    RC(search_impl(c, h, f, flt, flags, &local));
  }
  if (st) *st = local;
  if (local.n_out > capacity)
    return fail(FAST_LSH_E_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)local.n_out,
                (unsigned long long)capacity);
  return fast_lsh_copy_result(c, oi, oj, ov, capacity);
}

}  // extern "C"
