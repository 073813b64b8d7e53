// C-ABI entry points and host orchestration of the fast_lsh library.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "host.hpp"

using namespace fl;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

int fl_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// ---------------------------------------------------------------------------
// Context and workspace
// ---------------------------------------------------------------------------
void prof_begin(fast_lsh_ctx* c, int stage) {
  if (!c->prof) return;
  if ((size_t)c->nrec >= c->rec_stage.size()) {
    // grow the pool by 256 intervals; when an event cannot be created the
    // launch goes untimed and fast_lsh_profile_read reports E_DEVICE
    const size_t old = c->ev.size();
    c->ev.resize(old + 512, nullptr);
    for (size_t k = old; k < c->ev.size(); ++k)
      if (hipEventCreate(&c->ev[k]) != hipSuccess) {
        (void)hipGetLastError();
        c->ev.resize(k & ~(size_t)1);
        c->prof_lost = true;
        return;
      }
    c->rec_stage.resize(c->ev.size() / 2);
  }
  c->rec_stage[c->nrec] = stage;
  (void)hipEventRecord(c->ev[2 * c->nrec], c->stream);
  c->rec_open = true;
}

void prof_end(fast_lsh_ctx* c) {
  if (!c->prof || !c->rec_open) return;
  (void)hipEventRecord(c->ev[2 * c->nrec + 1], c->stream);
  ++c->nrec;
  c->rec_open = false;
}

// Accumulate recorded intervals (the caller has synchronised the stream).
void prof_collect(fast_lsh_ctx* c) {
  for (int k = 0; k < c->nrec; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]) == hipSuccess) {
      c->prof_ms[c->rec_stage[k]] += ms;
      c->prof_launches[c->rec_stage[k]] += 1;
    }
  }
  c->nrec = 0;
}

int ws_get(fast_lsh_ctx* c, const char* name, size_t bytes, void** out) {
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
    return fl_fail(FAST_LSH_E_NOMEM, "workspace '%s' (%zu bytes) exceeds the HBM budget (%llu in use of %llu)", name,
                want, (unsigned long long)c->ws_total, (unsigned long long)c->budget);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fl_fail(FAST_LSH_E_NOMEM, "hipMalloc of workspace '%s' (%zu bytes) failed", name, want);
  }
  b.cap = want;
  c->ws_total += want;
  ++c->ws_generation;
  *out = b.p;
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

uint32_t fl_n_funcs(const fast_lsh_hash* h) {
  return h->scheme == FAST_LSH_MINHASH ? h->num_tables * h->band_rows : h->num_tables * (h->band_rows / 2);
}

uint32_t fl_key_bits(uint32_t dim) {
  uint32_t b = 0;
  while ((1ull << b) < dim) ++b;
  return b;
}

int fl_check_hash(const fast_lsh_hash* h) {
  if (!h) return fl_fail(FAST_LSH_E_INVALID, "hash is NULL");
  if (h->dim < 2 || h->dim > 65536) return fl_fail(FAST_LSH_E_INVALID, "dim %u outside [2, 65536]", h->dim);
  if (h->num_tables < 1 || h->num_tables > 255)
    return fl_fail(FAST_LSH_E_INVALID, "num_tables %u outside [1, 255]", h->num_tables);
  if (h->band_rows < 1 || h->band_rows > 64)
    return fl_fail(FAST_LSH_E_INVALID, "band_rows %u outside [1, 64]", h->band_rows);
  if (h->scheme != FAST_LSH_MINHASH && h->scheme != FAST_LSH_MINMAX)
    return fl_fail(FAST_LSH_E_INVALID, "unknown scheme %u", h->scheme);
  if (h->scheme == FAST_LSH_MINMAX && (h->band_rows & 1))
    return fl_fail(FAST_LSH_E_INVALID, "Min-Max needs an even band_rows (got %u)", h->band_rows);
  if (!h->a || !h->b) return fl_fail(FAST_LSH_E_INVALID, "hash a/b is NULL");
  const uint32_t F = fl_n_funcs(h);
  for (uint32_t f = 0; f < F; ++f) {
    if (h->a[f] < 1 || h->a[f] >= kP) return fl_fail(FAST_LSH_E_INVALID, "a[%u] = %u outside [1, p-1]", f, h->a[f]);
    if (h->b[f] >= kP) return fl_fail(FAST_LSH_E_INVALID, "b[%u] = %u outside [0, p-1]", f, h->b[f]);
  }
  return FAST_LSH_OK;
}

int fl_check_fps(const fast_lsh_fps* f) {
  if (!f) return fl_fail(FAST_LSH_E_INVALID, "fps is NULL");
  if (f->n >= (1ull << 31)) return fl_fail(FAST_LSH_E_INVALID, "n = %llu must be below 2^31", (unsigned long long)f->n);
  if (f->n && !f->indices) return fl_fail(FAST_LSH_E_INVALID, "fps indices is NULL");
  if (f->n && !f->offsets && f->fixed_nnz == 0) return fl_fail(FAST_LSH_E_INVALID, "fixed_nnz is 0");
  return FAST_LSH_OK;
}

// Upload (2a, 2b, a^-1, b) per function: 4F words.
int fl_upload_hash(fast_lsh_ctx* c, const fast_lsh_hash* h, uint32_t** dev) {
  const uint32_t F = fl_n_funcs(h);
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
int fl_row_capacity(fast_lsh_ctx* c, const fast_lsh_fps* f, int* cap, bool* vec) {
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
    if (h[1] == 0) return fl_fail(FAST_LSH_E_INVALID, "a fingerprint has no set element");
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

SigArgs fl_sig_args(const fast_lsh_hash* h, const fast_lsh_fps* f, const uint32_t* dhash, int* err) {
  const uint32_t F = fl_n_funcs(h);
  SigArgs a;
  memset(&a, 0, sizeof a);
  a.ind = f->indices;
  a.off = f->offsets;
  a.n = f->n;
  a.nnz = f->fixed_nnz;
  a.dim = h->dim;
  a.r = h->band_rows;
  a.fpt = h->scheme == FAST_LSH_MINHASH ? h->band_rows : h->band_rows / 2;
  a.kbits = fl_key_bits(h->dim);
  a.packed = (uint64_t)a.kbits * h->band_rows <= 64;
  a.a2 = dhash;
  a.b2 = dhash + F;
  a.ainv = dhash + 2 * F;
  a.b = dhash + 3 * F;
  a.err = err;
  a.tables_per_group = 1;
  a.row_dw = 4;
  a.row_pitch = 4;
  a.out_stride = f->n;
  return a;
}

// ---------------------------------------------------------------------------
// Public API
// ---------------------------------------------------------------------------
extern "C" {

int fast_lsh_version(void) { return 10000; }

const char* fast_lsh_last_error(void) { return g_err.c_str(); }

int fast_lsh_ctx_create(int device, void* hip_stream, uint64_t hbm_budget, fast_lsh_ctx** out) {
  if (!out) return fl_fail(FAST_LSH_E_INVALID, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIPCK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fl_fail(FAST_LSH_E_INVALID, "device %d not present (%d devices)", device, ndev);
  HIPCK(hipSetDevice(device));
  RC(fl_scratch_init(device));
  fast_lsh_ctx* c = new fast_lsh_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->budget = hbm_budget;
  c->config.radix_tile = radix_tile_elems(0);
  c->config.bucket_chunk = 512;
  c->config.autotune = 0;
  c->config.bin_bits = 0;
  c->config.keep_groups = FAST_LSH_KEEP_AUTO;
  c->config.queue_slot = 0;
  *out = c;
  g_err.clear();
  return FAST_LSH_OK;
}

void fast_lsh_ctx_destroy(fast_lsh_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev) (void)hipEventDestroy(e);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  for (auto& kv : c->ws)
    if (kv.second.p) (void)hipFree(kv.second.p);
  delete c;
}

int fast_lsh_make_hash(uint64_t seed, uint32_t n_funcs_, uint32_t* a, uint32_t* b) {
  if ((!a || !b) && n_funcs_) return fl_fail(FAST_LSH_E_INVALID, "a/b is NULL");
  uint64_t s = seed;
  for (uint32_t f = 0; f < n_funcs_; ++f) {
    a[f] = (uint32_t)(1 + splitmix64(&s) % (kP - 1));
    b[f] = (uint32_t)(splitmix64(&s) % kP);
  }
  return FAST_LSH_OK;
}

int fast_lsh_signatures(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f, uint32_t table_begin,
                        uint32_t table_count, uint64_t* keys, uint32_t* sigs) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  RC(fl_check_hash(h));
  RC(fl_check_fps(f));
  if (table_count == 0 || table_begin + (uint64_t)table_count > h->num_tables)
    return fl_fail(FAST_LSH_E_INVALID, "table range [%u, %u+%u) outside [0, %u)", table_begin, table_begin,
                   table_count, h->num_tables);
  if (!keys && !sigs) return fl_fail(FAST_LSH_E_INVALID, "keys and sigs are both NULL");
  if (f->n == 0) return FAST_LSH_OK;
  HIPCK(hipSetDevice(c->device));
  uint32_t* dh;
  RC(fl_upload_hash(c, h, &dh));
  int cap;
  bool vec;
  RC(fl_row_capacity(c, f, &cap, &vec));
  int* err;
  RC(ws<int>(c, "err", 1, &err));
  fill_u32(reinterpret_cast<uint32_t*>(err), 1, 0, c->stream);
  SigArgs a = fl_sig_args(h, f, dh, err);
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
  if (herr) return fl_fail(FAST_LSH_E_INVALID, "a fingerprint is empty or holds an index >= dim (%u)", h->dim);
  return FAST_LSH_OK;
}

int fast_lsh_workspace_bytes(fast_lsh_ctx* c, uint64_t* bytes) {
  if (!c || !bytes) return fl_fail(FAST_LSH_E_INVALID, "ctx or bytes is NULL");
  *bytes = c->ws_total;
  return FAST_LSH_OK;
}

int fast_lsh_profile_enable(fast_lsh_ctx* c, int enable) {
  if (!c) return fl_fail(FAST_LSH_E_INVALID, "ctx is NULL");
  c->prof = enable != 0;
  c->nrec = 0;
  c->rec_open = false;
  c->prof_lost = false;
  for (int k = 0; k < FAST_LSH_PROFILE_STAGES; ++k) {
    c->prof_ms[k] = 0;
    c->prof_launches[k] = 0;
  }
  return FAST_LSH_OK;
}

int fast_lsh_profile_read(fast_lsh_ctx* c, fast_lsh_profile* out) {
  if (!c || !out) return fl_fail(FAST_LSH_E_INVALID, "ctx or out is NULL");
  if (c->prof_lost) return fl_fail(FAST_LSH_E_DEVICE, "stage timing lost launches: a HIP event could not be created");
  for (int k = 0; k < FAST_LSH_PROFILE_STAGES; ++k) {
    out->ms[k] = c->prof_ms[k];
    out->launches[k] = c->prof_launches[k];
  }
  return FAST_LSH_OK;
}

int fast_lsh_last_work(fast_lsh_ctx* c, fast_lsh_work* out) {
  if (!c || !out) return fl_fail(FAST_LSH_E_INVALID, "ctx or out is NULL");
  *out = c->last_work;
  return FAST_LSH_OK;
}

int fast_lsh_configure(fast_lsh_ctx* c, const fast_lsh_config* cfg) {
  if (!c || !cfg) return fl_fail(FAST_LSH_E_INVALID, "ctx or config is NULL");
  uint32_t tile = cfg->radix_tile ? cfg->radix_tile : c->config.radix_tile;
  bool known = false;
  for (uint32_t v = 0; v < kRadixTileVariants; ++v) known |= radix_tile_elems(v) == tile;
  if (!known) return fl_fail(FAST_LSH_E_INVALID, "radix_tile %u is not 16384, 8192 or 4096", cfg->radix_tile);
  const uint32_t chunk = cfg->bucket_chunk ? cfg->bucket_chunk : c->config.bucket_chunk;
  if (chunk < 256 || chunk > 1536 || chunk % 256)
    return fl_fail(FAST_LSH_E_INVALID, "bucket_chunk %u is not a multiple of 256 in [256, 1536]", cfg->bucket_chunk);
  if (cfg->autotune > 1) return fl_fail(FAST_LSH_E_INVALID, "autotune must be 0 or 1");
  if (cfg->bin_bits % 8 || cfg->bin_bits > 32)
    return fl_fail(FAST_LSH_E_INVALID, "bin_bits %u is not 0, 8, 16, 24 or 32", cfg->bin_bits);
  if (cfg->queue_slot != FAST_LSH_QUEUE_OFF && cfg->queue_slot > (1u << 20))
    return fl_fail(FAST_LSH_E_INVALID, "queue_slot %u is above 2^20", cfg->queue_slot);
  c->config.radix_tile = tile;
  c->config.bucket_chunk = chunk;
  c->config.autotune = cfg->autotune;
  c->config.bin_bits = cfg->bin_bits;
  c->config.keep_groups = cfg->keep_groups;
  c->config.queue_slot = cfg->queue_slot;
  return FAST_LSH_OK;
}

int fast_lsh_config_used(fast_lsh_ctx* c, fast_lsh_config* out) {
  if (!c || !out) return fl_fail(FAST_LSH_E_INVALID, "ctx or out is NULL");
  out->radix_tile = radix_tile_elems(c->last_choice.radix_variant);
  out->bucket_chunk = c->last_choice.bucket_chunk;
  out->autotune = c->config.autotune;
  out->bin_bits = c->last_bin_bits;
  out->keep_groups = c->last_kept;
  out->queue_slot = c->last_qcap;
  return FAST_LSH_OK;
}

}  // extern "C"
