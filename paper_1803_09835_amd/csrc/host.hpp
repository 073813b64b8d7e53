// Host-side pieces shared by the C-ABI sources: the context, its workspace,
// error reporting, stage timing and the kernel launchers.
#pragma once

#include <stdint.h>

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
constexpr uint32_t kRadixTileVariants = 3;               // 16384, 8192, 4096 elements
uint32_t radix_tile_elems(uint32_t variant);
uint32_t radix_tiles(uint64_t n, uint32_t variant);
uint64_t scan_sums_elems(uint64_t len, uint32_t S);
void scan_u64(uint64_t* data, uint64_t len, uint32_t S, uint64_t* sums, uint64_t* seg_total, hipStream_t s);
void radix_pass(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, uint64_t n, uint32_t S,
                uint32_t shift, uint32_t* hist, uint32_t* sums, uint32_t variant, hipStream_t s);
void launch_bucket(const BucketArgs& a, uint32_t S, hipStream_t s);
void launch_split_keys(const uint32_t* hi32, const uint32_t* rows, uint64_t n, uint32_t tb, uint32_t tc,
                       uint32_t tables_per_group, uint32_t row_pitch, uint64_t* mkeys, hipStream_t s);
uint64_t bucket_desc_slack(uint64_t big_max, uint32_t S);  // extra big-descriptor slots launch_bucket may use
uint32_t device_cus();  // compute units of the current device
void launch_bigbin(const BucketArgs& a, const uint4* bins, uint32_t grid, uint64_t* tk, uint32_t* tv,
                   hipStream_t s);
// pairs.hip
// Largest bucket the wave kernel takes for a pair form (kSmallBucket or kSmallBucketGeneral).
uint32_t pair_small_max(uint32_t need, bool distinct, uint32_t parts, uint32_t row_dw);
void launch_pairs_wave(const PairArgs& a, const uint8_t* marks, uint32_t S, uint32_t rswl, uint32_t small_max,
                       hipStream_t s);
// Whether a pair launch with these arguments queues its candidates, and the
// launch that checks (and empties) the queue after it.
bool pair_launch_queues(const PairArgs& a);
void launch_check_queue(const PairArgs& a, hipStream_t s);
void launch_tile_counts(const uint4* big, uint32_t nbig, uint32_t tb, uint64_t* tiles, unsigned long long* work,
                        hipStream_t s);
void launch_work_reduce(const unsigned long long* work, unsigned long long* out, hipStream_t s);
void launch_part_flag(const uint8_t* ex, const uint32_t* cand, uint64_t lo, uint64_t hi, uint32_t num, uint32_t den,
                      uint8_t* fp, unsigned int* nfp, hipStream_t s);
void launch_part_merge(uint8_t* ex, uint8_t* fp, uint8_t* ex_next, uint64_t n, hipStream_t s);
void launch_unit_owner(const uint64_t* toff, uint32_t nbig, uint32_t* owner, hipStream_t s);
void launch_pairs_tile(const PairArgs& a, const uint64_t* toff, const uint32_t* owner, uint64_t unit_base, uint32_t nunits,
                       const uint4* big, uint32_t tb_size, uint32_t rswl, hipStream_t s);
void launch_split_out(const uint64_t* key, const uint32_t* val, uint64_t count, uint32_t* oi, uint32_t* oj,
                      uint8_t* ov, const uint64_t* base, uint32_t nb, hipStream_t s);
void launch_station_offsets(const uint64_t* key, uint64_t count, const uint64_t* base, uint32_t nb,
                            unsigned long long* offs, hipStream_t s);
void launch_pack_out(const uint32_t* oi, const uint32_t* oj, const uint8_t* ov, uint64_t count, uint64_t* key,
                     uint32_t* val, hipStream_t s);
void launch_count_flags(const uint8_t* flags, uint64_t n, unsigned long long* out, unsigned long long* total,
                        hipStream_t s);
void launch_spread_reduce(const unsigned long long* e_raw, const unsigned int* max_bucket,
                          const unsigned long long* e_voted, const unsigned long long* n_distinct, uint32_t S,
                          unsigned long long* out, hipStream_t s);
void fill_u8(uint8_t* p, uint64_t count, uint8_t v, hipStream_t s);
void fill_u32(uint32_t* p, uint64_t count, uint32_t v, hipStream_t s);
void fill_u64(uint64_t* p, uint64_t count, uint64_t v, hipStream_t s);
}  // namespace fl

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
int fl_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIPCK(expr)                                                                                 \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return fl_fail(FAST_LSH_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCK()                                                                                        \
  do {                                                                                                    \
    hipError_t e_ = hipGetLastError();                                                                    \
    if (e_ != hipSuccess) return fl_fail(FAST_LSH_E_DEVICE, "kernel launch (%s:%d): %s", __FILE__, __LINE__, \
                                         hipGetErrorString(e_));                                          \
  } while (0)

#define RC(expr)                        \
  do {                                  \
    int rc_ = (expr);                   \
    if (rc_ != FAST_LSH_OK) return rc_; \
  } while (0)

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

// Launch shapes that change speed, never results.
struct TuneChoice {
  uint32_t radix_variant = 0;  // index into the radix tile shapes
  uint32_t bucket_chunk = 512;
};

struct fast_lsh_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;  // private stream that graph capture records on
  uint64_t budget = 0;
  std::map<std::string, Buf> ws;
  uint64_t ws_total = 0;
  uint64_t ws_generation = 0;  // bumped on every (re)allocation: invalidates captured graphs
  std::vector<uint32_t> hparams;  // host staging for hash parameters
  std::vector<uint64_t> hstage;   // host staging for small uploads
  // last search result (kept for fast_lsh_copy_result)
  uint64_t res_count = 0;
  uint32_t res_stations = 0;
  bool res_valid = false;
  fast_lsh_work last_work = {0, 0, 0, 0};  // work counters of the last search
  // launch-shape tuning
  fast_lsh_config config;
  std::map<std::vector<uint64_t>, TuneChoice> tuned;  // shape key -> choice
  TuneChoice last_choice;
  uint32_t last_bin_bits = 0;  // bin bits of the last search
  uint32_t last_kept = 0;      // table groups the last bounded search kept for its pass 2
  uint32_t last_qcap = 0;      // candidate queue entries per slot of the last search (FAST_LSH_QUEUE_OFF: none)
  uint64_t pair_redos = 0;     // second pair runs of the current search
  // captured search prefix
  hipGraphExec_t graph = nullptr;
  std::vector<uint64_t> graph_key;
  uint64_t graph_replays = 0;
  // stage timing (HIP events on the context stream around each launch; the
  // event pool grows with the launches of one call)
  bool prof = false;
  std::vector<hipEvent_t> ev;  // two per recorded interval
  std::vector<int> rec_stage;
  int nrec = 0;
  bool rec_open = false;   // an interval's start is recorded, its end not yet
  bool prof_lost = false;  // an event could not be created: some launches went untimed
  double prof_ms[FAST_LSH_PROFILE_STAGES] = {0};
  uint64_t prof_launches[FAST_LSH_PROFILE_STAGES] = {0};
};

void prof_begin(fast_lsh_ctx* c, int stage);
void prof_end(fast_lsh_ctx* c);
void prof_collect(fast_lsh_ctx* c);

int ws_get(fast_lsh_ctx* c, const char* name, size_t bytes, void** out);

template <typename T>
static inline int ws(fast_lsh_ctx* c, const char* name, uint64_t count, T** out) {
  void* p = nullptr;
  RC(ws_get(c, name, count * sizeof(T), &p));
  *out = static_cast<T*>(p);
  return FAST_LSH_OK;
}

template <typename T>
static inline int d2h(fast_lsh_ctx* c, T* host, const T* dev, uint64_t count = 1) {
  HIPCK(hipMemcpyAsync(host, dev, count * sizeof(T), hipMemcpyDeviceToHost, c->stream));
  HIPCK(hipStreamSynchronize(c->stream));
  return FAST_LSH_OK;
}

template <typename T>
static inline int h2d(fast_lsh_ctx* c, T* dev, const T* host, uint64_t count) {
  if (count == 0) return FAST_LSH_OK;
  HIPCK(hipMemcpyAsync(dev, host, count * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HIPCK(hipStreamSynchronize(c->stream));
  return FAST_LSH_OK;
}

// Hash parameters and fingerprints
uint32_t fl_n_funcs(const fast_lsh_hash* h);
uint32_t fl_key_bits(uint32_t dim);
int fl_check_hash(const fast_lsh_hash* h);
int fl_check_fps(const fast_lsh_fps* f);
int fl_upload_hash(fast_lsh_ctx* c, const fast_lsh_hash* h, uint32_t** dev);
int fl_row_capacity(fast_lsh_ctx* c, const fast_lsh_fps* f, int* cap, bool* vec);
fl::SigArgs fl_sig_args(const fast_lsh_hash* h, const fast_lsh_fps* f, const uint32_t* dhash, int* err);

// Search over a set of stations (search.hip)
int fl_search_stations(fast_lsh_ctx* c, const fast_lsh_hash* h, uint32_t S, const fast_lsh_fps* f,
                       const fast_lsh_filter* flt, uint32_t flags, fast_lsh_stats* per_station,
                       uint64_t* station_offsets, uint32_t parts = 0);
// Device address of the allocation-free calls' scratch array, taken once per
// device (align.hip).
int fl_scratch_init(int device);
int fl_search_bounded(fast_lsh_ctx* c, const fast_lsh_hash* h, const fast_lsh_fps* f, const fast_lsh_filter* flt,
                      uint32_t flags, uint32_t group_tables, fast_lsh_stats* stats);
