/*
 * fast_lsh — MinHash / Min-Max LSH similarity search for binary waveform
 * fingerprints on AMD Instinct MI355X (gfx950).
 *
 * The method is the similarity-search stage of the FAST earthquake-detection
 * pipeline as scaled by Rong et al., "Locality-Sensitive Hashing for
 * Earthquake Detection: A Case Study of Scaling Data-Driven Science",
 * VLDB 2018:
 *   - every fingerprint (a sparse binary vector, given as the sorted list of
 *     its non-zero element indices) gets one band key per hash table, made
 *     of r MinHash (section 6.1) or Min-Max (section 6.2) values;
 *   - fingerprints with equal band keys share that table's bucket
 *     (section 6.1 "Hash table construction");
 *   - a pair's vote count is the number of tables in which the two share a
 *     bucket; pairs with at least `min_votes` votes are reported, the count
 *     standing in for similarity (section 6.1 "Search", section 6.3 S-curve,
 *     section 7.2 triplets);
 *   - pairs closer than `min_lag` fingerprints are self-matches and dropped
 *     (section 7.1);
 *   - the occurrence filter excludes every fingerprint that lands in an
 *     over-full bucket (section 6.5).
 *
 * Definitions fixed by this library where the paper leaves them open:
 *   - hash function f: h_f(x) = (a_f * x + b_f) mod (2^31 - 1), x the 0-based
 *     element index, a_f in [1, 2^31 - 2], b_f in [0, 2^31 - 2];
 *   - MinHash: table u, row s uses function u*r + s (F = t*r functions).
 *     Min-Max: table u uses functions u*r/2 + q; row 2q is the minimum and
 *     row 2q+1 the maximum of that function (F = t*r/2; r must be even);
 *   - band key: the r element indices attaining the r values, each in
 *     b = ceil(log2 dim) bits, row s at bit b*s (lossless when b*r <= 64,
 *     so equal keys means equal values).  For b*r > 64 the key is the chain
 *     k_0 = 0, k_{s+1} = fmix64(k_s + x_s + 1) (murmur3's 64-bit finaliser);
 *   - occurrence filter: fingerprint i is excluded when, in some table, its
 *     bucket holds more than occ_num/occ_den of the n fingerprints
 *     (size * occ_den > n * occ_num, sizes counted before exclusion); an
 *     excluded fingerprint is part of no pair in any table;
 *   - output: pairs (i, j) with i < j, j - i >= min_lag, neither excluded,
 *     votes >= min_votes, sorted by (i, j).  The paper's triplet
 *     (dt, idx1, sim) is (j - i, i, votes).
 *
 * Conventions for every entry point:
 *   - Bulk arrays (fingerprint indices, offsets, keys, outputs) are DEVICE
 *     pointers on the context's device; small parameter arrays (hash a/b,
 *     stats) are HOST pointers.  The caller owns all of them.  The library
 *     owns only its context workspace.
 *   - Work is ordered on the context's HIP stream.  Calls that return counts
 *     (search) synchronise that stream before returning.
 *   - Return value: FAST_LSH_OK or an error code; fast_lsh_last_error()
 *     gives a message for the calling thread.  On error no output buffer is
 *     guaranteed to hold anything meaningful.
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef FAST_LSH_H
#define FAST_LSH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FAST_LSH_OK = 0,
  FAST_LSH_E_INVALID = 1,  /* bad argument or bad fingerprint data            */
  FAST_LSH_E_NOMEM = 2,    /* workspace would exceed the context's HBM budget */
  FAST_LSH_E_CAPACITY = 3, /* more output pairs than the caller's capacity    */
  FAST_LSH_E_DEVICE = 4,   /* a HIP runtime call failed                       */
  FAST_LSH_E_BUSY = 5      /* asynchronous work not finished yet              */
};

enum { FAST_LSH_MINHASH = 0, FAST_LSH_MINMAX = 1 };

typedef struct fast_lsh_ctx fast_lsh_ctx;

/* Hash family for t tables of r rows (section 6.1, section 6.3 parameters
 * k = r, t; section 6.2 Min-Max).  a and b are HOST arrays of F entries. */
typedef struct {
  uint32_t dim;        /* d: fingerprint dimension, 2..65536                 */
  uint32_t num_tables; /* t: 1..255                                          */
  uint32_t band_rows;  /* r: values per band key, 1..64 (even for Min-Max)  */
  uint32_t scheme;     /* FAST_LSH_MINHASH or FAST_LSH_MINMAX                */
  const uint32_t *a;   /* host, F entries, each in [1, 2^31 - 2]             */
  const uint32_t *b;   /* host, F entries, each in [0, 2^31 - 2]             */
} fast_lsh_hash;

/* n fingerprints as index lists.  offsets == NULL: row i is
 * indices[i*fixed_nnz .. (i+1)*fixed_nnz).  Otherwise row i is
 * indices[offsets[i] .. offsets[i+1]) (offsets has n+1 entries).  Every row
 * must be non-empty and every index < dim; the order of indices within a row
 * does not matter. */
typedef struct {
  const uint16_t *indices; /* device */
  const uint64_t *offsets; /* device, n+1 entries, or NULL                   */
  uint32_t fixed_nnz;      /* row length when offsets == NULL                */
  uint32_t reserved;
  uint64_t n;              /* number of fingerprints, < 2^31                 */
} fast_lsh_fps;

/* Search filters: self-match lag (section 7.1), vote threshold (section 6.1,
 * "at least m of t" in section 6.3), occurrence filter (section 6.5;
 * occ_den == 0 switches it off). */
typedef struct {
  uint32_t min_lag;   /* L: keep pairs with j - i >= L                       */
  uint32_t min_votes; /* v >= 1                                              */
  uint32_t occ_num;
  uint32_t occ_den;
} fast_lsh_filter;

/* Counters of one search (all exact):
 *   n_out       pairs reported (votes >= v);
 *   e_raw       sum over tables and buckets of C(size, 2), before any filter
 *               (the candidate comparisons a plain LSH query loop performs);
 *   e_voted     sum of votes over all pairs that pass lag and exclusion;
 *   n_distinct  number of such pairs with at least one vote (computed only
 *               when the search is asked for it, else UINT64_MAX);
 *   n_flagged   fingerprints excluded by the occurrence filter;
 *   max_bucket  largest bucket over all tables, before any filter. */
typedef struct {
  uint64_t n_out, e_raw, e_voted, n_distinct, n_flagged, max_bucket;
} fast_lsh_stats;

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int fast_lsh_version(void);

/* Message describing the last error on the calling thread ("" if none). */
const char *fast_lsh_last_error(void);

/* Create a context on HIP device `device`, ordering work on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  `hbm_budget` bounds the
 * workspace the context may allocate, in bytes (0 = no bound beyond the
 * device's free memory).  *out receives the context. */
int fast_lsh_ctx_create(int device, void *hip_stream, uint64_t hbm_budget, fast_lsh_ctx **out);

/* Release the context and its workspace (NULL is ignored). */
void fast_lsh_ctx_destroy(fast_lsh_ctx *ctx);

/* Hash mappings from a seed (the role of single_hash in Appendix D,
 * Algorithm 1): splitmix64 seeded with `seed` (Steele, Lea & Flood 2014);
 * for f = 0..n_funcs-1 in order: a[f] = 1 + next() mod (2^31 - 2),
 * b[f] = next() mod (2^31 - 1).  a and b are HOST arrays of n_funcs entries.
 * Host-only; needs no context. */
int fast_lsh_make_hash(uint64_t seed, uint32_t n_funcs, uint32_t *a, uint32_t *b);

/* Signatures (section 6.1; section 6.2; Appendix D, Algorithm 1
 * minmax_batch) for tables [table_begin, table_begin + table_count).
 *   keys  device, uint64[table_count][n]: keys[u][i] is the band key of
 *         fingerprint i in table table_begin + u;
 *   sigs  device, uint32[n][table_count][r] or NULL: the r hash values of
 *         each band key in row order (min / max for Min-Max).
 * E_INVALID for bad parameters, an empty row or an index >= dim. */
int fast_lsh_signatures(fast_lsh_ctx *ctx, const fast_lsh_hash *hash, const fast_lsh_fps *fps,
                        uint32_t table_begin, uint32_t table_count, uint64_t *keys, uint32_t *sigs);

/* Flags for fast_lsh_search_ex and fast_lsh_search_batched.
 *   FAST_LSH_WANT_DISTINCT  also compute stats n_distinct (costs a full
 *                           comparison of every candidate pair);
 *   FAST_LSH_USE_GRAPH      run the fixed-shape part of the search
 *                           (signatures through the small-bucket pair
 *                           kernel) as one captured HIP graph, replayed on
 *                           later calls whose shapes, device pointers and
 *                           workspace are unchanged.  Results are identical
 *                           with and without it. */
enum { FAST_LSH_WANT_DISTINCT = 1, FAST_LSH_USE_GRAPH = 2 };

/* Full similarity search (section 6.1 "Search"; filters of sections 6.5 and
 * 7.1): writes the sorted pairs to out_i, out_j (device uint32) and
 * out_votes (device uint8), at most `capacity` of them, and the counters to
 * *stats (host, may be NULL).  Blocking.
 * If more than `capacity` pairs qualify the call returns E_CAPACITY with
 * stats->n_out set; the result stays in the context until its next search,
 * so fast_lsh_copy_result can fetch it into larger buffers.
 * The band key must fit 64 bits (ceil(log2 dim) * r <= 64). */
int fast_lsh_search(fast_lsh_ctx *ctx, const fast_lsh_hash *hash, const fast_lsh_fps *fps,
                    const fast_lsh_filter *filter, uint32_t *out_i, uint32_t *out_j, uint8_t *out_votes,
                    uint64_t capacity, fast_lsh_stats *stats);

/* fast_lsh_search with option flags (FAST_LSH_WANT_DISTINCT also computes
 * stats->n_distinct, which costs a full comparison of every candidate). */
int fast_lsh_search_ex(fast_lsh_ctx *ctx, const fast_lsh_hash *hash, const fast_lsh_fps *fps,
                       const fast_lsh_filter *filter, uint32_t flags, uint32_t *out_i, uint32_t *out_j,
                       uint8_t *out_votes, uint64_t capacity, fast_lsh_stats *stats);

/* Largest number of stations in one batched search. */
enum { FAST_LSH_MAX_STATIONS = 16 };

/* Batched search: the search of fast_lsh_search applied to each of
 * n_stations independent stations (the paper searches each station's
 * fingerprints on their own, section 7 and section 8 data sets), run as one
 * pass of every kernel over all stations.  Pairs never mix stations, and the
 * occurrence filter uses each station's own n.
 *   stations         host array of n_stations fingerprint sets (1..16);
 *   out_i, out_j     device uint32: pairs of station 0, then station 1, ...,
 *   out_votes        each station's pairs sorted by (i, j), ids local to the
 *                    station (0 = its first fingerprint);
 *   station_offsets  host, n_stations + 1 entries (may be NULL): station s
 *                    owns output entries [offsets[s], offsets[s+1]);
 *   per_station      host, n_stations entries (may be NULL): each station's
 *                    counters, as fast_lsh_search would report them.
 * The stations' total n must be below 2^31, and with more than one station
 * the band key must leave its top 4 bits free for the station tag
 * (ceil(log2 dim) * r <= 60).  Capacity overflow behaves as in
 * fast_lsh_search (E_CAPACITY, offsets and counters still written). */
int fast_lsh_search_batched(fast_lsh_ctx *ctx, const fast_lsh_hash *hash, uint32_t n_stations,
                            const fast_lsh_fps *stations, const fast_lsh_filter *filter, uint32_t flags,
                            uint32_t *out_i, uint32_t *out_j, uint8_t *out_votes, uint64_t capacity,
                            uint64_t *station_offsets, fast_lsh_stats *per_station);

/* Bounded-memory search: the result and counters of fast_lsh_search_ex
 * (identical bytes), computed with the tables taken group_tables at a time,
 * the way the paper bounds memory by partitioning the search (section 6.4).
 * Sorting and bucket segmentation need room for one group of tables only.
 * Pass 1 computes each group's signatures once, groups and segments it
 * (bucket sizes and exclusions over all tables) and stores a 16-bit
 * sub-key row and a 32-bit key word per table and fingerprint, which exact
 * key comparisons use instead of full 64-bit keys.  Pass 2 emits the pairs
 * group by group: from pass 1's kept grouping (ids in bucket order, marks,
 * large-bucket descriptors) for as many groups as fast_lsh_config's
 * keep_groups and the free HBM allow, otherwise after rebuilding, sorting
 * and segmenting the group's keys again.  Workspace, in bytes, is about
 *   n * (4 t + 2 t' + 1) + group_tables * n * (24 + 1) + small tables
 *   + kept groups * group_tables * n * 5 + candidate queue,
 * with t' = t rounded up to whole 32-bit words per group of the vote filter
 * and the candidate queue 16 * 1024 * queue_slot bytes (512 MiB at the
 * automatic size from n >= 2,097,152; fast_lsh_config) plus one byte per 64
 * positions of a group's tables and per tile of the tiled pairs (the
 * fast_lsh_search workspace is about n * (2 t' + 1) + 33 t n plus the
 * queue); like
 * every workspace buffer it stays allocated in the context (reported by
 * fast_lsh_workspace_bytes) until the context is destroyed.
 * Requires band keys of at most 48 bits (ceil(log2 dim) * r <= 48) and does
 * not take FAST_LSH_USE_GRAPH. */
int fast_lsh_search_bounded(fast_lsh_ctx *ctx, const fast_lsh_hash *hash, const fast_lsh_fps *fps,
                            const fast_lsh_filter *filter, uint32_t flags, uint32_t group_tables,
                            uint32_t *out_i, uint32_t *out_j, uint8_t *out_votes, uint64_t capacity,
                            fast_lsh_stats *stats);

/* Copy the last search's result (kept in the context) into caller buffers
 * with room for `capacity` pairs.  E_CAPACITY if it still does not fit,
 * E_INVALID if there is no result.  Ids are local to their station. */
int fast_lsh_copy_result(fast_lsh_ctx *ctx, uint32_t *out_i, uint32_t *out_j, uint8_t *out_votes,
                         uint64_t capacity);

/* Launch shapes.  They change speed only: every choice gives the same output
 * bytes and counters.
 *   radix_tile    elements per workgroup of the grouping passes: 16384,
 *                 8192 or 4096 (0 keeps the current value);
 *   bucket_chunk  sorted positions per wavefront of the bucket kernel (the
 *                 span it stages in LDS): 256..1536, a multiple of 256
 *                 (0 keeps the current value);
 *   autotune      1: on the first search of each shape (stations, total n,
 *                 tables, bin bits) time every radix tile and bucket chunk
 *                 on that search's own data, keep the fastest for later
 *                 searches of that shape (the fixed values above are then
 *                 ignored); 0: use the fixed values;
 *   bin_bits      top bits of the mixed key the grouping passes sort on
 *                 (8, 16, 24 or 32: one radix pass per 8 bits; equal keys
 *                 share every bit, so any choice gives the same buckets,
 *                 coarser bins leave more keys for the bucket kernel to
 *                 separate); 0: the automatic rule (bins of the largest
 *                 station averaging at most about 4 fingerprints);
 *   keep_groups   bounded search: the most table groups whose grouping
 *                 (bucket-ordered ids, small-bucket marks, large-bucket
 *                 descriptors: 5 bytes per fingerprint and table, plus the
 *                 descriptors) pass 1 keeps for pass 2, which then runs the
 *                 pair kernels on them instead of sorting and segmenting
 *                 those groups again.  FAST_LSH_KEEP_AUTO: as many as the
 *                 free HBM (less a margin of 4 GiB and 2 %) and the
 *                 context's budget hold; 0: none.  fast_lsh_config_used
 *                 reports the number the last bounded search kept;
 *   queue_slot    pair kernels of the need == 2 form (min_votes v split
 *                 over v - 1 table groups, need = 2): a pair whose sub-keys
 *                 pass the group test is queued, up to queue_slot entries
 *                 per spread slot (16 bytes each, 1024 slots), and a later
 *                 launch gives the queued pairs their exact key checks one
 *                 lane per pair; a workgroup whose slot fills up runs again
 *                 with the checks in place (fast_lsh_work.pair_redos).
 *                 0: automatic (n / 64, between 64 and 32768; none on
 *                 a context with an HBM budget, or when the free HBM does
 *                 not hold it); FAST_LSH_QUEUE_OFF: no queue, checks in
 *                 place; at most 2^20 (E_NOMEM when it does not fit).  Any
 *                 value gives the same result.
 *                 fast_lsh_config_used reports the last search's size. */
#define FAST_LSH_KEEP_AUTO 0xFFFFFFFFu
#define FAST_LSH_QUEUE_OFF 0xFFFFFFFFu
typedef struct {
  uint32_t radix_tile;
  uint32_t bucket_chunk;
  uint32_t autotune;
  uint32_t bin_bits;
  uint32_t keep_groups;
  uint32_t queue_slot;
} fast_lsh_config;

/* Set the launch shapes of later searches (defaults: 16384, 512, no
 * autotune, automatic bin bits, FAST_LSH_KEEP_AUTO, automatic queue).  E_INVALID for a value
 * outside the lists above. */
int fast_lsh_configure(fast_lsh_ctx *ctx, const fast_lsh_config *config);

/* The launch shapes the last search used (after autotuning, its choice). */
int fast_lsh_config_used(fast_lsh_ctx *ctx, fast_lsh_config *out);

/* ---------------------------------------------------------------------------
 * Serving form: stations whose tables stay resident, searched chunk by chunk.
 *
 * A server owns a HIP stream and a worker thread.  Each station is admitted
 * with its history (built into resident tables: per table, the mixed band
 * keys and ids sorted by key, 12 bytes per row and table, plus room to grow);
 * chunks of new rows are then submitted as they arrive.  Each chunk is
 * searched against everything its station holds at that point (history,
 * earlier chunks, and its own earlier rows) and then inserted, so chunk c's
 * result is every pair (i, j) with j in chunk c, i < j, j - i >= min_lag and
 * votes >= min_votes (section 6.1 "Search" applied as a query, section 6.4),
 * with station ids (history rows 0..n-1, then the chunks' rows in order).
 * The union of the chunk results is the fast_lsh_search result of the whole
 * station minus the history's own pairs.  The occurrence filter depends on
 * the whole station and is not offered here (filter occ_den must be 0).
 *
 * Continuous batching: while a batch runs, arriving chunks wait; the next
 * batch takes the oldest waiting chunks, at most one per station (a
 * station's chunk waits for the one before it) and at most max_batch.
 * A chunk's ticket is done as soon as its result is on the host; the batch's
 * chunks are then inserted into their stations (merging a full delta into
 * the history) before the next batch runs.  If an insertion fails (a device
 * or allocation error), that chunk's result stands and every later chunk of
 * the station fails with the insertion's error.
 * HBM admission: a station is admitted only if its tables, its share of the
 * shared history-merge buffer and its build buffers fit the budget.  A chunk
 * is admitted only if its rows fit the station's tables (history rows plus
 * slack_rows, less the rows of the chunks already queued for the station):
 * otherwise submit returns E_NOMEM and the station is unchanged, so no
 * admitted chunk can fail its insertion.  With a budget, the first submit
 * also checks that a full batch's workspace (max_batch chunks of max_chunk
 * rows) fits beside the resident tables.
 * Chunk rows are DEVICE memory that must stay valid until the chunk's ticket
 * is done; results are returned in HOST arrays.  Entry points other than
 * submit/poll/take/now/info must not run concurrently with each other.
 * ------------------------------------------------------------------------- */
typedef struct fast_lsh_server fast_lsh_server;

typedef struct {
  uint32_t max_batch;   /* chunks per batch, 1..16                                   */
  uint32_t max_chunk;   /* rows per chunk, 1..4096                                   */
  uint64_t delta_rows;  /* rows of recent chunks kept per station before they are
                           merged into its history tables (>= max_chunk)            */
  uint64_t slack_rows;  /* rows each station may grow by                             */
  uint64_t hbm_budget;  /* bytes for all resident tables and workspace (0: no bound) */
} fast_lsh_server_config;

typedef struct {
  uint32_t stations, waiting;  /* admitted stations, chunks waiting            */
  uint64_t resident_bytes;     /* station tables and the shared merge buffer   */
  uint64_t workspace_bytes;    /* batch workspace                              */
  uint64_t batches, chunks;    /* batches run, chunks they held                */
  uint64_t largest_batch;
} fast_lsh_server_state;

/* cfg may be NULL: {8, 3600, 262144, 2000000, 0}. */
int fast_lsh_server_create(int device, const fast_lsh_hash *hash, const fast_lsh_filter *filter,
                           const fast_lsh_server_config *cfg, fast_lsh_server **out);
/* Stops the worker after the waiting chunks are done and frees everything. */
void fast_lsh_server_destroy(fast_lsh_server *server);
/* Admit a station with its history (device rows; may be empty); *station
 * receives its index.  Stations are added before the first submit (E_BUSY
 * after).  E_NOMEM when the budget cannot hold it. */
int fast_lsh_server_add_station(fast_lsh_server *server, const fast_lsh_fps *history, uint32_t *station);
/* Queue a chunk (device rows, 1..max_chunk of them) of `station`;
 * arrival_ns is the caller's arrival time on the server clock
 * (fast_lsh_server_now_ns) and is kept for latency accounting.  *ticket
 * receives the chunk's ticket.  Thread-safe, does not block.  E_NOMEM when
 * the chunk's rows do not fit its station (see HBM admission above). */
int fast_lsh_server_submit(fast_lsh_server *server, uint32_t station, const fast_lsh_fps *chunk,
                           uint64_t arrival_ns, uint64_t *ticket);
/* FAST_LSH_OK with the chunk's counters (as fast_lsh_search defines them, for
 * the chunk's pairs; max_bucket: the largest bucket holding one of its rows)
 * and its completion time on the server clock once it is done, E_BUSY
 * before (wait != 0 blocks until done), or the chunk's own error (E_INVALID
 * for a bad row: the station is left unchanged). */
int fast_lsh_server_poll(fast_lsh_server *server, uint64_t ticket, int wait, fast_lsh_stats *stats,
                         uint64_t *done_ns);
/* Copy a done chunk's pairs, sorted by (i, j), into HOST arrays and release
 * the ticket (E_CAPACITY keeps it). */
int fast_lsh_server_take(fast_lsh_server *server, uint64_t ticket, uint32_t *out_i, uint32_t *out_j,
                         uint8_t *out_votes, uint64_t capacity);
/* Nanoseconds on the server clock (steady, from server creation). */
uint64_t fast_lsh_server_now_ns(fast_lsh_server *server);
int fast_lsh_server_info(fast_lsh_server *server, fast_lsh_server_state *out);
/* The batching rule on its own (host only): stations[k] is the station of
 * the k-th waiting chunk, oldest first; picked[0..*n_picked) receives the
 * indices of the chunks the next batch takes. */
int fast_lsh_plan_batch(const uint32_t *stations, uint32_t n_waiting, uint32_t max_batch, uint32_t *picked,
                        uint32_t *n_picked);

/* Device memory the context's workspace holds now, in bytes (it grows to
 * the largest search run on the context and is freed by ctx_destroy). */
int fast_lsh_workspace_bytes(fast_lsh_ctx *ctx, uint64_t *bytes);

/* Stage timing.  While enabled, the context records a pair of HIP events on
 * its stream around every kernel launch of the stages below and accumulates
 * their elapsed times when each call completes (there is no limit on the
 * number of launches a call records).  Enabling resets the counters.
 * Stages: */
enum {
  FAST_LSH_STAGE_SIGNATURES = 0, /* signature kernel                          */
  FAST_LSH_STAGE_GROUP = 1,      /* the radix passes that bin every table     */
  FAST_LSH_STAGE_BUCKETS = 2,    /* per-bin sort, bucket sizes, filter flags  */
  FAST_LSH_STAGE_BIG_BINS = 3,   /* bins too large for LDS                    */
  FAST_LSH_STAGE_PAIRS = 4,      /* in-bucket pairs and votes, small buckets  */
  FAST_LSH_STAGE_BIG_PAIRS = 5,  /* tiled pairs of large buckets              */
  FAST_LSH_STAGE_OUTPUT = 6,     /* canonical sort of the reported pairs      */
  FAST_LSH_STAGE_GRAPH = 7,      /* replay of the captured graph (stages 0-4
                                    together, FAST_LSH_USE_GRAPH only)        */
  FAST_LSH_STAGE_SPLIT_KEYS = 8, /* bounded search, second pass: a group's
                                    mixed keys rebuilt from stored words      */
  FAST_LSH_STAGE_CHANNEL_MERGE = 9, /* fast_lsh_channel_merge                 */
  FAST_LSH_STAGE_CLUSTERS = 10,  /* fast_lsh_station_clusters                 */
  FAST_LSH_STAGE_FINGERPRINTS = 11, /* fast_lsh_fingerprints: images, Haar,
                                       statistics, top-K                      */
  FAST_LSH_STAGE_SPECTROGRAM = 12,  /* fast_lsh_fingerprints: STFT power      */
  FAST_LSH_STAGE_PAIR_CHECKS = 13,  /* exact checks of the pairs the pair
                                       kernels queued (need == 2 form)        */
  FAST_LSH_PROFILE_STAGES = 14
};

typedef struct {
  double ms[FAST_LSH_PROFILE_STAGES];         /* summed kernel time per stage */
  uint64_t launches[FAST_LSH_PROFILE_STAGES]; /* timed intervals per stage    */
} fast_lsh_profile;

int fast_lsh_profile_enable(fast_lsh_ctx *ctx, int enable);
int fast_lsh_profile_read(fast_lsh_ctx *ctx, fast_lsh_profile *out);

/* Work counters of the last search on the context (fast_lsh_search,
 * _search_ex, _search_batched, _search_bounded), for rooflines: the buckets
 * above 64 members, whose pairs the tiled kernel checks.  big_members sums
 * their sizes m and big_candidates their in-bucket pairs C(m, 2) (over every
 * table; part of e_raw); big_voted counts those pairs that pass the lag and
 * the exclusion (part of e_voted).  search_calls counts the searches
 * completed on the context; pair_redos the second runs of pair launches
 * (workgroups whose candidate queue slot filled up) in the last search.
 * Zero before the first search. */
typedef struct {
  uint64_t big_voted, big_members, big_candidates, search_calls, pair_redos;
} fast_lsh_work;

int fast_lsh_last_work(fast_lsh_ctx *ctx, fast_lsh_work *out);

/* Partitioned search with the dynamic occurrence filter (section 6.4
 * "Partition", section 6.5 "Removing correlated noise").  The n
 * fingerprints are split into n_partitions consecutive id ranges
 * [n p / P, n (p + 1) / P) (P = min(n_partitions, n)), taken in order.  For
 * partition p: (1) every fingerprint of p not excluded yet counts its
 * near-neighbour candidates: the distinct other fingerprints at least
 * min_lag away, not excluded, that share a bucket with it in some table;
 * (2) when occ_den != 0, the fingerprints of p whose count c satisfies
 * c * occ_den > |p| * occ_num are excluded together with all their
 * candidates (counts taken before any exclusion of p); (3) the pairs (i, j)
 * with i in p, i < j, j - i >= min_lag, neither excluded, votes >= min_votes
 * are reported.  Exclusions only affect later output.  With occ_den == 0
 * the output equals fast_lsh_search's without filter, for every partition
 * count.  Output and capacity as fast_lsh_search (one table group: pass
 * FAST_LSH_WANT_DISTINCT for n_distinct); stats: e_raw and max_bucket of
 * all tables (no static filter), e_voted / n_distinct over the pairs the
 * partitions could report, n_flagged the fingerprints excluded at the end.
 * E_INVALID for n_partitions == 0, FAST_LSH_USE_GRAPH or bad inputs.
 * Cost: one pass over all buckets when nothing is excluded (it counts and
 * reports every partition); otherwise that pass, one counting and one
 * reporting pass, and for each partition that excludes an exclusion pass
 * and at most one more counting and reporting pass. */
int fast_lsh_search_partitioned(fast_lsh_ctx *ctx, const fast_lsh_hash *hash, const fast_lsh_fps *fps,
                                const fast_lsh_filter *filter, uint32_t flags, uint32_t n_partitions,
                                uint32_t *out_i, uint32_t *out_j, uint8_t *out_votes, uint64_t capacity,
                                fast_lsh_stats *stats);

/* Fingerprint extraction parameters (section 5.1; the paper gives no
 * values).  window: samples per STFT frame (periodic Hann), at most 256;
 * hop: samples between frames (1-64; window * 65 + 256 * hop <= 16384);
 * [band_lo, band_hi): the frequency bins kept (bin k = k / window cycles
 * per sample), 8, 16, 32 or 64 of them = the image rows; fp_frames frames
 * per fingerprint, averaged time_ds at a time into fp_frames / time_ds
 * image columns (a power of two); rows * cols in [64, 2048]; fp_lag: frames
 * between consecutive fingerprints; top_k: set bits per fingerprint
 * (<= rows * cols).  The fingerprint dimension is 2 * rows * cols. */
typedef struct {
  uint32_t window, hop, band_lo, band_hi, fp_frames, time_ds, fp_lag, top_k;
} fast_lsh_fp_params;

/* Fingerprint extraction (section 5.1; section 5.2 normalization statistics
 * from a sample) of one channel: samples[n_samples] (DEVICE float32) ->
 * n_fp = (n_frames - fp_frames) / fp_lag + 1 fingerprints, n_frames =
 * (n_samples - window) / hop + 1.  Steps: STFT power in the band; per
 * fingerprint the spectral image (rows = bins, columns = averaged frames);
 * the 2-D orthonormal Haar transform (rows, then columns; per axis the
 * final average, then details coarsest to finest; coefficient c = row *
 * cols + column); z = (w - median) / MAD per coefficient (z = 0 where
 * MAD = 0), median and MAD the lower middle values over the fingerprints
 * sample_ids[n_sample] (DEVICE, each < n_fp; the caller draws the sample);
 * the top_k coefficients of largest |z| (ties: smaller c; z != 0 only);
 * bit 2c for z > 0, 2c + 1 for z < 0.  Output: out[n_fp][top_k] (DEVICE
 * uint16, ascending bit indices; a fingerprint with fewer than top_k
 * non-zero z fills the rest with 0xFFFF), out_count[n_fp] (DEVICE, optional:
 * bits per fingerprint), med_mad (DEVICE, optional: 2 * rows * cols floats,
 * the medians then the MADs).  *n_fp (HOST) is set even on E_CAPACITY
 * (n_fp > capacity: nothing written).  Arithmetic in float32.  Workspace:
 * the spectrogram (4 * rows bytes per frame) and 24 bytes per (sampled
 * fingerprint, coefficient).  Blocking. */
int fast_lsh_fingerprints(fast_lsh_ctx *ctx, const float *samples, uint64_t n_samples,
                          const fast_lsh_fp_params *params, const uint64_t *sample_ids, uint64_t n_sample,
                          uint16_t *out, uint32_t *out_count, uint64_t capacity, uint64_t *n_fp, float *med_mad);

/* Query-only hashing (section 6.4, "Partition"): only the queries are
 * hashed into the t tables; every dataset item is looked up in each table,
 * and (query q, item x) gets one vote per table in which x falls in q's
 * bucket.  Output: every pair with votes >= min_votes, ordered by (q, x),
 * in DEVICE arrays out_q, out_x (query and item indices), out_votes
 * (caller-owned); the same pairs a search over tables holding the whole
 * dataset reports for the queries.  No lag and no occurrence filter apply
 * (queries and items are separate sets).  stats (HOST, optional): n_out;
 * e_raw = e_voted = the (table, query, item) matches; n_distinct is not
 * computed (all ones); the rest 0.  Queries and dataset hold fewer than
 * 2^32 fingerprints each.  E_CAPACITY when n_out > capacity (nothing
 * written, stats set); E_INVALID for bad hash parameters or fingerprints.
 * Workspace: the queries' tables (24 bytes per query and table), the
 * dataset's keys for a group of tables (at most 8 GB), 24 bytes per
 * match.  Blocking. */
int fast_lsh_query(fast_lsh_ctx *ctx, const fast_lsh_hash *hash, const fast_lsh_fps *queries,
                   const fast_lsh_fps *dataset, uint32_t min_votes, uint32_t *out_q, uint32_t *out_x,
                   uint8_t *out_votes, uint64_t capacity, fast_lsh_stats *stats);

/* ------------------------------------------------------------------------
 * Spatiotemporal alignment of search outputs (section 7)
 * ------------------------------------------------------------------------ */

/* One channel's search output: count pairs (i[k], j[k], votes[k]) with
 * i < j, all DEVICE pointers (the arrays a search returns).  As a triplet of
 * section 7.2 a pair is (dt, idx1, sim) = (j - i, i, votes). */
typedef struct {
  const uint32_t *i, *j;
  const uint8_t *votes;
  uint64_t count;
} fast_lsh_pairs;

/* Channel-level merge (section 7.1 "Channel Level"; section 7.2 "Channel",
 * sort-merge-reduce): the similarity matrices of the n_channels channels of
 * one station (same time base) are summed, and entries whose summed
 * similarity is below min_sim are dropped.
 *
 * channels: HOST array of n_channels descriptors (device arrays; any order
 * of pairs within a channel; a channel should not repeat a pair, repeats
 * are summed like entries of different channels).  n_fingerprints: the
 * station's fingerprint count, every id must be below it (at most 2^32 - 1).
 * Output: DEVICE arrays out_dt, out_idx1, out_sim (uint32, caller-owned) of
 * the combined entries with sim >= min_sim, ordered by (dt, idx1); *n_out
 * (HOST) is their number.  E_CAPACITY when *n_out > capacity (nothing
 * written; call again with room for *n_out); E_INVALID for NULL pointers or
 * a pair with j <= i or j >= n_fingerprints.  Workspace: about 40 bytes per
 * input pair.  Blocking (returns when the outputs are written). */
int fast_lsh_channel_merge(fast_lsh_ctx *ctx, uint32_t n_channels, const fast_lsh_pairs *channels,
                           uint64_t n_fingerprints, uint32_t min_sim, uint32_t *out_dt, uint32_t *out_idx1,
                           uint32_t *out_sim, uint64_t capacity, uint64_t *n_out);

/* Allocation-free channel merge, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, semantics and errors as
 * fast_lsh_channel_merge, but every intermediate buffer lives in one
 * fixed scratch array of FAST_LSH_NOALLOC_SCRATCH_BYTES per device, which
 * the library's code object holds from its first use on that device until
 * the process ends; the call allocates nothing (no hipMalloc, no workspace
 * growth, no stage timing).  Inputs whose buffers exceed the array (about
 * 36 bytes per input pair plus small scan and histogram arrays: at most
 * 1,860,736 pairs) are rejected with FAST_LSH_E_NOMEM.  The array is shared
 * by every call on the device: calls that overlap on one device (several
 * contexts or threads at once) race and must be serialised by the caller;
 * each call clears the parts it needs, so earlier contents never matter. */
#define FAST_LSH_NOALLOC_SCRATCH_BYTES (64ull << 20)
int fast_lsh_channel_merge_noalloc(fast_lsh_ctx *ctx, uint32_t n_channels, const fast_lsh_pairs *channels,
                                   uint64_t n_fingerprints, uint32_t min_sim, uint32_t *out_dt,
                                   uint32_t *out_idx1, uint32_t *out_sim, uint64_t capacity, uint64_t *n_out);

/* Station-level clustering parameters (section 7.2 "Station"; the paper
 * gives no values).  A run along one diagonal continues while consecutive
 * entries' idx1 differ by at most max_gap; runs of diagonals dt and dt + 1
 * join when their idx1 spans [lo, hi] come within max_gap of each other
 * (equivalently: the clusters are the connected components of the entries,
 * two entries being neighbours when their dt differ by at most one and their
 * idx1 by at most max_gap).  A cluster is kept when its width
 * dt_max - dt_min + 1 is at most max_width ("relatively narrow"), it holds
 * at least min_entries entries and its summed similarity is at least
 * min_sum (small clusters and isolated matches are pruned). */
typedef struct {
  uint32_t max_gap, max_width, min_entries, reserved; /* reserved: set to 0 */
  uint64_t min_sum;
} fast_lsh_cluster_params;

/* One kept cluster: its bounding box, entry count, summed similarity and
 * strongest entry (largest sim; among equal sims the first in (dt, idx1)
 * order).  40 bytes. */
typedef struct {
  uint32_t dt_min, dt_max, idx1_min, idx1_max;
  uint32_t n_entries, peak_sim, peak_dt, peak_idx1;
  uint64_t sim_sum;
} fast_lsh_cluster;

/* Station-level clustering (section 7.1 "Station Level"; section 7.2
 * "Station") of n combined entries (dt[k], idx1[k], sim[k]), DEVICE arrays
 * strictly ordered by (dt, idx1) (the channel merge's output), n < 2^32,
 * every sim below 2^24.  Output: the kept clusters in the order of their
 * first entry, written to the DEVICE array out (caller-owned); *n_out
 * (HOST) is their number.  E_CAPACITY when *n_out > capacity (nothing
 * written); E_INVALID for NULL pointers, entries out of order or repeated,
 * or a sim of 2^24 or more.  Workspace: about 50 bytes per entry.  Blocking. */
int fast_lsh_station_clusters(fast_lsh_ctx *ctx, const uint32_t *dt, const uint32_t *idx1, const uint32_t *sim,
                              uint64_t n, const fast_lsh_cluster_params *params, fast_lsh_cluster *out,
                              uint64_t capacity, uint64_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* FAST_LSH_H */
