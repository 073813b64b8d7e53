// Shared device helpers and launch-argument structs of the fast_lsh HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

constexpr uint32_t kP = 0x7FFFFFFFu;  // Mersenne prime 2^31 - 1 of the hash family

// Counters updated by many workgroups are spread over kSpread slots (summed
// on the host): atomics of every workgroup on one address serialise.
constexpr uint32_t kSpread = 1024;

__device__ __forceinline__ uint32_t spread_slot() {
  return (blockIdx.x + blockIdx.y * 977u + blockIdx.z * 7919u) % kSpread;
}

// --------------------------------------------------------------------------
// Universal hash h(x) = (a x + b) mod p evaluated from pre-doubled
// parameters a2 = 2a, b2 = 2b (both < 2^32).  With y = a x + b < 2^48,
// Y = a2 x + b2 = 2y, so the low word of Y shifted right by one is y & p and
// the high word is y >> 31; their sum is congruent to y mod p and below
// 2^31 + 2^17, so one conditional subtraction (done as an unsigned min with
// the wrapped difference) gives the canonical residue.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t hash_mod(uint32_t a2, uint32_t b2, uint32_t x) {
  uint64_t y2 = (uint64_t)a2 * x + b2;
  uint32_t s = ((uint32_t)y2 >> 1) + (uint32_t)(y2 >> 32);
  return min(s, s - kP);
}

// The folded hash before its last correction: s = (y & p) + (y >> 31) with
// y = a x + b, congruent to y mod p.  For x < 2^16, s < 2^31 + 2^16 + 1, and
// s is the canonical residue exactly when s < p; otherwise the residue is
// s - p (below 2^16 + 2).
__device__ __forceinline__ uint32_t hash_fold(uint32_t a2, uint32_t b2, uint32_t x) {
  uint64_t y2 = (uint64_t)a2 * x + b2;
  return ((uint32_t)y2 >> 1) + (uint32_t)(y2 >> 32);
}

// Twice the folded hash, wrapped: t = 2 s mod 2^32 = (Y mod 2^32) +
// 2 (Y >> 32) for Y = a2 x + b2 = 2y (one multiply-add and one shift-add).
// Doubling keeps the order of the values below 2^31; s = p gives t = 2p, and
// s >= 2^31 (possible only when s >= p) wraps to t = 2 (s - 2^31) < 2 dim.
// Written as the one shift-add instruction: from C the compiler, knowing the
// high word is below 2^17, rewrites the shift as a funnel shift and a mask.
__device__ __forceinline__ uint32_t hash_fold2(uint32_t a2, uint32_t b2, uint32_t x) {
  const uint64_t y2 = (uint64_t)a2 * x + b2;
  uint32_t t;
  asm("v_lshl_add_u32 %0, %1, 1, %2" : "=v"(t) : "v"((uint32_t)(y2 >> 32)), "v"((uint32_t)y2));
  return t;
}

// (u * w) mod p for u, w < p, canonical.
__device__ __forceinline__ uint32_t mul_mod(uint32_t u, uint32_t w) {
  uint64_t z = (uint64_t)u * w;  // < 2^62
  uint32_t s = ((uint32_t)z & kP) + (uint32_t)(z >> 31);  // < 2^32
  s = s >= kP ? s - kP : s;
  s = s >= kP ? s - kP : s;
  return s;
}

// murmur3 64-bit finaliser: a bijection of 64-bit words.  Used (1) for the
// chained band key when the packed key would not fit 64 bits and (2) to
// spread band keys uniformly before grouping (equal keys stay equal).
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// A bijection of 60-bit words (xor-shifts and odd multipliers modulo 2^60),
// used when the top four bits of the mixed key hold a station id: keys of
// one station then stay contiguous after sorting, and equal keys stay equal.
__device__ __forceinline__ uint64_t mix60(uint64_t k) {
  constexpr uint64_t M = (1ull << 60) - 1;
  k &= M;
  k ^= k >> 31;
  k = (k * 0xbf58476d1ce4e5b9ull) & M;
  k ^= k >> 29;
  k = (k * 0x94d049bb133111ebull) & M;
  k ^= k >> 32;
  return k;
}

// A bijection of 48-bit words, for band keys of at most 48 bits: with the
// mixed key m = mix48(key) << 16, the sub-key (bits 16-31) and the high word
// (bits 32-63) together determine the band key.
__device__ __forceinline__ uint64_t mix48(uint64_t k) {
  constexpr uint64_t M = (1ull << 48) - 1;
  k &= M;
  k ^= k >> 24;
  k = (k * 0xff51afd7ed558ccdull) & M;
  k ^= k >> 23;
  k = (k * 0xc4ceb9fe1a85ec53ull) & M;
  k ^= k >> 24;
  return k;
}

// Mixed-key forms (SigArgs::mix).
enum : uint32_t {
  kMixFull = 0,    // fmix64(band key); sub-key = bits 0-15
  kMixStation = 1, // station << 60 | mix60(band key); sub-key = bits 0-15
  kMixSplit = 2    // mix48(band key) << 16; sub-key = bits 16-31, high word = bits 32-63
};

// --------------------------------------------------------------------------
// Sub-key rows.  Each fingerprint carries, per group of tables, a row of
// 16-bit sub-keys (the low bits of its mixed band key in each table of the
// group), field k in bits [16k, 16k+16) of the row, in row_dw dwords.
// Equal band keys give equal sub-keys.  Consecutive fingerprints' rows lie
// row_pitch dwords apart: row_dw itself (dense), or padded so that no row
// crosses a 128-byte line, which halves the memory requests of a random row
// read.
// --------------------------------------------------------------------------
constexpr uint32_t kSubBits = 16;
constexpr uint32_t kSubMask = (1u << kSubBits) - 1;

__host__ __device__ constexpr uint32_t row_dwords(uint32_t tables) { return (kSubBits * tables + 31) / 32; }
__host__ __device__ constexpr uint32_t row_fields(uint32_t dwords) { return 32 * dwords / kSubBits; }
// Line-aligned pitch: the next power of two up to 32 dwords (one 128-byte
// line), whole lines above that (rows start at 128-byte aligned bases).
__host__ __device__ constexpr uint32_t row_pitch_lines(uint32_t dwords) {
  uint32_t p = 1;
  while (p < dwords && p < 32) p *= 2;
  return dwords <= 32 ? p : (dwords + 31) / 32 * 32;
}

// Field k of the row r.
__device__ __forceinline__ uint32_t row_field(const uint32_t* r, uint32_t k) {
  return (r[k >> 1] >> (16 * (k & 1))) & kSubMask;
}

// --------------------------------------------------------------------------
// Launch arguments
// --------------------------------------------------------------------------
struct SigArgs {
  const uint16_t* ind;   // fingerprint indices
  const uint64_t* off;   // n+1 offsets or nullptr (fixed nnz)
  uint64_t n;
  uint32_t nnz;          // fixed row length when off == nullptr
  uint32_t dim;
  uint32_t r;            // rows per band key
  uint32_t fpt;          // functions per table (r or r/2)
  uint32_t table_begin;
  uint32_t table_count;
  uint32_t kbits;        // ceil(log2 dim)
  uint32_t packed;       // 1: key = packed indices; 0: chained fmix64
  uint32_t vec_load;     // 1: rows are CAP halfwords, 16-byte aligned
  const uint32_t* a2;    // per function: 2a
  const uint32_t* b2;    // 2b
  const uint32_t* ainv;  // a^-1 mod p
  const uint32_t* b;     // b
  uint64_t* keys;        // [table_count][n] band keys, or nullptr
  uint32_t* sigs;        // [n][table_count][r] values, or nullptr
  uint64_t* mkeys;       // [table_count][out_stride] mixed keys, or nullptr
  uint32_t* rows;        // sub-key rows [G][out_stride][row_pitch], or nullptr
  uint64_t out_stride;   // fingerprints per table in mkeys / rows (all stations)
  uint64_t out_base;     // first position of this station in mkeys / rows
  uint64_t tag;          // station id << 60 (kMixStation): keeps stations apart
  uint32_t mix;          // kMixFull, kMixStation or kMixSplit
  uint32_t* hi32;        // [num_tables][out_stride] high words of split keys (global table index), or nullptr
  uint32_t tables_per_group;
  uint32_t row_dw;       // dwords per row
  uint32_t row_pitch;    // dwords from one fingerprint's row to the next
  int* err;              // set to 1 on an empty row or an index >= dim
};

struct BucketArgs {
  const uint64_t* keys;  // sorted by the bin bits, [S][n]
  uint32_t* vals;        // ids, same order; rewritten sorted by (key, id)
  uint64_t n;
  uint32_t chunk;
  uint32_t bin_shift;    // bin = key >> bin_shift (64 - B)
  // occurrence filter: station of an id found from station_base (nstation+1 entries)
  const uint64_t* station_base;
  const uint64_t* occ_max;  // per station: largest bucket within the threshold (all ones: no filter)
  uint32_t nstation;
  uint32_t occ_num, occ_den;
  uint32_t min_lag;      // buckets whose id span is below this yield no pair
  uint8_t* flags;        // per fingerprint
  uint32_t small_max;    // buckets of size <= small_max are marked in place
  uint8_t* marks;        // [S][n]: size of the small pair-capable bucket starting here, else 0
  uint4* big_desc;       // {pos, seg, size, 0}
  uint32_t* big_count;
  uint4* bin_desc;       // oversized bins {lo, hi, seg, 0}
  uint32_t* bin_count;
  unsigned long long* e_raw;    // [nstation][kSpread]
  unsigned int* max_bucket;     // [nstation][kSpread]
};

struct PairArgs {
  const uint32_t* order;      // bucket members by position [S][n]
  const uint8_t* flags;
  const uint32_t* rows;       // sub-key rows [G][n][row_pitch]
  const uint64_t* mkeys;      // exact mixed keys [t][n], or nullptr when hi32 is given
  const uint32_t* hi32;       // high words of split keys [t][n] (with equal sub-keys: equal keys)
  uint64_t n;
  uint32_t t, G, tables_per_group, row_dw;
  uint32_t row_pitch;         // dwords from one fingerprint's row to the next
  uint32_t table_offset;      // table of launch segment 0 (segment s is table table_offset + s)
  uint32_t min_lag, min_votes, need;
  uint32_t want_distinct;
  uint32_t* out_i;
  uint32_t* out_j;
  uint8_t* out_v;
  unsigned int* out_count;
  uint32_t out_cap;
  unsigned long long* e_voted;     // [nstation][kSpread]
  unsigned long long* n_distinct;  // [nstation][kSpread]
  const uint64_t* station_base;    // nstation + 1 entries
  uint32_t nstation;
  const unsigned long long* n_flagged;  // total excluded (device), 0: skip flag lookups
  unsigned long long* big_voted;   // [kSpread] pairs counted in e_voted by the tiled kernel (or nullptr)
  // Partitioned search with the dynamic occurrence filter (one table group,
  // first shared table found exactly as for the distinct count).  part_mode
  // 0: plain search; 1: every candidate pair, at its first shared table,
  // adds one to cand[] of its members in [plo, phi); 2: at its first shared
  // table, a pair with exactly one member in fp[] (the partition's
  // over-threshold fingerprints) sets ex_next[] of the other; 3: the plain
  // search restricted to pairs whose smaller id lies in [plo, phi); 4: modes
  // 1 and 3 over all ids in one pass (before any exclusion).
  uint32_t part_mode;
  uint32_t plo, phi;
  uint32_t* cand;
  const uint8_t* fp;
  uint8_t* ex_next;
  // Candidate queue of the need == 2 form: a pair that passes the sub-key
  // group test is appended as (i, j, table, chunk) to its workgroup's
  // spread slot, q[slot][0, qcap), and given its exact checks by a later
  // launch with one lane per pair, instead of stalling its wavefront on
  // them.  The chunk is the small-bucket kernel's 64 positions of a table
  // (segment * nchunk + chunk) or the tiled kernel's unit.  A pair that
  // finds its slot full sets q_ovf[chunk] and *q_any; the checks skip the
  // chunk's entries and the host runs the launch again with redo set (only
  // the marked chunks work, checks in place, no vote tallies).  qcap == 0:
  // checks in place.
  uint4* q;
  unsigned int* q_count;  // [kSpread] appends per slot (may pass qcap)
  uint32_t qcap;
  uint8_t* q_ovf;         // per chunk of the launch
  unsigned int* q_any;
  uint32_t redo;
};

// Station of a (global) fingerprint id, for nb stations with ascending bases.
__device__ __forceinline__ uint32_t station_of(const uint64_t* base, uint32_t nb, uint64_t id) {
  uint32_t s = 0;
  while (s + 1 < nb && base[s + 1] <= id) ++s;
  return s;
}

// Workgroups of a launch are handed to the eight XCDs in turn (workgroup b
// to XCD b mod 8), each XCD with its own L2.  Kernels whose neighbouring
// workgroups share data take their work item from xcd_block: a bijection of
// [0, nb) that gives each XCD a contiguous range of items (b goes to the
// (b / 8)-th item of XCD (b mod 8)'s range; the first nb mod 8 XCDs hold
// q + 1 items, the others q, q = nb / 8).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  constexpr uint32_t kXcd = 8;
  const uint32_t q = nb / kXcd, r = nb % kXcd, x = b % kXcd, idx = b / kXcd;
  return x < r ? x * (q + 1) + idx : r * (q + 1) + (x - r) * q + idx;
}

// Buckets of at most kSmallBucket members are handled by the wave-per-chunk
// pair kernel (their members staged in LDS); larger ones by the tile kernel.
// The pair forms that compare each pair against a row held in registers
// (the FAST test on 10- or 17-dword rows) take buckets of up to 64 members
// there; the forms with longer rows or full counts take up to 32, since the
// wave kernel's LDS span, and with it its residency, grows with the limit.
constexpr uint32_t kSmallBucket = 64;
constexpr uint32_t kSmallBucketGeneral = 32;


}  // namespace fl
