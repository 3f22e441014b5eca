// Kernel launch descriptors and kernel declarations of libmj (internal).
#pragma once
#include "mj_device.h"

namespace mj {

// ---------------------------------------------------------------- partition
#ifndef MJ_PART_THREADS
#define MJ_PART_THREADS 512
#endif
#ifndef MJ_PART_TILE
#define MJ_PART_TILE 8192
#endif
#ifndef MJ_DB_THREADS
#define MJ_DB_THREADS 512
#endif
#ifndef MJ_CELL_THREADS
#define MJ_CELL_THREADS 512
#endif
constexpr int PART_THREADS = MJ_PART_THREADS;
#ifndef MJ_PART_SCATTER_THREADS
#define MJ_PART_SCATTER_THREADS 1024
#endif
constexpr int PART_SCATTER_THREADS = MJ_PART_SCATTER_THREADS;   // scatter: more tuples in flight per tile
constexpr int PART_TILE = MJ_PART_TILE;  // tuples per block (<= 2^16)
constexpr int PART_SCAN_CHUNK = 4096;    // row-scan chunk (LDS entries)
constexpr int MJ_PART_MAX_JOBS = 4;
constexpr uint32_t PART_MAX_BITS = 12;   // at most 4096 buckets per pass
constexpr size_t LDS_BYTES = 160 * 1024; // per workgroup on gfx950
// the scatter's dynamic LDS (two words per bucket, a staged tile of pairs)
// plus its static wave scratch must fit one workgroup
static_assert((size_t(8) << PART_MAX_BITS) + size_t(8) * PART_TILE + 4 * (PART_SCATTER_THREADS / 64 + 1) <= LDS_BYTES,
              "partition tile does not fit LDS");
static_assert(PART_TILE <= 65536 && PART_TILE % (2 * PART_THREADS) == 0 &&
              PART_TILE % (2 * PART_SCATTER_THREADS) == 0, "partition tile shape");

// Work items of a per-bucket kernel when a bucket holds too many tuples
// for one workgroup (skew: a heavy key or a crowded range).  k_part_scan
// writes them when the job asks: a bucket of more than `chunk` tuples is
// split into split_pieces(len, chunk) pieces, each a workgroup of its own;
// item g = bucket | piece << 12.  The pieces of a split bucket leave their
// sums in scratch rows hrow[bucket] + piece, and the last piece to finish
// (counted in done[bucket]) adds the rows and writes the bucket's outputs,
// then sets done[bucket] back to 0 for the next kernel over the same items.
struct BucketItems {     // null unless set, however the holder is declared
    uint32_t* items = nullptr;   // [nb + n / chunk + 1]; null: one workgroup per bucket
    uint32_t* nitems = nullptr;  // [1]
    uint32_t* hrow = nullptr;    // [nb]
    uint32_t* done = nullptr;    // [nb]
    uint32_t chunk = 0;          // at least SPLIT_MIN_CHUNK
};
constexpr uint32_t SPLIT_MIN_CHUNK = 4096;   // pieces < 2^20 for any n < 2^32
__host__ __device__ inline uint32_t split_pieces(uint32_t len, uint32_t chunk) {
    return len > chunk ? (len - 1) / chunk + 1 : 1u;
}

struct PartJob {
    const uint32_t* col0;
    const uint32_t* col1;
    int64_t stride;
    uint64_t n;
    uint32_t packed;     // stride 2, col1 == col0 + 1, 16-byte aligned: 16-byte loads
    uint32_t key0_col;   // column (0/1) hashed for the first digit
    uint32_t key1_col;   // column hashed for the second digit (bits1 > 0)
    uint32_t seed0, bits0;
    uint32_t seed1, bits1;
    uint32_t* hist;      // [nb][ntiles] per-tile counts, then run offsets
    uint32_t* counts;    // [nb] bucket sizes
    uint32_t* starts;    // [nb + 1] bucket starts
    uint2* out_pair;     // both columns as (col0, col1), or
    uint32_t* out_single;// one column (single_col, also the bucketed column)
    uint32_t single_col;
    uint32_t range_on;   // bucket = min(key0 >> range_shift, 2^bits0 - 1) (no hash; pairs only)
    uint32_t range_shift;
    uint32_t swap_out;   // pairs written as (col1, col0)
    uint32_t tile_begin; // first block of this job in the grid
    uint32_t ntiles;
    BucketItems split;   // optional work items of the buckets (k_part_scan)
};

struct PartLaunch {
    PartJob job[MJ_PART_MAX_JOBS];
    int njobs;
    uint32_t* clear = nullptr;   // words k_part_hist sets to 0 first (flags of the caller's kernels)
    uint32_t nclear = 0;
};

MJ_KERNEL_DECL(k_part_hist, PartLaunch);
MJ_KERNEL_DECL(k_part_rowscan, PartLaunch);
MJ_KERNEL_DECL(k_part_scan, PartLaunch);
MJ_KERNEL_DECL(k_part_scatter, PartLaunch);
size_t part_scatter_smem(uint32_t max_bits);

// ------------------------------------------------- multiplicity tables (D)
// Per bucket j an open-addressing table of (key, multiplicity) pairs lives
// in a pool; dir[j] locates it.  Key 0xFFFFFFFF is kept in `special`.
struct DirEntry {
    unsigned long long offset;   // first slot in the pool
    uint32_t log2cap;
    uint32_t special;            // multiplicity of key 0xFFFFFFFF in this bucket
};

constexpr int DB_THREADS = MJ_DB_THREADS;
constexpr uint32_t DB_CAP = 8192;                  // LDS slots per build
// distinct keys before spilling; after the flag each thread claims at most
// one more slot, so the table keeps at least one empty slot
constexpr uint32_t DB_LIMIT = DB_CAP - (DB_CAP / 8 > DB_THREADS ? DB_CAP / 8 : DB_THREADS) - 1;
static_assert(DB_LIMIT + DB_THREADS < DB_CAP, "LDS table slack");
static_assert(DB_CAP % DB_THREADS == 0, "rehash takes DB_CAP / DB_THREADS slots per thread");
constexpr uint32_t DB_MIN_CAP = 16;

struct DBuildArgs {
    const uint32_t* keys;        // partitioned single-column relation
    const uint32_t* starts;      // [nbkt + 1]
    uint32_t nbkt;
    uint32_t slot_seed;
    DirEntry* dir;               // [nbkt]
    uint2* pool;                 // (key, count) slots
    unsigned long long* pool_cursor;
    unsigned long long pool_cap;
    uint32_t* err;               // set to 1 if the pool is exhausted
    // optional (heavy keys): buckets split into pieces, one workgroup each;
    // each piece's counts (DB_CAP slots of (key, count)) and its count of
    // key 0xFFFFFFFF by scratch row; split.done[bucket] counts finished
    // pieces, its top bit set when a piece's table overflowed
    BucketItems split;
    uint2* rows = nullptr;
    uint32_t* row_special = nullptr;
};
MJ_KERNEL_DECL(k_dbuild, DBuildArgs);

// Lookup in a bucketed multiplicity table; 0 when absent.
__device__ __forceinline__ uint32_t dtab_lookup(const DirEntry* __restrict__ dir,
                                                const uint2* __restrict__ pool,
                                                uint32_t key, uint32_t bkt_seed,
                                                uint32_t bkt_bits, uint32_t slot_seed) {
    const uint32_t j = top_bits(mix32(key, bkt_seed), bkt_bits);
    const DirEntry e = dir[j];
    if (key == EMPTY_KEY) return e.special;
    const uint32_t mask = (1u << e.log2cap) - 1u;
    uint32_t s = slot_hash(key, slot_seed) & mask;
    const uint2* base = pool + e.offset;
    while (true) {
        uint2 kv = base[s];
        if (kv.x == key) return kv.y;
        if (kv.x == EMPTY_KEY) return 0u;
        s = (s + 1u) & mask;
    }
}

// Four independent lookups: the directory loads, then the first slot loads
// are issued together so that four table reads are in flight per lane;
// only keys that collide walk further.
// The rest of an open-addressing probe whose first slot `s` has been read
// as `v`: walk on until the key or an empty slot; `none` when absent.
// (A function of scalars, so that callers holding several probes in
// flight keep them in registers.)
__device__ __forceinline__ uint32_t probe_from(const uint2* __restrict__ base, uint32_t mask, uint32_t key,
                                               uint2 v, uint32_t s, uint32_t none) {
    while (v.x != key && v.x != EMPTY_KEY) {
        s = (s + 1u) & mask;
        v = base[s];
    }
    return v.x == key ? v.y : none;
}

__device__ __forceinline__ void dtab_lookup4(const DirEntry* __restrict__ dir,
                                             const uint2* __restrict__ pool,
                                             const uint32_t (&key)[4], const bool (&live)[4],
                                             uint32_t bkt_seed, uint32_t bkt_bits,
                                             uint32_t slot_seed, uint32_t (&out)[4]) {
    DirEntry e[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (live[u]) e[u] = dir[top_bits(mix32(key[u], bkt_seed), bkt_bits)];
    uint32_t s[4];
    uint2 kv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (live[u] && key[u] != EMPTY_KEY) {
            s[u] = slot_hash(key[u], slot_seed) & ((1u << e[u].log2cap) - 1u);
            kv[u] = pool[e[u].offset + s[u]];
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (!live[u]) { out[u] = 0u; continue; }
        if (key[u] == EMPTY_KEY) { out[u] = e[u].special; continue; }
        out[u] = probe_from(pool + e[u].offset, (1u << e[u].log2cap) - 1u, key[u], kv[u], s[u], 0u);
    }
}

// --------------------------------------------------------- linear cells
constexpr int CELL_THREADS = MJ_CELL_THREADS;
constexpr uint32_t CELL_CAP = 4096;                      // W-table slots (LDS)
constexpr uint32_t CELL_LIMIT = CELL_CAP - (CELL_CAP / 8 > CELL_THREADS ? CELL_CAP / 8 : CELL_THREADS) - 1;
static_assert(CELL_LIMIT + CELL_THREADS < CELL_CAP, "LDS table slack");

struct LinearCellArgs {
    const uint2* R;              // partitioned (a, b) by bucket of b
    const uint32_t* rstarts;     // [nb + 1]
    const uint2* S;              // partitioned (b, c) by bucket of b
    const uint32_t* sstarts;     // [nb + 1]
    const DirEntry* ddir;        // multiplicity tables of T.c
    const uint2* dpool;
    uint32_t c_seed, c_bits, slot_seed;
    uint32_t w_seed;             // hash for W slots and pass split
    unsigned long long* count;   // [a_domain]
    uint32_t a_domain;
    uint32_t* err;
};
__global__ void k_linear_cell(LinearCellArgs A);

// ------------------------------ linear: W tables and counts per range of A
// W[b] = sum over s(b, c) in S of mult_T(c), one open-addressing table per
// b-bucket (the cells' buckets) in a pool of 16-byte slots; then one
// workgroup per range of A values adds W[r.b] into an LDS count per a and
// writes its range of the output once.
struct WDirEntry {
    unsigned long long offset;   // first slot in the pool
    unsigned long long special;  // W of key 0xFFFFFFFF in this bucket
    uint32_t log2cap;
    uint32_t pad;
};
struct __align__(16) WSlot {
    uint32_t key;
    uint32_t pad;
    unsigned long long w;
};
constexpr uint32_t W_MIN_CAP = 16;

struct WBuildArgs {
    const uint2* S;              // partitioned (b, c) by bucket of b
    const uint32_t* sstarts;     // [nb + 1]
    const DirEntry* ddir;        // multiplicity tables of T.c
    const uint2* dpool;
    uint32_t c_seed, c_bits, slot_seed;
    uint32_t w_seed;             // hash of W slots and of the pass split
    WDirEntry* wdir;             // [nb]
    WSlot* wpool;                // slots [0, W_MIN_CAP) stay empty
    unsigned long long* wcursor;
    unsigned long long wcap;
    uint32_t* err;               // set to 1 if the pool is exhausted
    // optional (heavy keys): buckets of S split into pieces, one workgroup
    // each; each piece's W table (CELL_CAP slots) and its sum for
    // b = 0xFFFFFFFF by scratch row; split.done[bucket] counts finished
    // pieces, its top bit set when a piece's table overflowed (the last
    // piece then builds the bucket from its tuples)
    BucketItems split;
    WSlot* rows = nullptr;
    unsigned long long* row_special = nullptr;
};
__global__ void k_wbuild(WBuildArgs A);

// ------------------------------------------------ S-largest linear join
// Sec. 4, the paragraph after Algorithm 1: R split into L_R parts by the
// bucket of B, T into L_T parts by the bucket of C, S into the L_R x L_T
// pairs.  R_i's distinct B values form a table (the multiplicity tables of
// R's B column, slots hashed with the W seed) with a u64 sum beside every
// slot; a workgroup per (i, j, piece of S_ij) copies T_j's multiplicities
// and R_i's keys into LDS, streams its piece of S_ij, sums w = mult_Tj(c)
// per B value of R_i in LDS (B values absent from R_i are skipped) and adds
// its sums to the table's once.
#ifndef MJ_SL_LOG2
#define MJ_SL_LOG2 12
#endif
#ifndef MJ_SL_THREADS
#define MJ_SL_THREADS 1024
#endif
constexpr uint32_t SL_T_LOG2 = MJ_SL_LOG2;     // T_j tables of at most 2^SL_T_LOG2 slots staged
constexpr uint32_t SL_R_LOG2 = MJ_SL_LOG2;     // R_i key tables of at most 2^SL_R_LOG2 slots staged
constexpr int SL_THREADS = MJ_SL_THREADS;
struct SlCellArgs {
    const uint2* S;              // S partitioned by (bucket of b, bucket of c)
    const uint32_t* sstarts;     // [L_R * L_T + 1]
    uint32_t r_bits, t_bits;     // log2 L_R, log2 L_T
    uint32_t pieces;             // workgroups per (i, j)
    const DirEntry* rdir;        // R's B tables (keys; slots hashed with w_seed)
    const uint2* rpool;
    uint32_t w_seed;
    unsigned long long* wval;    // sums beside the slots of rpool
    unsigned long long* wspecial;// [L_R] sum for b = 0xFFFFFFFF
    const DirEntry* tdir;        // T's C tables
    const uint2* tpool;
    uint32_t slot_seed;
};
__global__ void k_sl_cell(SlCellArgs A);
// R's B tables with their sums, rewritten as W tables (the format the
// per-A counts read): one workgroup per part of R
__global__ void k_sl_wtables(const DirEntry* rdir, const uint2* rpool, const unsigned long long* wval,
                             const unsigned long long* wspecial, WDirEntry* wdir, WSlot* wpool);

static_assert(CELL_CAP % CELL_THREADS == 0, "rehash takes CELL_CAP / CELL_THREADS slots per thread");
constexpr int COUNT_THREADS = 512;
constexpr uint32_t ACELL_MAX_SHIFT = 12;     // at most 4096 A values (32 KB of LDS) per range

constexpr int RANGE_THREADS = 1024;         // range sums: one workgroup per range of keys

// Direct-indexed tables (keys in a small dense domain).  Per range of keys,
// one workgroup: out[key] = sum over the range's tuples of weight(v), summed
// in LDS and written once (zeros included); weight(v) = 1 without a table,
// else table[v] (0 for v >= table_n).  A key outside [0, domain) sets err.
template <class TW, class TWN, class TO, class TON>
struct RangeAccArgs {
    const uint2* pairs;          // (key, v) by range of key; null: keys only
    const uint32_t* keys;        // keys by range (when pairs is null)
    const uint32_t* starts;      // [ranges + 1]
    uint32_t shift;              // range k holds keys [k << shift, (k + 1) << shift)
    uint32_t domain;
    const TW* table;             // null: weight 1
    uint32_t table_n;
    TO* out;                     // [domain]
    uint32_t* err;
    // optional narrow forms, read by the next kernel instead of the full
    // array.  Flagged (deg): out_narrow receives out cut to TON and `wide` is
    // set when some entry does not fit; table_narrow is read instead of
    // table while `use_wide` is clear.  Saturating (W): an entry that does
    // not fit is stored as TON's largest value, and a reader that finds that
    // value reads the entry from table instead (wide and use_wide unused).
    TON* out_narrow;
    uint32_t* wide;
    const TWN* table_narrow;
    const uint32_t* use_wide;
    // optional: ranges split into pieces (items.items null: one workgroup
    // per range); rows: scratch of row_len entries of TO per piece
    BucketItems split;
    void* rows = nullptr;
    uint32_t row_len = 0;
};
// deg[c]: keys only, weight 1 (flagged 16-bit copy)
typedef RangeAccArgs<uint32_t, uint16_t, uint32_t, uint16_t> RangeDegArgs;
MJ_KERNEL_DECL(k_range_deg, RangeDegArgs);
// W[b] += deg[s.c] (reads deg's flagged copy; writes a saturating 16-bit copy)
typedef RangeAccArgs<uint32_t, uint16_t, unsigned long long, uint16_t> RangeWArgs;
MJ_KERNEL_DECL(k_range_w, RangeWArgs);
// count[a] += W[r.b] (reads W's saturating copy)
typedef RangeAccArgs<unsigned long long, uint16_t, unsigned long long, uint32_t> RangeCountArgs;
MJ_KERNEL_DECL(k_range_count, RangeCountArgs);
// every entry of out set to all ones when *err is set (a certified key bound broken)
struct PoisonArgs { unsigned long long* out; uint64_t n; const uint32_t* err; };   // out[0..n) = ~0 when *err
MJ_KERNEL_DECL(k_poison_u64, PoisonArgs);
// *err set when a size found on the device (*got) is not the one the plan
// was made with (a plan reused on data of the same sizes but other contents)
struct CheckSizeArgs { const unsigned long long* got; unsigned long long want; uint32_t* err; };   // err = 1 when *got != want
MJ_KERNEL_DECL(k_check_size, CheckSizeArgs);

struct CountArgs {
    const uint2* R;              // partitioned (a, b) by range of a
    const uint32_t* rstarts;     // [number of ranges + 1]
    const WDirEntry* wdir;
    const WSlot* wpool;
    uint32_t b_seed, b_bits, w_seed;
    uint32_t a_shift;            // range k holds a in [k << a_shift, (k + 1) << a_shift)
    uint32_t a_domain;
    unsigned long long* count;   // [a_domain], every entry written
    uint32_t* err;               // set to 1 for an a >= a_domain
    BucketItems split;           // optional: ranges split into pieces
    unsigned long long* rows = nullptr;  // scratch rows of 2^a_shift entries
};
__global__ void k_count(CountArgs A);

// probe S.b (or any column) against a bucketed multiplicity table and sum
struct ProbeSumArgs {
    const uint32_t* col;
    int64_t stride;
    uint64_t n;
    const DirEntry* dir;
    const uint2* pool;
    uint32_t bkt_seed, bkt_bits, slot_seed;
    unsigned long long* total;
};
__global__ void k_probe_sum(ProbeSumArgs A);

// ------------------------------------------------------------- star join
// The linear query when R and T are small dimension relations and S a large
// fact relation (Sec. 6, star 3-way join): R's and T's tables (one bucket
// each) are held on chip -- copied into every workgroup's LDS while each has
// at most STAR_LDS_SLOTS slots -- and S is streamed once.  R's distinct B
// values are numbered 0..k-1 (a prefix sum over the occupied slots of its
// table, the key 0xFFFFFFFF taking the extra slot pool_slots); the pass over
// S adds mult_T(c) per number in LDS and each workgroup writes its sums once.
// Tables too large for LDS are probed in L2 and the sums go to global
// memory.  The star cascade materialises I = R |x| S and groups it by A.
constexpr int STAR_THREADS = 1024;         // one workgroup per CU
constexpr int STAR_REDUCE_THREADS = 1024;  // 64 groups x 16 rows of per-block sums
constexpr uint32_t STAR_LDS_SLOTS = 8192;  // table slots held in LDS
constexpr uint32_t STAR_GROUPS = 4096;     // A values per LDS array (the cascade)
constexpr uint32_t STAR_STRIDE = STAR_LDS_SLOTS / 2 + 1;   // sums per workgroup (ids, or A values)
constexpr uint32_t STAR_NONE = 0xFFFFFFFFu;
constexpr uint32_t STAR_GRID = 1024;       // most workgroups of a launch
constexpr uint64_t STAR_ROWS_PER_BLOCK = 16384;
static_assert(STAR_GROUPS < STAR_STRIDE, "the cascade's sums fit a workgroup's stride");

struct StarTable {                 // a one-bucket table of (key, multiplicity) slots
    const DirEntry* dir;           // [1]
    const uint2* pool;
    uint32_t bkt_seed, slot_seed;
    uint32_t pool_slots;           // the slot of key 0xFFFFFFFF
};

// occ[i] = 1 for i < cursor holding a key, and for i = pool_slots when key
// 0xFFFFFFFF occurs
struct StarOccArgs {
    StarTable R;
    const unsigned long long* cursor;
    uint32_t* occ;                 // [pool_slots + 1]
};
MJ_KERNEL_DECL(k_star_occ, StarOccArgs);

// idtab[slot] = (key, id) for the occupied slots of R's table (same
// positions, so a probe of idtab with the table's hash yields the id)
struct StarIdArgs {
    StarTable R;
    const unsigned long long* rid;
    uint2* idtab;                  // [pool_slots]
};
MJ_KERNEL_DECL(k_star_ids, StarIdArgs);

struct StarGroupArgs {
    const uint32_t* col0;          // (key, c) rows: S as (b, c) or I as (a, c)
    const uint32_t* col1;
    int64_t stride;
    uint64_t n;
    StarTable T;                   // weights mult_T(c)
    StarTable R;                   // grouping by B: R's table
    const uint2* idtab;            // (key, id) slots of R's table
    const unsigned long long* rid; // [pool_slots + 2] exclusive prefix of occ
    uint32_t ngroups_max;          // grouping by A: a_domain
    unsigned long long* partial;   // [gridDim][STAR_STRIDE] per-block sums (LDS modes)
    unsigned long long* out;       // global sums (global modes)
    uint32_t* err;                 // set for an A value >= a_domain
};
// by B (the star three-way join's pass over S): sums per id of b
MJ_KERNEL_DECL(k_star_group_b, StarGroupArgs);
// by A value (the star cascade's second join): sums per a
MJ_KERNEL_DECL(k_star_group_a, StarGroupArgs);

struct StarReduceArgs {
    const unsigned long long* partial;
    uint32_t nblocks;
    uint32_t by_b;                 // 1: per id of b (when both tables were in LDS); 0: per a
    const DirEntry* rdir;
    const DirEntry* tdir;
    const unsigned long long* rid;
    uint32_t pool_slots;           // R's
    uint32_t ngroups_max;          // by A: a_domain
    unsigned long long* out;       // overwritten (LDS modes) or left (global modes)
};
MJ_KERNEL_DECL(k_star_reduce, StarReduceArgs);

// count[a] += W[id(b)] over R's tuples
struct StarCountArgs {
    const uint32_t* col0;
    const uint32_t* col1;
    int64_t stride;
    uint64_t n;
    StarTable R;
    const unsigned long long* rid;
    const unsigned long long* W;
    unsigned long long* count;
    uint32_t a_domain;
    uint32_t* err;
};
MJ_KERNEL_DECL(k_star_count, StarCountArgs);

// Star cascade (binary joins): R grouped by the id of B, I = R |x| S
// materialised as (a, c) pairs, then I grouped by a with weights mult_T(c).
struct StarRIndexArgs {            // counting sort of R's A values by id(b)
    const uint32_t* col0;
    const uint32_t* col1;
    int64_t stride;
    uint64_t n;
    StarTable R;
    const unsigned long long* rid;
    const unsigned long long* roff;  // [k + 1] exclusive prefix of multiplicities
    uint32_t* rcur;                  // [k] fill cursors (zeroed)
    uint32_t* ra;                    // [n] A values by id
};
struct StarRMultArgs { StarRIndexArgs x; uint32_t* mult; };   // mult[id] = multiplicity
MJ_KERNEL_DECL(k_star_rmult, StarRMultArgs);
MJ_KERNEL_DECL(k_star_rfill, StarRIndexArgs);

struct StarExpandArgs {
    const uint32_t* col0;            // S as (b, c)
    const uint32_t* col1;
    int64_t stride;
    uint64_t n;
    StarTable R;
    const uint2* idtab;
    const unsigned long long* rid;
    const unsigned long long* roff;
    const uint32_t* ra;
    uint32_t* icnt;                  // [n] pairs per S tuple (count pass)
    const unsigned long long* ioff;  // [n + 1] (write pass)
    uint2* I;                        // (a, c) pairs
    uint64_t i_cap;                  // pairs I holds; positions beyond are reported
    uint32_t* err;
};
MJ_KERNEL_DECL(k_star_icount, StarExpandArgs);
MJ_KERNEL_DECL(k_star_expand, StarExpandArgs);

// ------------------------------------------------------------- cascade
constexpr int CAS_THREADS = 512;
constexpr uint32_t CAS_CAP = 4096;
constexpr uint32_t CAS_LIMIT = CAS_CAP - (CAS_CAP / 8 > CAS_THREADS ? CAS_CAP / 8 : CAS_THREADS) - 1;
static_assert(CAS_LIMIT + CAS_THREADS < CAS_CAP, "LDS table slack");
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_TILE = 4096;
constexpr int EXP_THREADS = 256;
constexpr int EXP_TILE = 4096;
constexpr uint32_t EXP_WIN = 2048;        // list starts of one expansion tile held in LDS

struct CasIndexArgs {
    const uint2* R;              // partitioned (a, b) by bucket of b
    const uint32_t* rstarts;
    const uint2* S;              // partitioned (b, c) by bucket of b
    const uint32_t* sstarts;
    uint32_t* Rgrp;              // A values of R grouped by B inside each bucket
    uint32_t* ecnt;              // per S tuple: |{r : r.b = s.b}|
    uint32_t* elist;             // per S tuple: start of its list in Rgrp
    uint32_t seed;
};
MJ_KERNEL_DECL(k_cas_index, CasIndexArgs);

struct CasExpandArgs {
    const unsigned long long* eoff;   // [ns + 1] exclusive scan of ecnt
    const uint32_t* elist;
    const uint32_t* Rgrp;
    const uint2* S;
    uint64_t ns;
    unsigned long long lo, hi;        // chunk of I positions
    uint2* I;                         // [hi - lo]
    uint32_t swap;                    // write (S value, grouped value) instead of (grouped value, S value)
};
MJ_KERNEL_DECL(k_cas_expand, CasExpandArgs);

// I's pairs (a, c) come with the pairs of one A value consecutive (the
// first join probes with R): each wave sums its runs of equal a before one
// atomic per run
struct CasProbeArgs {
    const uint2* I;
    uint64_t n;
    const DirEntry* ddir;
    const uint2* dpool;
    uint32_t c_seed, c_bits, slot_seed;
    unsigned long long* count;
    uint32_t a_domain;
    uint32_t* err;
    // dense keys: mult_T(c) = deg[c] (its 2-byte copy while *use_wide is clear)
    // for c < c_domain, instead of the bucketed tables
    const uint32_t* deg;
    const uint16_t* deg16;
    uint32_t c_domain;
    const uint32_t* use_wide;
};
MJ_KERNEL_DECL(k_cas_probe, CasProbeArgs);


// out[i] = sum of in[0..i) for i in [0, n]: per tile of SCAN_TILE a partial
// sum (k_scan_reduce), the partials' exclusive prefix in place with
// partial[nblk] = the total (k_scan_partials), then each tile's prefix
// (k_scan_apply); or, for at most one tile, all of it in one workgroup
// (k_scan_one)
template <class In>
struct ScanArgsT {
    const In* in;
    uint64_t n;
    unsigned long long* partial;   // [nblk + 1]
    unsigned long long* out;       // [n + 1]
    uint32_t nblk;                 // tiles of SCAN_TILE
};
typedef ScanArgsT<uint32_t> ScanArgs;
typedef ScanArgsT<unsigned long long> Scan64Args;
MJ_KERNEL_DECL(k_scan_reduce, ScanArgs);
MJ_KERNEL_DECL(k_scan_reduce64, Scan64Args);
MJ_KERNEL_DECL(k_scan_partials, ScanArgs);
MJ_KERNEL_DECL(k_scan_apply, ScanArgs);
MJ_KERNEL_DECL(k_scan_apply64, Scan64Args);
MJ_KERNEL_DECL(k_scan_one, ScanArgs);
MJ_KERNEL_DECL(k_scan_one64, Scan64Args);

// ------------------------------------------------------------- radix sort
constexpr int RS_THREADS = 256;
constexpr int RS_TILE = 4096;
struct RsArgs {
    const unsigned long long* in;
    unsigned long long* out;
    uint64_t n;
    uint32_t shift;              // digit = (key >> shift) & 255
    uint32_t ntiles;
    uint32_t* hist;              // [256][ntiles]
    const uint32_t* starts;      // [257] digit starts
};
MJ_KERNEL_DECL(k_rs_hist, RsArgs);
MJ_KERNEL_DECL(k_rs_scatter, RsArgs);
// small arrays: the whole sort in one workgroup, or one scan launch per pass
constexpr uint32_t RS_SMALL_BITS = 14;
constexpr uint32_t RS_SMALL = 1u << RS_SMALL_BITS;   // keys sorted whole in LDS
constexpr int RS_SMALL_THREADS = 1024;
constexpr uint32_t RS_SCAN1_TILES = 32;              // tiles scanned by one workgroup
static_assert(size_t(RS_SMALL) * 8 <= LDS_BYTES && RS_SMALL_BITS <= 16, "small sort shape");
struct RsSmallArgs { unsigned long long* keys; uint32_t n; uint32_t shift; };
struct RsScan1Args { RsArgs rs; uint32_t* starts; };
MJ_KERNEL_DECL(k_rs_small, RsSmallArgs);
MJ_KERNEL_DECL(k_rs_scan1, RsScan1Args);

// --------------------------------------------------------------- triangle
constexpr int TRI_THREADS = 256;           // light kernel: one table per wave
constexpr int TRI_HEAVY_THREADS = 1024;    // heavy kernel: one table per workgroup
constexpr uint32_t TRI_LIGHT_X = 512;      // R list length handled by one wave
constexpr uint32_t TRI_LIGHT_CAP = 1024;   // its LDS table (load <= 1/2)
static_assert(TRI_LIGHT_CAP <= 65536, "used slots are kept as 16-bit numbers");
constexpr uint32_t TRI_LIGHT_S = 4096;     // S group size handled by one wave
constexpr uint32_t TRI_HEAVY_X = 4096;     // R slice handled by one workgroup
constexpr uint32_t TRI_HEAVY_CAP = 8192;
constexpr uint32_t TRI_HEAVY_S = 2048;     // S tuples per heavy item (chunks of 64 per wave)
constexpr uint32_t TRI_SHORT_LIST = 16;    // heavy: lists walked by one lane

struct RunIndex {                          // runs of equal high words of sorted keys
    const uint32_t* run_key;               // [nruns]
    const uint32_t* run_start;             // [nruns + 1]
    const uint32_t* dir;                   // [2^bits + 1] first run with prefix >= p
    uint32_t bits;
    const unsigned long long* nruns;
};

// the run of `key` (start and length) through the prefix directory
__device__ __forceinline__ bool run_lookup(const RunIndex& X, uint32_t key, uint32_t& start,
                                           uint32_t& len) {
    const uint32_t p = top_bits(key, X.bits);
    uint32_t r = X.dir[p];
    const uint32_t rend = X.dir[p + 1];
    for (; r < rend; ++r) {
        const uint32_t k = X.run_key[r];
        if (k == key) {
            start = X.run_start[r];
            len = X.run_start[r + 1] - start;
            return true;
        }
        if (k > key) break;
    }
    return false;
}

// the index of the run of `key`, or 0xFFFFFFFF
__device__ __forceinline__ uint32_t run_find(const RunIndex& X, uint32_t key) {
    const uint32_t p = top_bits(key, X.bits);
    const uint32_t rend = X.dir[p + 1];
    for (uint32_t r = X.dir[p]; r < rend; ++r) {
        const uint32_t k = X.run_key[r];
        if (k == key) return r;
        if (k > key) break;
    }
    return 0xFFFFFFFFu;
}

// run_find for four keys at once: their dependent loads (directory, then run
// keys) are issued together, so that one thread keeps four lookups in flight
__device__ __forceinline__ void run_find4(const RunIndex& X, const uint32_t (&key)[4], const bool (&live)[4],
                                          uint32_t (&out)[4]) {
    uint32_t r[4], rend[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        out[u] = 0xFFFFFFFFu;
        r[u] = rend[u] = 0;
        if (live[u]) {
            const uint32_t p = top_bits(key[u], X.bits);
            r[u] = X.dir[p];
            rend[u] = X.dir[p + 1];
        }
    }
    bool more = true;
    while (more) {
        more = false;
        uint32_t k[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) k[u] = r[u] < rend[u] ? X.run_key[r[u]] : 0u;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (r[u] >= rend[u]) continue;
            if (k[u] == key[u]) { out[u] = r[u]; rend[u] = 0; }
            else if (k[u] > key[u]) rend[u] = 0;
            else if (++r[u] < rend[u]) more = true;
        }
    }
}

// ------------------------------------- Flajolet-Martin distinct count per A
// sketch[a] = the FM sketch (FM_WORDS bitmaps of 32 bits) of the set of D
// values a reaches through R |x| S |x| T.  A sketch is a union, so it is
// built along the linear join with OR in place of +: per C value from T's
// D values, per B value from S's C values, per A value from R's B values.
// T and S are grouped by sorting mixed 64-bit keys (runs of equal high
// words, as in the cyclic join); T's low words, mix(d) with the sketch's
// seed, are the sketch's hash values.
constexpr int FM_WORDS = 16;
constexpr int FM_THREADS = 256;
constexpr uint32_t FM_RANGE_MAX_SHIFT = 10;   // A values per LDS range (64 KB of sketches)
constexpr uint32_t FM_NONE = 0xFFFFFFFFu;
constexpr uint32_t FM_SHORT = 64;             // runs up to this length: one thread; longer: one wave

struct FmTArgs {                   // per run of T by C: OR of the bits of its D values
    RunIndex T;
    const unsigned long long* Tk;  // (mix(c) << 32 | mix(d)), sorted
    uint32_t* tsk;                 // [runs][FM_WORDS]
};
__global__ void k_fm_tsketch(FmTArgs A);        // runs of at most FM_SHORT elements, one thread each
__global__ void k_fm_tsketch_long(FmTArgs A);   // longer runs, one wave each

struct FmWArgs {                   // per run of S by B: OR of T's sketches of its C values
    RunIndex S;
    const unsigned long long* Sk;  // (mix(b) << 32 | mix(c)), sorted
    RunIndex T;
    const uint32_t* tsk;
    uint32_t* wsk;                 // [runs][FM_WORDS]
};
__global__ void k_fm_wsketch(FmWArgs A);        // runs of at most FM_SHORT elements, one thread each
__global__ void k_fm_wsketch_long(FmWArgs A);   // longer runs, one wave each

struct FmAArgs {                   // per A value: OR of the sketches of its B values
    const uint2* R;                // (a, b): by range of a (range mode), or as given (global mode)
    const uint32_t* rstarts;       // range mode: [ranges + 1]
    uint64_t n;                    // global mode: rows
    uint32_t a_shift;              // range mode: range k holds a in [k << a_shift, (k + 1) << a_shift)
    uint32_t a_domain;
    uint32_t seed;                 // mixes B the way S's keys were mixed
    RunIndex S;
    const uint32_t* wsk;
    uint32_t* sketch;              // [a_domain][FM_WORDS]
    double* est;                   // [a_domain] or null
    uint32_t* err;                 // set for an a >= a_domain
};
__global__ void k_fm_asketch(FmAArgs A);         // range mode: writes sketches and estimates
__global__ void k_fm_asketch_global(FmAArgs A);  // global mode: ORs into the zeroed output
__global__ void k_fm_estimate(FmAArgs A);        // global mode: estimates

struct TriKeyArgs {
    const uint32_t* key_col;
    const uint32_t* val_col;
    int64_t stride;
    uint64_t n;
    uint32_t seed;
    uint32_t raw_low;              // 1: the low word is the value itself, not its mix
    unsigned long long* out;
};

struct TriHeavyItem { uint32_t r0, r1, s0, s1; };

// One pass of the cyclic join: the lists of the staged relation (R per B,
// or T per C) are loaded into LDS one group at a time; the groups come from
// S sorted by that same attribute; each s of a group whose iterated list
// (T's list of c, or R's list of b) is the shorter one -- strictly shorter
// when `strict` -- streams that list past the staged one.  Two passes
// (staging R with strict = 1, staging T with strict = 0) see every S tuple
// exactly once, always iterating the shorter of its two lists.
struct TriClassifyArgs {
    RunIndex Stg, Grp;
    uint32_t share;
    uint32_t* nlight;
    uint32_t* light;
    uint32_t* nheavy_groups;
    uint32_t* heavy_group;
    uint32_t* heavy_items;
};

struct TriJoinArgs {
    RunIndex Stg, Grp, Itr;
    const uint32_t* Stgl;                  // low words (the other key) of the
    const uint32_t* Grpl;                  // sorted staged, grouped and
    const uint32_t* Itrl;                  // iterated relations
    uint32_t strict;
    const uint32_t* nlight;
    const uint32_t* light;
    uint32_t* light_next;
    const uint32_t* heavy_group;
    const unsigned long long* heavy_off;
    uint32_t n_heavy_cap;
    uint32_t* heavy_next;
    uint32_t share;
    unsigned long long* total;
};

struct CasProbeTriArgs {
    const uint2* I;                   // (a, c) pairs of R |x| S
    uint64_t n;
    RunIndex T;                       // T's lists per m(c), sorted by m(a)
    const unsigned long long* Tk;
    uint32_t seed;
    unsigned long long* total;
};
MJ_KERNEL_DECL(k_cas_probe_tri, CasProbeTriArgs);
struct TriBatchArgs {
    const TriJoinArgs* joins;            // [njoins] on the device
    uint32_t njoins;
    unsigned long long* light_base;      // [njoins + 1]
    unsigned long long* heavy_base;      // [njoins + 1]
    unsigned long long* next;            // [2] work counters
};
__global__ void k_tri_light_batch(TriBatchArgs B);
__global__ void k_tri_heavy_batch(TriBatchArgs B);
__global__ void k_tri_batch_prefix(TriBatchArgs B);

struct LinearBatchArgs {
    const LinearCellArgs* joins;         // [njoins] on the device
    const uint32_t* cell_base;           // [njoins + 1] first cell of each join
    uint32_t njoins;
};
__global__ void k_linear_cell_batch(LinearBatchArgs B);

MJ_KERNEL_DECL(k_tri_keys, TriKeyArgs);
// runs of equal high words of sorted keys: flags of run heads (and the low
// words, when `low` is set), then each head's run start and key, then a
// directory of the runs by the top `bits` bits of their keys
struct RunFlagsArgs { const unsigned long long* keys; uint64_t n; uint32_t* flags; uint32_t* low; };
struct RunCompactArgs {
    const unsigned long long* keys;
    uint64_t n;
    const uint32_t* flags;
    const unsigned long long* ridx;   // [n + 1] exclusive scan of flags
    uint32_t* run_key;
    uint32_t* run_start;
    unsigned long long* nruns;
};
// dir[p] = first run whose key prefix (top `bits` bits) is >= p, p in [0, 2^bits]
struct RunDirArgs { const uint32_t* run_key; const unsigned long long* nruns; uint32_t bits; uint32_t* dir; };
MJ_KERNEL_DECL(k_run_flags, RunFlagsArgs);
MJ_KERNEL_DECL(k_run_compact, RunCompactArgs);
MJ_KERNEL_DECL(k_run_dir, RunDirArgs);
MJ_KERNEL_DECL(k_tri_classify, TriClassifyArgs);
MJ_KERNEL_DECL(k_tri_light, TriJoinArgs);
MJ_KERNEL_DECL(k_tri_heavy, TriJoinArgs);

// ------------------------------------------------ materialised linear join
// The result tuples (a, b, c, d) of R |x| S |x| T written out in nested-loop
// order: r in R's order, then the s with s.b = r.b in S's order, then the t
// with t.c = s.c in T's order.  S and T are grouped by a stable sort on the
// mixed key (high word) with the raw other value as low word, so a run keeps
// its relation's order.  Positions come from three prefix sums:
//   P_S[i]  over S in run order: number of t for the S elements before i
//   O_I[j]  over R: number of (r, s) pairs of the R tuples before j
//   O_R[j]  over R: number of result tuples of the R tuples before j
struct EmitSArgs {                 // per S element (run order): its T run
    const uint32_t* sc;            // [ns] c, raw
    uint64_t ns;
    RunIndex T;
    uint32_t seed;
    uint32_t* tdeg;                // [ns] number of t with t.c = c
    uint32_t* tst;                 // [ns] first of them in T's run order
};
struct EmitRArgs {                 // per R tuple (R's order): its S run
    const uint32_t* r1;            // R's B column
    int64_t rstride;
    uint64_t nr;
    RunIndex S;
    uint32_t seed;
    const unsigned long long* P_S; // [ns + 1]
    uint32_t* sst;                 // [nr] first s with s.b = r.b in S's run order
    uint32_t* pdeg;                // [nr] number of such s
    unsigned long long* wout;      // [nr] number of result tuples of r
};
constexpr int EMIT_THREADS = 256;
constexpr uint32_t EMIT_TILE = 16384;      // output positions per workgroup
constexpr uint32_t EMIT_JWIN = 2048;       // R tuples of a tile whose pair starts fit LDS
struct EmitArgs {
    const uint32_t* r0;            // R's columns (a, b)
    const uint32_t* r1;
    int64_t rstride;
    uint64_t nr;
    const unsigned long long* O_R; // [nr + 1]
    const unsigned long long* O_I; // [nr + 1]
    const uint32_t* sst;           // [nr]
    const unsigned long long* P_S; // [ns + 1]
    const uint32_t* sc;            // [ns]
    const uint32_t* tst;           // [ns]
    const uint32_t* td;            // [nt] d, raw, in T's run order
    uint64_t first, cap;           // window of output positions (one launch's chunk)
    uint4* out;                    // [cap]
    ulonglong4* tiles;             // per tile: first and last pair, first and last R tuple
};
constexpr uint32_t EMIT_CHUNK_TILES = 65536;   // tiles per launch (2^30 output positions)
__global__ void k_emit_sdeg(EmitSArgs A);
__global__ void k_emit_rdeg(EmitRArgs A);
__global__ void k_emit_tiles(EmitArgs A, uint32_t ntiles);
__global__ void k_emit(EmitArgs A);

// ------------------------------------------- degree-oriented cyclic join
struct OrientArgs {
    const uint32_t* c0;            // the relation (u, v)
    const uint32_t* c1;
    int64_t stride;
    uint64_t n;
    RunIndex U;                    // runs of mix(u): the degrees
    uint32_t seed;
    uint32_t* flags;               // [n] 1: edge kept (points up in rank)
    const unsigned long long* ridx;// [n + 1] exclusive scan of flags
    uint2* E;                      // [n] kept edges, compacted in input order
    uint32_t* err;                 // set when the relation is not symmetric and simple
    unsigned long long* total;
    const uint32_t* deg;           // dense ids: [vdom] degree of each vertex (else unused)
    uint32_t vdom;
};
MJ_KERNEL_DECL(k_orient_flags, OrientArgs);
MJ_KERNEL_DECL(k_orient_flags_dense, OrientArgs);
MJ_KERNEL_DECL(k_orient_compact, OrientArgs);
struct OrientFinishArgs { OrientArgs o; uint64_t expect; };   // expect: the oriented edges' count
MJ_KERNEL_DECL(k_orient_finish, OrientFinishArgs);
__global__ void k_sym_check(const unsigned long long* K1, const unsigned long long* K2, uint64_t n, uint32_t* bad);

// ------------------------------------------------------------ learned planner
// outputs: 2 cardinalities, MLP_NPLAN plan logits (in mj_algo order:
// three-way, cascade, star, star cascade, oriented, S-largest), 3 share logits
constexpr int MLP_NPLAN = 6, MLP_PLAN0 = 2, MLP_SHARE0 = MLP_PLAN0 + MLP_NPLAN;
constexpr int MLP_IN = 100, MLP_H = 64, MLP_OUT = MLP_SHARE0 + 3;
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_OUT * MLP_H;
constexpr int MLP_P = MLP_OFF_B3 + MLP_OUT;
constexpr int MLP_WB_W1 = 0;
constexpr int MLP_WB_W2 = MLP_WB_W1 + MLP_H * MLP_IN;
constexpr int MLP_WB_W3 = MLP_WB_W2 + MLP_H * MLP_H;
constexpr int MLP_WB = MLP_WB_W3 + MLP_OUT * MLP_H;
constexpr int MLP_ACT = 4 * MLP_H;        // z1, a1, z2, a2 per sample
constexpr int MLP_SPB = 32;               // samples per backward block

struct MlpFwdArgs {
    const float* params;                  // fp32 masters (biases read here)
    const uint16_t* wbf16;
    const float* X;                       // [B][MLP_IN]
    float* Y;                             // [B][MLP_OUT]
    float* act;                           // [B][MLP_ACT] or null
};
struct MlpLossArgs {
    const float* Y;
    float* dY;
    const float* targets;                 // [B][2]
    const int* plan_label;                // [B]
    const int* share_label;               // [B], -1 = none
    uint32_t B;
    float* loss;                          // += mean loss
};
struct MlpBwdArgs {
    const uint16_t* wbf16;
    const float* X;
    const float* act;
    const float* dY;
    uint32_t B;
    float* grad;                          // [MLP_P]
};
struct MlpAdamArgs {
    float* buf;                           // master | grad | m | v
    uint16_t* wbf16;
    float lr, wd, beta1, beta2, eps, bc1, bc2;
};
__global__ void k_mlp_fwd(MlpFwdArgs A);
__global__ void k_mlp_loss(MlpLossArgs A);
__global__ void k_mlp_bwd(MlpBwdArgs A);
__global__ void k_mlp_adamw(MlpAdamArgs A);
__global__ void k_mlp_sync(float* buf, uint16_t* wbf16);
__global__ void k_deg_hist(const DirEntry* dir, const uint2* pool, uint32_t nbkt, uint32_t* hist);
__global__ void k_sketch_features(const uint32_t* hist3, uint64_t nr, uint64_t ns, uint64_t nt,
                                  int kind, float* f);

// max of a column (key-range check)
__global__ void k_col_max(const uint32_t* col, int64_t stride, uint64_t n, uint32_t* out);
struct FillU64Args { unsigned long long* p; uint64_t n; unsigned long long v; };   // p[0..n) = v
struct FillU32Args { uint32_t* p; uint64_t n; uint32_t v; };
MJ_KERNEL_DECL(k_fill_u64, FillU64Args);
MJ_KERNEL_DECL(k_fill_u32, FillU32Args);
struct CopyU64Args { unsigned long long* dst; const unsigned long long* src; uint64_t n; };   // dst[0..n) = src[0..n)
MJ_KERNEL_DECL(k_copy_u64, CopyU64Args);

}  // namespace mj
