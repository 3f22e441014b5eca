// Kernel launch descriptors and kernel declarations of libmj (internal).
#pragma once
#include "mj_device.h"

namespace mj {

// ---------------------------------------------------------------- partition
constexpr int PART_THREADS = 256;
constexpr int PART_TILE = 4096;          // tuples per block
constexpr int MJ_PART_MAX_JOBS = 4;
constexpr uint32_t PART_MAX_BITS = 12;   // at most 4096 buckets per pass

struct PartJob {
    const uint32_t* col0;
    const uint32_t* col1;
    int64_t stride;
    uint64_t n;
    uint32_t key0_col;   // column (0/1) hashed for the first digit
    uint32_t key1_col;   // column hashed for the second digit (bits1 > 0)
    uint32_t seed0, bits0;
    uint32_t seed1, bits1;
    uint32_t* counts;    // [nb] zeroed before the hist pass
    uint32_t* starts;    // [nb + 1]
    uint32_t* cursor;    // [nb]
    uint2* out_pair;     // both columns as (col0, col1), or
    uint32_t* out_single;// one column (single_col) when out_pair == nullptr
    uint32_t single_col;
    uint32_t tile_begin; // first block of this job in the grid
    uint32_t ntiles;
};

struct PartLaunch {
    PartJob job[MJ_PART_MAX_JOBS];
    int njobs;
};

__global__ void k_part_hist(PartLaunch L);
__global__ void k_part_scan(PartLaunch L);
__global__ void k_part_scatter(PartLaunch L);
size_t part_scatter_smem(uint32_t max_bits);

// ------------------------------------------------- multiplicity tables (D)
// Per bucket j an open-addressing table of (key, multiplicity) pairs lives
// in a pool; dir[j] locates it.  Key 0xFFFFFFFF is kept in `special`.
struct DirEntry {
    unsigned long long offset;   // first slot in the pool
    uint32_t log2cap;
    uint32_t special;            // multiplicity of key 0xFFFFFFFF in this bucket
};

constexpr int DB_THREADS = 256;
constexpr uint32_t DB_CAP = 8192;                  // LDS slots per build
constexpr uint32_t DB_LIMIT = DB_CAP - DB_CAP / 8; // distinct keys before spilling
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
};
__global__ void k_dbuild(DBuildArgs A);

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

// --------------------------------------------------------- linear cells
constexpr int CELL_THREADS = 256;
constexpr uint32_t CELL_CAP = 4096;                      // W-table slots (LDS)
constexpr uint32_t CELL_LIMIT = CELL_CAP - CELL_CAP / 8;

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

// max of a column (key-range check)
__global__ void k_col_max(const uint32_t* col, int64_t stride, uint64_t n, uint32_t* out);
__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v);
__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v);

}  // namespace mj
