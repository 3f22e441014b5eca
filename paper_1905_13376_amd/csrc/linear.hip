// Linear three-way join R(A,B) |x| S(B,C) |x| T(C,D) with per-A COUNT
// (Sec. 4, Algorithm 1 and its steps 1-4; Example 1).
//
// Mapping onto MI355X:
//  * the "chip" of the paper is the whole GPU and a "PMU" is one CU's LDS;
//    R is not split at the top level (H = 1) as long as the b-buckets of R
//    and S fit the LDS of the workgroups that own them (h = nb buckets);
//  * T is partitioned by g(C) (nc buckets).  Each bucket T_j is reduced once
//    to a table of C -> multiplicity (its D column takes no part in a COUNT)
//    and that compact table is what every workgroup "receives" when the paper
//    broadcasts T_j to all PMUs: the tables stay L2/MALL resident and every
//    cell reads them in place (k_dbuild);
//  * a cell is one b-bucket: its workgroup keeps, in LDS, the per-B state
//    W[b] = sum over s(b,c) in S_i of mult_T(c) for all of S_i -- the
//    per-R_i-tuple state of Sec. 4.1's footnote -- and then streams R_i,
//    adding W[r.b] to count[r.a] (k_linear_cell).  When the distinct B values
//    of a bucket do not fit the LDS table the bucket is split again by
//    another hash of B (the paper's sub-partitions), recursively.
#include "mj_kernels.h"

namespace mj {

// ------------------------------------------------------------------ helpers
MJ_KERNEL(k_fill_u64, 256, FillU64Args) {
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n; i += (uint64_t)vg.nblk * blockDim.x)
        A.p[i] = A.v;
}

MJ_KERNEL(k_copy_u64, 256, CopyU64Args) {
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n; i += (uint64_t)vg.nblk * blockDim.x)
        A.dst[i] = A.src[i];
}

MJ_KERNEL(k_fill_u32, 256, FillU32Args) {
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n; i += (uint64_t)vg.nblk * blockDim.x)
        A.p[i] = A.v;
}

__global__ void k_col_max(const uint32_t* col, int64_t stride, uint64_t n, uint32_t* out) {
    uint32_t m = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        m = max(m, ld_col(col, i, stride));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor(m, off, WAVE));
    if (lane_id() == 0) atomicMax(out, m);
}

__device__ __forceinline__ uint32_t next_pow2_u32(uint32_t x) {
    return x <= 1 ? 1u : 1u << (32 - __clz(x - 1));
}

// Insert `key` with count increment into a global open-addressing region
// (claim with CAS on the key word, then add to the count word).
__device__ __forceinline__ void gtab_add(uint2* base, uint32_t mask, uint32_t key,
                                         uint32_t inc, uint32_t slot_seed) {
    uint32_t s = slot_hash(key, slot_seed) & mask;
    uint32_t* kw = reinterpret_cast<uint32_t*>(base);
    while (true) {
        uint32_t old = atomicCAS(&kw[2 * s], EMPTY_KEY, key);
        if (old == EMPTY_KEY || old == key) {
            atomicAdd(&kw[2 * s + 1], inc);
            return;
        }
        s = (s + 1u) & mask;
    }
}

// ------------------------------------------------ multiplicity tables (D)
// count[k] += c in the LDS table; sets *over when the distinct keys reach
// DB_LIMIT (no new key is claimed after the overflow flag -- the bucket is
// then rebuilt in global memory -- so the LDS table never fills).
__device__ __forceinline__ void db_add(uint32_t* tkeys, uint32_t* tvals, uint32_t* distinct, uint32_t* over,
                                       uint32_t k, uint32_t c, uint32_t slot_seed) {
    const uint32_t mask = DB_CAP - 1;
    uint32_t s = slot_hash(k, slot_seed) & mask;
    for (uint32_t step = 0;; ++step) {
        uint32_t cur = tkeys[s];
        if (cur == k) { atomicAdd(&tvals[s], c); break; }
        if (cur == EMPTY_KEY || step >= DB_CAP) {
            if (*(volatile uint32_t*)over || step >= DB_CAP) { *over = 1; break; }
            uint32_t old = atomicCAS(&tkeys[s], EMPTY_KEY, k);
            if (old == EMPTY_KEY) {
                if (atomicAdd(distinct, 1u) + 1 >= DB_LIMIT) *over = 1;
                atomicAdd(&tvals[s], c);
                break;
            }
            if (old == k) { atomicAdd(&tvals[s], c); break; }
        }
        s = (s + 1u) & mask;
    }
}

// The keys of [beg, end) counted into the LDS table, four per thread and
// round (their loads in flight together).
__device__ __forceinline__ void db_count(const uint32_t* keys, uint32_t beg, uint32_t end, uint32_t* tkeys,
                                         uint32_t* tvals, uint32_t* special, uint32_t* distinct, uint32_t* over,
                                         uint32_t slot_seed) {
    for (uint32_t i0 = beg + threadIdx.x; i0 < end; i0 += 4 * blockDim.x) {
        if (*(volatile uint32_t*)over) break;
        uint32_t kk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = i0 + u * blockDim.x;
            kk[u] = i < end ? keys[i] : EMPTY_KEY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i0 + u * blockDim.x >= end) break;
            if (kk[u] == EMPTY_KEY) { atomicAdd(special, 1u); continue; }
            db_add(tkeys, tvals, distinct, over, kk[u], 1u, slot_seed);
        }
    }
}

// One workgroup per bucket: the (key, count) table in LDS, then one table
// per bucket in the pool.  A bucket crowded by heavy keys runs as pieces,
// one workgroup each, and the last piece to finish adds up their tables.
MJ_KERNEL(k_dbuild, DB_THREADS, DBuildArgs) {
    __shared__ uint32_t tkeys[DB_CAP];
    __shared__ uint32_t tvals[DB_CAP];
    __shared__ uint32_t s_special, s_distinct, s_over, s_log2, s_last;
    __shared__ unsigned long long s_base;
    uint32_t j = vg.bid, piece = 0, pcs = 1;
    if (A.split.items) {                                         // uniform over the block
        if (vg.bid >= *A.split.nitems) return;
        const uint32_t it = A.split.items[vg.bid];
        j = it & 0xFFFu;
        piece = it >> 12;
        pcs = split_pieces(A.starts[j + 1] - A.starts[j], A.split.chunk);
    }
    const uint32_t beg = A.starts[j], end = A.starts[j + 1];
    const uint32_t n = end - beg;

    for (uint32_t s = threadIdx.x; s < DB_CAP; s += blockDim.x) { tkeys[s] = EMPTY_KEY; tvals[s] = 0; }
    if (threadIdx.x == 0) { s_special = 0; s_distinct = 0; s_over = 0; }
    __syncthreads();
    if (pcs == 1) {
        db_count(A.keys, beg, end, tkeys, tvals, &s_special, &s_distinct, &s_over, A.slot_seed);
    } else {
        // a piece: its counts to its scratch row (or, when its keys overflow
        // the table, a flag); the last piece to finish builds the bucket
        const uint32_t q0 = beg + (uint32_t)(uint64_t(n) * piece / pcs);
        const uint32_t q1 = beg + (uint32_t)(uint64_t(n) * (piece + 1) / pcs);
        db_count(A.keys, q0, q1, tkeys, tvals, &s_special, &s_distinct, &s_over, A.slot_seed);
        __syncthreads();
        const bool ovf = s_over != 0;
        const uint64_t r = uint64_t(A.split.hrow[j]) + piece;
        if (!ovf) {
            uint2* row = A.rows + r * DB_CAP;
            for (uint32_t s = threadIdx.x; s < DB_CAP; s += blockDim.x) row[s] = make_uint2(tkeys[s], tvals[s]);
            if (threadIdx.x == 0) A.row_special[r] = s_special;
        }
        handoff_release();
        __syncthreads();
        if (threadIdx.x == 0) {
            if (ovf) atomicOr(&A.split.done[j], 0x80000000u);
            const uint32_t old = atomicAdd(&A.split.done[j], 1u);
            s_last = (old & 0x7FFFFFFFu) == pcs - 1 ? 1u : 0u;
        }
        __syncthreads();
        if (!s_last) return;                                     // uniform over the block
        handoff_acquire();
        const bool merged = (atomicAdd(&A.split.done[j], 0u) & 0x80000000u) == 0;
        for (uint32_t s = threadIdx.x; s < DB_CAP; s += blockDim.x) { tkeys[s] = EMPTY_KEY; tvals[s] = 0; }
        __syncthreads();
        if (threadIdx.x == 0) { s_special = 0; s_distinct = 0; s_over = merged ? 0u : 1u; }
        __syncthreads();
        if (merged) {                     // the pieces' tables added up (an overflow here spills too)
            const uint2* first = A.rows + uint64_t(A.split.hrow[j]) * DB_CAP;
            for (uint32_t p = 0; p < pcs; ++p)
                for (uint32_t s = threadIdx.x; s < DB_CAP; s += blockDim.x) {
                    if (*(volatile uint32_t*)&s_over) break;
                    const uint2 e = first[uint64_t(p) * DB_CAP + s];
                    if (e.x != EMPTY_KEY && e.y) db_add(tkeys, tvals, &s_distinct, &s_over, e.x, e.y, A.slot_seed);
                }
            if (threadIdx.x == 0) {
                uint32_t sp = 0;
                for (uint32_t p = 0; p < pcs; ++p) sp += A.row_special[A.split.hrow[j] + p];
                s_special = sp;
            }
        }
    }
    __syncthreads();
    const bool spill = s_over != 0;
    // a table of at most DB_CAP / 2 keys is rehashed in LDS at its final
    // capacity and written out whole; larger ones are inserted key by key
    const bool local = !spill && 2u * s_distinct <= DB_CAP;
    if (threadIdx.x == 0) {
        const uint32_t want = spill ? (n > (1u << 30) ? (1u << 31) : 2u * n) : 2u * s_distinct;
        uint32_t cap = max(DB_MIN_CAP, next_pow2_u32(want));
        unsigned long long base = atomicAdd(A.pool_cursor, (unsigned long long)cap);
        if (base + cap > A.pool_cap) {       // cannot happen with a planned workspace
            atomicExch(A.err, 1u);
            base = 0;                        // the pool's first DB_MIN_CAP slots stay empty
            cap = DB_MIN_CAP;
        }
        s_base = base;
        s_log2 = 31 - __clz(cap);
        if (spill) s_special = 0;            // recounted below
    }
    __syncthreads();
    const unsigned long long base = s_base;
    const uint32_t cap = 1u << s_log2;
    uint2* region = A.pool + base;
    if (base != 0 && local) {
        // take the entries out, clear, reinsert with mask cap - 1 (the
        // lookup's probe sequence), then copy slots [0, cap) out coalesced
        constexpr int PER = DB_CAP / DB_THREADS;
        uint32_t ek[PER], ev[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t s = threadIdx.x + u * DB_THREADS;
            ek[u] = tkeys[s];
            ev[u] = tvals[s];
        }
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < cap; s += blockDim.x) { tkeys[s] = EMPTY_KEY; tvals[s] = 0; }
        __syncthreads();
        const uint32_t cmask = cap - 1;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            if (ek[u] == EMPTY_KEY) continue;
            uint32_t s = slot_hash(ek[u], A.slot_seed) & cmask;
            while (atomicCAS(&tkeys[s], EMPTY_KEY, ek[u]) != EMPTY_KEY) s = (s + 1u) & cmask;
            tvals[s] = ev[u];
        }
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < cap; s += blockDim.x) region[s] = make_uint2(tkeys[s], tvals[s]);
    } else if (base != 0) {
        for (uint32_t s = threadIdx.x; s < cap; s += blockDim.x) region[s] = make_uint2(EMPTY_KEY, 0u);
        __threadfence();
        __syncthreads();
        if (!spill) {
            for (uint32_t s = threadIdx.x; s < DB_CAP; s += blockDim.x) {
                uint32_t k = tkeys[s];
                if (k != EMPTY_KEY) gtab_add(region, cap - 1, k, tvals[s], A.slot_seed);
            }
        } else {
            for (uint32_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
                const uint32_t k = A.keys[i];
                if (k == EMPTY_KEY) atomicAdd(&s_special, 1u);
                else gtab_add(region, cap - 1, k, 1u, A.slot_seed);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        DirEntry e;
        e.offset = base;
        e.log2cap = s_log2;
        e.special = s_special;
        A.dir[j] = e;
    }
}

// --------------------------------------------------------------- probe-sum
__global__ void k_probe_sum(ProbeSumArgs A) {
    unsigned long long acc = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t k = ld_col(A.col, i, A.stride);
        acc += dtab_lookup(A.dir, A.pool, k, A.bkt_seed, A.bkt_bits, A.slot_seed);
    }
    acc = wave_sum_u64(acc);
    if (lane_id() == 0 && acc) atomicAdd(A.total, acc);
}

// ------------------------------------------------------------ linear cells
__device__ __forceinline__ uint32_t pass_of(uint32_t b, uint32_t seed, uint32_t level) {
    return top_bits(mix32(b, seed ^ 0x3C6EF372u), level);
}

// A cell's LDS table of W[b] (key 0xFFFFFFFF kept in `special`).
struct WTable {
    uint32_t* keys;
    unsigned long long* vals;
    unsigned long long* special;
    uint32_t* distinct;
    uint32_t* over;
};

// W[b] += v in the LDS table; sets *over when the distinct b exceed
// CELL_LIMIT (no slot is claimed after that, so every probe still ends).
__device__ __forceinline__ void w_table_add(const WTable& T, uint32_t b, unsigned long long v, uint32_t w_seed) {
    const uint32_t mask = CELL_CAP - 1;
    uint32_t s = slot_hash(b, w_seed) & mask;
    for (uint32_t step = 0;; ++step) {
        uint32_t cur = T.keys[s];
        if (cur == b) { atomicAdd(&T.vals[s], v); break; }
        if (cur == EMPTY_KEY || step >= CELL_CAP) {
            // a new key: once the pass has overflowed no new slot is
            // claimed (the pass is redone split), so the table can
            // never fill up and every probe finds an empty slot
            if (*(volatile uint32_t*)T.over || step >= CELL_CAP) { *T.over = 1; break; }
            uint32_t old = atomicCAS(&T.keys[s], EMPTY_KEY, b);
            if (old == EMPTY_KEY || old == b) {
                if (old == EMPTY_KEY && atomicAdd(T.distinct, 1u) + 1 >= CELL_LIMIT) *T.over = 1;
                atomicAdd(&T.vals[s], v);
                break;
            }
        }
        s = (s + 1u) & mask;
    }
}

// W[b] += mult_T(c) over the S tuples of [s0, s1) whose b belongs to the
// pass (level, pass); sets *over when the distinct b exceed CELL_LIMIT (no
// slot is claimed after that, so every probe still ends).
__device__ void w_accumulate(const uint2* S, uint32_t s0, uint32_t s1, const DirEntry* ddir,
                             const uint2* dpool, uint32_t c_seed, uint32_t c_bits,
                             uint32_t slot_seed, uint32_t w_seed, uint32_t level, uint32_t pass,
                             const WTable& T) {
    const int nthr = blockDim.x;
    for (uint32_t q = s0 + threadIdx.x; q < s1; q += 4 * nthr) {
        if (*(volatile uint32_t*)T.over) break;
        uint2 sv[4];
        uint32_t w[4], cc[4];
        bool live[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uint32_t idx = q + u * nthr;
            sv[u] = idx < s1 ? S[idx] : make_uint2(0u, 0u);
            live[u] = idx < s1 && (level == 0 || pass_of(sv[u].x, w_seed, level) == pass);
            cc[u] = sv[u].y;
        }
        dtab_lookup4(ddir, dpool, cc, live, c_seed, c_bits, slot_seed, w);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const unsigned long long v = w[u];
            if (v == 0) continue;
            const uint32_t b = sv[u].x;
            if (b == EMPTY_KEY) { atomicAdd(T.special, v); continue; }
            w_table_add(T, b, v, w_seed);
        }
    }
}

// The pieces' W tables of a split bucket added into the LDS table (and
// their sums for b = 0xFFFFFFFF into T.special); sets *over as above.
__device__ void w_merge_rows(const WSlot* rows, const unsigned long long* rspecial, uint32_t pcs,
                             uint32_t w_seed, const WTable& T) {
    for (uint32_t r = 0; r < pcs; ++r) {
        const WSlot* row = rows + uint64_t(r) * CELL_CAP;
        for (uint32_t t = threadIdx.x; t < CELL_CAP; t += blockDim.x) {
            if (*(volatile uint32_t*)T.over) break;
            const WSlot e = row[t];
            if (e.key != EMPTY_KEY && e.w) w_table_add(T, e.key, e.w, w_seed);
        }
    }
    if (threadIdx.x == 0) {
        unsigned long long sp = 0;
        for (uint32_t r = 0; r < pcs; ++r) sp += rspecial[r];
        if (sp) atomicAdd(T.special, sp);
    }
}

__device__ void linear_cell_run(const LinearCellArgs& A, uint32_t i) {
    __shared__ uint32_t wkeys[CELL_CAP];
    __shared__ unsigned long long wvals[CELL_CAP];
    __shared__ unsigned long long w_special;
    __shared__ uint32_t s_distinct, s_over;
    __shared__ uint32_t st_level[64], st_pass[64];
    __shared__ int s_sp;
    const WTable T{wkeys, wvals, &w_special, &s_distinct, &s_over};

    const uint32_t s0 = A.sstarts[i], s1 = A.sstarts[i + 1];
    const uint32_t r0 = A.rstarts[i], r1 = A.rstarts[i + 1];
    if (s0 == s1 || r0 == r1) return;      // nothing can match in this cell
    const uint32_t mask = CELL_CAP - 1;
    const int nthr = blockDim.x;

    if (threadIdx.x == 0) { s_sp = 1; st_level[0] = 0; st_pass[0] = 0; }
    while (true) {
        // every wave reads the top of the pass stack before thread 0 pops it
        __syncthreads();
        const int sp = s_sp;
        if (sp == 0) break;
        const uint32_t level = st_level[sp - 1];
        const uint32_t pass = st_pass[sp - 1];
        for (uint32_t s = threadIdx.x; s < CELL_CAP; s += nthr) { wkeys[s] = EMPTY_KEY; wvals[s] = 0; }
        __syncthreads();
        if (threadIdx.x == 0) { w_special = 0; s_distinct = 0; s_over = 0; s_sp = sp - 1; }
        __syncthreads();

        // phase 1: W[b] += mult_T(c) over the S tuples of this (sub-)bucket
        w_accumulate(A.S, s0, s1, A.ddir, A.dpool, A.c_seed, A.c_bits, A.slot_seed, A.w_seed,
                     level, pass, T);
        __syncthreads();
        if (s_over) {
            // too many distinct B values: split this pass in two by one more
            // hash bit (the barrier at the loop head orders the push)
            if (threadIdx.x == 0) {
                st_level[sp - 1] = level + 1; st_pass[sp - 1] = 2 * pass + 1;
                st_level[sp] = level + 1;     st_pass[sp] = 2 * pass;
                s_sp = sp + 1;
            }
            continue;
        }
        // phase 2: count[r.a] += W[r.b] over the R tuples of this (sub-)bucket
        for (uint32_t q = r0 + threadIdx.x; q < r1; q += nthr) {
            const uint2 rv = A.R[q];
            const uint32_t b = rv.y;
            if (level && pass_of(b, A.w_seed, level) != pass) continue;
            unsigned long long w = 0;
            if (b == EMPTY_KEY) {
                w = w_special;
            } else {
                uint32_t s = slot_hash(b, A.w_seed) & mask;
                while (true) {
                    uint32_t cur = wkeys[s];
                    if (cur == b) { w = wvals[s]; break; }
                    if (cur == EMPTY_KEY) break;
                    s = (s + 1u) & mask;
                }
            }
            if (w) {
                if (rv.x < A.a_domain) atomicAdd(&A.count[rv.x], w);
                else atomicExch(A.err, 1u);     // key outside [0, a_domain): reported, not written
            }
        }
    }
}

__global__ void __launch_bounds__(CELL_THREADS)
k_linear_cell(LinearCellArgs A) {
    linear_cell_run(A, blockIdx.x);
}

// All cells of all linear joins of a batch in one launch: block b is cell
// b - cell_base[j] of the join j with cell_base[j] <= b < cell_base[j + 1].
__global__ void __launch_bounds__(CELL_THREADS)
k_linear_cell_batch(LinearBatchArgs B) {
    const uint32_t b = blockIdx.x;
    uint32_t lo = 0, hi = B.njoins;
    while (hi - lo > 1) { uint32_t m = (lo + hi) >> 1; if (B.cell_base[m] <= b) lo = m; else hi = m; }
    linear_cell_run(B.joins[lo], b - B.cell_base[lo]);
}

// ------------------------------------------------------------- W tables
// One workgroup per b-bucket: W[b] for the bucket's S tuples in LDS (split
// into passes by hash bits of b while the distinct b overflow the table, as
// in the cells), then one table per bucket in the pool.  A bucket done in
// one pass is copied out whole (rehashed in LDS first at the least power of
// two >= twice its keys when that is below CELL_CAP); a split bucket gets a
// region sized for every S tuple of the bucket, cleared, into which each
// pass inserts its keys (every key belongs to one pass, so a claimed slot's
// W is stored once).  A bucket crowded by heavy keys runs as pieces, one
// workgroup each, and the last piece to finish adds up their tables.
__global__ void __launch_bounds__(CELL_THREADS)
k_wbuild(WBuildArgs A) {
    __shared__ uint32_t wkeys[CELL_CAP];
    __shared__ unsigned long long wvals[CELL_CAP];
    __shared__ unsigned long long w_special, s_special_tot, s_base;
    __shared__ uint32_t s_distinct, s_over, s_log2, s_global;
    __shared__ uint32_t st_level[64], st_pass[64];
    __shared__ int s_sp;
    __shared__ uint32_t s_last;
    const WTable T{wkeys, wvals, &w_special, &s_distinct, &s_over};
    // the block's work item: a bucket, or a piece of a split bucket (heavy
    // keys; listed first so that they start first)
    uint32_t i = blockIdx.x, piece = 0, pcs = 1;
    if (A.split.items) {                                         // uniform over the block
        if (blockIdx.x >= *A.split.nitems) return;
        const uint32_t it = A.split.items[blockIdx.x];
        i = it & 0xFFFu;
        piece = it >> 12;
        pcs = split_pieces(A.sstarts[i + 1] - A.sstarts[i], A.split.chunk);
    }
    const uint32_t s0 = A.sstarts[i], s1 = A.sstarts[i + 1];
    const int nthr = blockDim.x;
    bool merged = false;
    if (pcs > 1) {
        // a piece: its W table in LDS, written to its scratch row (or, when
        // its keys overflow the table, a flag that sends the bucket back to
        // its tuples); the last piece to finish builds the bucket's table
        const uint32_t len = s1 - s0;
        const uint32_t q0 = s0 + (uint32_t)(uint64_t(len) * piece / pcs);
        const uint32_t q1 = s0 + (uint32_t)(uint64_t(len) * (piece + 1) / pcs);
        for (uint32_t s = threadIdx.x; s < CELL_CAP; s += nthr) { wkeys[s] = EMPTY_KEY; wvals[s] = 0; }
        if (threadIdx.x == 0) { w_special = 0; s_distinct = 0; s_over = 0; }
        __syncthreads();
        w_accumulate(A.S, q0, q1, A.ddir, A.dpool, A.c_seed, A.c_bits, A.slot_seed, A.w_seed, 0, 0, T);
        __syncthreads();
        const bool ovf = s_over != 0;
        const uint64_t r = uint64_t(A.split.hrow[i]) + piece;
        if (!ovf) {
            WSlot* row = A.rows + r * CELL_CAP;
            for (uint32_t s = threadIdx.x; s < CELL_CAP; s += nthr) {
                WSlot v;
                v.key = wkeys[s]; v.pad = 0; v.w = wvals[s];
                row[s] = v;
            }
            if (threadIdx.x == 0) A.row_special[r] = w_special;
        }
        handoff_release();
        __syncthreads();
        if (threadIdx.x == 0) {
            if (ovf) atomicOr(&A.split.done[i], 0x80000000u);
            const uint32_t old = atomicAdd(&A.split.done[i], 1u);
            s_last = (old & 0x7FFFFFFFu) == pcs - 1 ? 1u : 0u;
        }
        __syncthreads();
        if (!s_last) return;                                     // uniform over the block
        handoff_acquire();
        merged = (atomicAdd(&A.split.done[i], 0u) & 0x80000000u) == 0;
        __syncthreads();
    }
    if (s0 == s1) {                       // an empty table: the pool's first slots
        if (threadIdx.x == 0) {
            WDirEntry e;
            e.offset = 0; e.special = 0; e.log2cap = 31 - __clz(W_MIN_CAP); e.pad = 0;
            A.wdir[i] = e;
        }
        return;
    }
    if (threadIdx.x == 0) {
        s_sp = 1; st_level[0] = 0; st_pass[0] = 0;
        s_global = 0; s_base = 0; s_log2 = 31 - __clz(W_MIN_CAP); s_special_tot = 0;
    }
    // a split bucket whose pieces all fit their tables: the first pass adds
    // up the pieces' tables instead of reading the tuples
    while (true) {
        __syncthreads();
        const int sp = s_sp;
        if (sp == 0) break;
        const uint32_t level = st_level[sp - 1];
        const uint32_t pass = st_pass[sp - 1];
        for (uint32_t s = threadIdx.x; s < CELL_CAP; s += nthr) { wkeys[s] = EMPTY_KEY; wvals[s] = 0; }
        __syncthreads();
        if (threadIdx.x == 0) { w_special = 0; s_distinct = 0; s_over = 0; s_sp = sp - 1; }
        __syncthreads();
        if (merged) {
            const uint64_t r0 = A.split.hrow[i];
            w_merge_rows(A.rows + r0 * CELL_CAP, A.row_special + r0, pcs, A.w_seed, T);
            __syncthreads();
            if (s_over) {                    // the union overflows: redo this pass from the tuples
                merged = false;
                if (threadIdx.x == 0) s_sp = sp;
                continue;
            }
        } else {
            w_accumulate(A.S, s0, s1, A.ddir, A.dpool, A.c_seed, A.c_bits, A.slot_seed, A.w_seed,
                         level, pass, T);
        }
        __syncthreads();
        if (s_over) {
            if (threadIdx.x == 0) {
                st_level[sp - 1] = level + 1; st_pass[sp - 1] = 2 * pass + 1;
                st_level[sp] = level + 1;     st_pass[sp] = 2 * pass;
                s_sp = sp + 1;
            }
            continue;
        }
        if (threadIdx.x == 0) s_special_tot += w_special;
        const bool whole = level == 0;       // the bucket's table is complete in LDS
        const bool need_region = !whole && !s_global;
        __syncthreads();
        if (whole || need_region) {
            if (threadIdx.x == 0) {
                // a whole table keeps load <= 1/2 when it can be halved, else
                // it leaves LDS as it is (CELL_CAP slots, load < 7/8)
                const uint64_t want = whole ? min<uint64_t>(2ull * s_distinct, CELL_CAP) : 2ull * (s1 - s0);
                uint32_t cap = max(W_MIN_CAP, (uint32_t)min<uint64_t>(uint64_t(1) << 31,
                                                                      next_pow2_u32((uint32_t)min<uint64_t>(want, 1ull << 31))));
                unsigned long long base = atomicAdd(A.wcursor, (unsigned long long)cap);
                if (base + cap > A.wcap) {   // cannot happen with a planned workspace
                    atomicExch(A.err, 1u);
                    base = 0;                // the pool's first W_MIN_CAP slots stay empty
                    cap = W_MIN_CAP;
                }
                s_base = base;
                s_log2 = 31 - __clz(cap);
                s_global = 1;
            }
            __syncthreads();
        }
        const unsigned long long base = s_base;
        const uint32_t cap = 1u << s_log2;
        WSlot* region = A.wpool + base;
        if (base == 0) continue;             // pool exhausted: reported above
        if (whole && cap < CELL_CAP) {
            // rehash in place at mask cap - 1, then copy slots [0, cap) out
            constexpr int PER = CELL_CAP / CELL_THREADS;
            uint32_t ek[PER];
            unsigned long long ev[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t s = threadIdx.x + u * CELL_THREADS;
                ek[u] = wkeys[s];
                ev[u] = wvals[s];
            }
            __syncthreads();
            for (uint32_t s = threadIdx.x; s < cap; s += nthr) { wkeys[s] = EMPTY_KEY; wvals[s] = 0; }
            __syncthreads();
            const uint32_t cmask = cap - 1;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                if (ek[u] == EMPTY_KEY) continue;
                uint32_t s = slot_hash(ek[u], A.w_seed) & cmask;
                while (atomicCAS(&wkeys[s], EMPTY_KEY, ek[u]) != EMPTY_KEY) s = (s + 1u) & cmask;
                wvals[s] = ev[u];
            }
            __syncthreads();
            for (uint32_t s = threadIdx.x; s < cap; s += nthr) {
                WSlot v;
                v.key = wkeys[s]; v.pad = 0; v.w = wvals[s];
                region[s] = v;
            }
        } else if (whole) {                  // same mask: the LDS table as it is
            for (uint32_t s = threadIdx.x; s < CELL_CAP; s += nthr) {
                WSlot v;
                v.key = wkeys[s]; v.pad = 0; v.w = wvals[s];
                region[s] = v;
            }
        } else {
            if (need_region) {
                for (uint32_t s = threadIdx.x; s < cap; s += nthr) {
                    WSlot v;
                    v.key = EMPTY_KEY; v.pad = 0; v.w = 0;
                    region[s] = v;
                }
                __threadfence();
                __syncthreads();
            }
            const uint32_t cmask = cap - 1;
            for (uint32_t t = threadIdx.x; t < CELL_CAP; t += nthr) {
                const uint32_t k = wkeys[t];
                if (k == EMPTY_KEY) continue;
                uint32_t s = slot_hash(k, A.w_seed) & cmask;
                while (atomicCAS(&region[s].key, EMPTY_KEY, k) != EMPTY_KEY) s = (s + 1u) & cmask;
                region[s].w = wvals[t];
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        WDirEntry e;
        e.offset = s_base; e.special = s_special_tot; e.log2cap = s_log2; e.pad = 0;
        A.wdir[i] = e;
    }
}

// The rest of a W-table probe whose first slot `s` has been read as `v`
// (scalar arguments, so that four probes in flight stay in registers).
__device__ __forceinline__ unsigned long long wprobe_from(const WSlot* __restrict__ base, uint32_t mask,
                                                          uint32_t key, WSlot v, uint32_t s) {
    while (v.key != key && v.key != EMPTY_KEY) {
        s = (s + 1u) & mask;
        v = base[s];
    }
    return v.key == key ? v.w : 0ull;
}

// Four independent W lookups (directory loads, then first slots, in flight
// together; only keys that collide walk further); 0 when absent.
__device__ __forceinline__ void wtab_lookup4(const WDirEntry* __restrict__ dir,
                                             const WSlot* __restrict__ pool,
                                             const uint32_t (&key)[4], const bool (&live)[4],
                                             uint32_t bkt_seed, uint32_t bkt_bits,
                                             uint32_t slot_seed, unsigned long long (&out)[4]) {
    WDirEntry e[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (live[u]) e[u] = dir[top_bits(mix32(key[u], bkt_seed), bkt_bits)];
    uint32_t s[4];
    WSlot kv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (live[u] && key[u] != EMPTY_KEY) {
            s[u] = slot_hash(key[u], slot_seed) & ((1u << e[u].log2cap) - 1u);
            kv[u] = pool[e[u].offset + s[u]];
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (!live[u]) { out[u] = 0; continue; }
        if (key[u] == EMPTY_KEY) { out[u] = e[u].special; continue; }
        out[u] = wprobe_from(pool + e[u].offset, (1u << e[u].log2cap) - 1u, key[u], kv[u], s[u]);
    }
}

// A piece of a split bucket: its sums acc[0, span) go to its scratch row;
// the last piece of the bucket to finish returns true with the bucket's
// totals in acc (the other pieces return false).
template <class TO>
__device__ __forceinline__ bool split_merge(const BucketItems& B, uint32_t k, uint32_t piece, uint32_t pcs,
                                            TO* rows, uint32_t row_len, TO* acc, uint32_t span) {
    __shared__ uint32_t s_last;
    TO* mine = rows + (uint64_t(B.hrow[k]) + piece) * row_len;
    for (uint32_t j = threadIdx.x; j < span; j += blockDim.x) mine[j] = acc[j];
    handoff_release();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&B.done[k], 1u) == pcs - 1 ? 1u : 0u;
    __syncthreads();
    if (!s_last) return false;                                      // uniform over the block
    handoff_acquire();
    const TO* first = rows + uint64_t(B.hrow[k]) * row_len;
    for (uint32_t j = threadIdx.x; j < span; j += blockDim.x) {
        TO v = 0;
        for (uint32_t r = 0; r < pcs; ++r) v += *(const volatile TO*)&first[uint64_t(r) * row_len + j];
        acc[j] = v;
    }
    if (threadIdx.x == 0) B.done[k] = 0;                            // for the next kernel over these items
    __syncthreads();
    return true;
}

// ------------------------------------------------------------- counts
// One workgroup per range of A values: count[a] = sum over r(a, b) of W[b]
// in LDS, then the range is written out whole (zeros included).
__global__ void __launch_bounds__(COUNT_THREADS)
k_count(CountArgs A) {
    extern __shared__ unsigned long long cnt[];          // [1 << a_shift]
    uint32_t k = blockIdx.x, piece = 0;
    if (A.split.items) {                                  // uniform over the block
        if (blockIdx.x >= *A.split.nitems) return;
        const uint32_t it = A.split.items[blockIdx.x];
        k = it & 0xFFFu;
        piece = it >> 12;
    }
    const uint64_t base = uint64_t(k) << A.a_shift;
    // ranges past a_domain only receive keys out of range (reported)
    const uint32_t span = base < A.a_domain
                              ? (uint32_t)min<uint64_t>(uint64_t(1) << A.a_shift, A.a_domain - base) : 0u;
    const int nthr = blockDim.x;
    for (uint32_t j = threadIdx.x; j < span; j += nthr) cnt[j] = 0;
    __syncthreads();
    const uint32_t s0 = A.rstarts[k], len = A.rstarts[k + 1] - s0;
    const uint32_t pcs = A.split.items ? split_pieces(len, A.split.chunk) : 1u;
    const uint32_t r0 = s0 + (uint32_t)(uint64_t(len) * piece / pcs);
    const uint32_t r1 = s0 + (uint32_t)(uint64_t(len) * (piece + 1) / pcs);
    const bool heavy = pcs > 1;                           // equal A values of a wave folded first
    for (uint32_t qb = r0; qb < r1; qb += 4 * nthr) {     // every lane runs every round
        const uint32_t q = qb + threadIdx.x;
        uint2 rv[4];
        uint32_t bb[4];
        bool live[4];
        unsigned long long w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t idx = q + u * nthr;
            live[u] = idx < r1;
            rv[u] = live[u] ? A.R[idx] : make_uint2(0u, 0u);
            bb[u] = rv[u].y;
        }
        wtab_lookup4(A.wdir, A.wpool, bb, live, A.b_seed, A.b_bits, A.w_seed, w);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            unsigned long long v = w[u];
            bool act = live[u] && v != 0;
            if (heavy && wave_fold_first(rv[u].x, act, v)) act = false;
            if (!act) continue;
            const uint64_t off = uint64_t(rv[u].x) - base;   // < span unless a >= a_domain
            if (rv[u].x >= A.a_domain || off >= span) { atomicExch(A.err, 1u); continue; }
            atomicAdd(&cnt[off], v);
        }
    }
    __syncthreads();
    if (pcs > 1 && !split_merge(A.split, k, piece, pcs, A.rows, 1u << A.a_shift, cnt, span)) return;
    for (uint32_t j = threadIdx.x; j < span; j += nthr) A.count[base + j] = cnt[j];
}

// ------------------------------------------------- direct-indexed tables
// When every B and C value is below a small bound the planner has found,
// T's multiplicities and the per-B sums W are arrays indexed by the key: the
// same partition-then-accumulate structure with the identity as hash.  Each
// workgroup owns one range of keys (the relation partitioned by range), sums
// its weights in LDS and writes the range once; the weight of a tuple is one
// read of the previous array.
// SAT_IN: table_narrow is a saturating copy; SAT_OUT: out_narrow is one.
template <bool SAT_IN, bool SAT_OUT, class TW, class TWN, class TO, class TON>
__device__ __forceinline__ void range_accumulate(const RangeAccArgs<TW, TWN, TO, TON>& A, TO* acc, VGrid vg) {
    uint32_t k = vg.bid, piece = 0;
    if (A.split.items) {                                            // uniform over the block
        if (vg.bid >= *A.split.nitems) return;
        const uint32_t it = A.split.items[vg.bid];
        k = it & 0xFFFu;
        piece = it >> 12;
    }
    const uint64_t base = uint64_t(k) << A.shift;
    const uint32_t span = base < A.domain ? (uint32_t)min<uint64_t>(uint64_t(1) << A.shift, A.domain - base) : 0u;
    const int nthr = blockDim.x;
    for (uint32_t j = threadIdx.x; j < span; j += nthr) acc[j] = 0;
    __syncthreads();
    bool narrow = false;                                            // uniform over the launch
    if constexpr (!SAT_IN) narrow = A.table_narrow && *A.use_wide == 0;
    const uint32_t s0 = A.starts[k], len = A.starts[k + 1] - s0;
    const uint32_t pcs = A.split.items ? split_pieces(len, A.split.chunk) : 1u;
    const uint32_t q0 = s0 + (uint32_t)(uint64_t(len) * piece / pcs);
    const uint32_t q1 = s0 + (uint32_t)(uint64_t(len) * (piece + 1) / pcs);
    // a split range is a heavy one: equal keys of a wave are folded first
    const bool heavy = pcs > 1;
    for (uint32_t qb = q0; qb < q1; qb += 4 * nthr) {               // every lane runs every round
        const uint32_t q = qb + threadIdx.x;
        uint32_t key[4];
        TO w[4];
        bool live[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t idx = q + u * nthr;
            live[u] = idx < q1;
            uint32_t v = 0;
            if (A.pairs) {
                const uint2 pv = live[u] ? A.pairs[idx] : make_uint2(0u, 0u);
                key[u] = pv.x;
                v = pv.y;
            } else {
                key[u] = live[u] ? A.keys[idx] : 0u;
            }
            if (A.table) {                                           // the reads in flight together
                const bool in = live[u] && v < A.table_n;
                if constexpr (SAT_IN) {
                    const TWN x = in ? A.table_narrow[v] : TWN(0);
                    w[u] = x == TWN(~TWN(0)) ? (TO)A.table[v] : (TO)x;
                } else {
                    w[u] = !in ? (TO)0 : (narrow ? (TO)A.table_narrow[v] : (TO)A.table[v]);
                }
            } else {
                w[u] = 1;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TO v = w[u];
            bool act = live[u] && v != 0;
            if (heavy && wave_fold_first(key[u], act, v)) act = false;
            if (!act) continue;
            const uint64_t off = uint64_t(key[u]) - base;
            if (key[u] >= A.domain || off >= span) { atomicExch(A.err, 1u); continue; }
            atomicAdd(&acc[off], v);
        }
    }
    __syncthreads();
    if (pcs > 1 && !split_merge(A.split, k, piece, pcs, reinterpret_cast<TO*>(A.rows), A.row_len, acc, span))
        return;                                                     // another piece writes the range
    bool big = false;
    for (uint32_t j = threadIdx.x; j < span; j += nthr) {
        const TO v = acc[j];
        A.out[base + j] = v;
        if (A.out_narrow) {
            constexpr uint64_t top = uint64_t(TON(~TON(0)));
            if constexpr (SAT_OUT) {
                A.out_narrow[base + j] = uint64_t(v) >= top ? TON(~TON(0)) : (TON)v;
            } else {
                A.out_narrow[base + j] = (TON)v;
                big = big || uint64_t(v) > top;
            }
        }
    }
    if (big) atomicOr(A.wide, 1u);
}

MJ_KERNEL(k_range_deg, RANGE_THREADS, RangeDegArgs) {
    extern __shared__ uint32_t acc32[];
    range_accumulate<false, false>(A, acc32, vg);
}

MJ_KERNEL(k_range_w, RANGE_THREADS, RangeWArgs) {
    extern __shared__ unsigned long long acc64w[];
    range_accumulate<false, true>(A, acc64w, vg);
}

MJ_KERNEL(k_range_count, RANGE_THREADS, RangeCountArgs) {
    extern __shared__ unsigned long long acc64c[];
    range_accumulate<true, false>(A, acc64c, vg);
}

MJ_KERNEL(k_check_size, 64, CheckSizeArgs) {
    if (threadIdx.x == 0 && vg.bid == 0 && *A.got != A.want) atomicExch(A.err, 1u);
}

// ------------------------------------------------ S-largest linear join
// Block (i, j, piece): T_j's multiplicities and R_i's B keys in LDS (each
// when it fits, else probed where it lies), the piece of S_ij streamed:
// w = mult_Tj(c); if b is one of R_i's keys its LDS sum grows by w.  At
// the end every nonzero sum is added to R_i's table once.
__global__ void __launch_bounds__(SL_THREADS)
k_sl_cell(SlCellArgs A) {
    __shared__ uint2 ttab[1u << SL_T_LOG2];
    __shared__ uint32_t rkeys[1u << SL_R_LOG2];
    __shared__ unsigned long long racc[1u << SL_R_LOG2];
    // 80 KB in all: two workgroups share a compute unit's LDS
    const uint32_t LT = 1u << A.t_bits;
    const uint32_t cell = blockIdx.x / A.pieces, piece = blockIdx.x % A.pieces;
    const uint32_t i = cell >> A.t_bits, j = cell & (LT - 1u);
    const uint32_t c0 = A.sstarts[cell], c1 = A.sstarts[cell + 1];
    const uint32_t len = c1 - c0;
    const uint32_t q0 = c0 + (uint32_t)((uint64_t)len * piece / A.pieces);
    const uint32_t q1 = c0 + (uint32_t)((uint64_t)len * (piece + 1) / A.pieces);
    if (q0 == q1) return;                                  // uniform over the block
    const int nthr = blockDim.x;
    const DirEntry te = A.tdir[j], re = A.rdir[i];
    const uint32_t tmask = (1u << te.log2cap) - 1u, rmask = (1u << re.log2cap) - 1u;
    const bool tl = te.log2cap <= SL_T_LOG2, rl = re.log2cap <= SL_R_LOG2;
    const uint2* tg = A.tpool + te.offset;
    const uint2* rg = A.rpool + re.offset;
    unsigned long long* wv = A.wval + re.offset;
    if (tl) for (uint32_t t = threadIdx.x; t <= tmask; t += nthr) ttab[t] = tg[t];
    if (rl) for (uint32_t t = threadIdx.x; t <= rmask; t += nthr) { rkeys[t] = rg[t].x; racc[t] = 0; }
    __syncthreads();
    const uint2* tab = tl ? ttab : tg;
    for (uint32_t q = q0 + threadIdx.x; q < q1; q += 4 * nthr) {
        uint2 sv[4], kv[4];
        uint32_t sl[4], w[4];
        bool live[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t idx = q + u * nthr;
            live[u] = idx < q1;
            sv[u] = live[u] ? A.S[idx] : make_uint2(0u, 0u);
            sl[u] = slot_hash(sv[u].y, A.slot_seed) & tmask;
            kv[u] = live[u] && sv[u].y != EMPTY_KEY ? tab[sl[u]] : make_uint2(EMPTY_KEY, 0u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (!live[u]) { w[u] = 0; continue; }
            if (sv[u].y == EMPTY_KEY) { w[u] = te.special; continue; }
            w[u] = probe_from(tab, tmask, sv[u].y, kv[u], sl[u], 0u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (w[u] == 0) continue;
            const uint32_t b = sv[u].x;
            if (b == EMPTY_KEY) {
                // b = 0xFFFFFFFF, kept beside the table (rare: a global add)
                if (re.special) atomicAdd(&A.wspecial[i], (unsigned long long)w[u]);
                continue;
            }
            // b among R_i's keys: its slot (linear probing from the W hash)
            uint32_t s = slot_hash(b, A.w_seed) & rmask;
            while (true) {
                const uint32_t k = rl ? rkeys[s] : rg[s].x;
                if (k == b) {
                    if (rl) atomicAdd(&racc[s], (unsigned long long)w[u]);
                    else atomicAdd(&wv[s], (unsigned long long)w[u]);
                    break;
                }
                if (k == EMPTY_KEY) break;                 // not in R_i: joins nothing
                s = (s + 1u) & rmask;
            }
        }
    }
    __syncthreads();
    if (rl)
        for (uint32_t t = threadIdx.x; t <= rmask; t += nthr)
            if (racc[t]) atomicAdd(&wv[t], racc[t]);
}

// R_i's table with its sums as the W table of bucket i (same slots).
__global__ void k_sl_wtables(const DirEntry* rdir, const uint2* rpool, const unsigned long long* wval,
                             const unsigned long long* wspecial, WDirEntry* wdir, WSlot* wpool) {
    const uint32_t i = blockIdx.x;
    const DirEntry e = rdir[i];
    const uint32_t cap = 1u << e.log2cap;
    for (uint32_t t = threadIdx.x; t < cap; t += blockDim.x) {
        WSlot v;
        v.key = rpool[e.offset + t].x;
        v.pad = 0;
        v.w = wval[e.offset + t];
        wpool[e.offset + t] = v;
    }
    if (threadIdx.x == 0) {
        WDirEntry d;
        d.offset = e.offset; d.special = wspecial[i]; d.log2cap = e.log2cap; d.pad = 0;
        wdir[i] = d;
    }
}

MJ_KERNEL(k_poison_u64, 256, PoisonArgs) {
    if (*A.err == 0) return;
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n; i += (uint64_t)vg.nblk * blockDim.x)
        A.out[i] = ~0ull;
}

}  // namespace mj
