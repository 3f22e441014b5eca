// Star three-way join (Sec. 6, "linear star 3-way join"): the linear query
// R(A,B) |x| S(B,C) |x| T(C,D) counted per A when R and T are small
// dimension relations and S is a large fact relation.  The paper loads R and
// T on chip and streams S once past them; no partitioning of S is needed.
//
// On MI355X the dimension tables are one-bucket multiplicity tables (built
// by the partitioner and k_dbuild of the linear path), and streaming S is a
// group-by on B weighted by mult_T(C):
//   W[b] = sum over s(b, c) in S of mult_T(c),   count[a] = sum over r(a, b) of W[b].
// R's distinct B values are numbered 0..k-1 (a prefix sum over the occupied
// slots of R's table).  "On chip" is each workgroup's LDS: one workgroup
// per CU copies T's table and R's (key, number) table there, streams its
// contiguous chunk of S, adds the weights per number in LDS and writes its
// sums once; k_star_reduce adds them up.  A random read of an L2-resident
// table costs about as much as a whole streamed tuple at these rates, which
// is why both tables are copied.  Tables larger than the LDS copies are
// probed in L2 and the sums go to global memory (exact at any size; the
// planner only picks the star plans for small R).
//
// The binary star cascade materialises I = R |x| S as (a, c) pairs (R
// grouped by B with a counting sort, one prefix sum over S for the output
// positions) and then groups I by A with the same kernel.
#include "mj_kernels.h"

namespace mj {

// slot of `key` in a one-bucket table (the extra slot pool_slots stands for
// key 0xFFFFFFFF), or STAR_NONE
__device__ __forceinline__ uint32_t star_slot(const StarTable& T, uint32_t key) {
    const DirEntry e = T.dir[0];
    if (key == EMPTY_KEY) return e.special ? T.pool_slots : STAR_NONE;
    const uint32_t mask = (1u << e.log2cap) - 1u;
    uint32_t s = slot_hash(key, T.slot_seed) & mask;
    while (true) {
        const uint2 kv = T.pool[e.offset + s];
        if (kv.x == key) return (uint32_t)(e.offset + s);
        if (kv.x == EMPTY_KEY) return STAR_NONE;
        s = (s + 1u) & mask;
    }
}

// id of `key` through R's (key, id) table in global memory, or STAR_NONE
__device__ __forceinline__ uint32_t star_id(const StarTable& R, const uint2* idtab,
                                            const unsigned long long* rid, uint32_t key) {
    const DirEntry e = R.dir[0];
    if (key == EMPTY_KEY) return e.special ? (uint32_t)rid[R.pool_slots] : STAR_NONE;
    const uint32_t mask = (1u << e.log2cap) - 1u;
    uint32_t s = slot_hash(key, R.slot_seed) & mask;
    while (true) {
        const uint2 kv = idtab[e.offset + s];
        if (kv.x == key) return kv.y;
        if (kv.x == EMPTY_KEY) return STAR_NONE;
        s = (s + 1u) & mask;
    }
}

// rows of two key columns; packed [n, 2] rows are read as 8-byte pairs
__device__ __forceinline__ uint2 star_row(const uint32_t* col0, const uint32_t* col1,
                                          int64_t stride, uint64_t i) {
    if (stride == 2 && col1 == col0 + 1 && (reinterpret_cast<uintptr_t>(col0) & 7) == 0)
        return reinterpret_cast<const uint2*>(col0)[i];
    return make_uint2(ld_col(col0, i, stride), ld_col(col1, i, stride));
}

// rows [beg, end) of this workgroup's contiguous chunk
__device__ __forceinline__ void star_chunk(uint64_t n, VGrid vg, uint64_t& beg, uint64_t& end) {
    const uint64_t per = (n + vg.nblk - 1) / vg.nblk;
    beg = uint64_t(vg.bid) * per;
    end = min<uint64_t>(n, beg + per);
}

// STAR_U lookups in a one-bucket table in global memory at once: the
// first-slot loads are in flight together and only colliding keys walk
// further.  `tab` holds (key, value) slots; an absent key gives `none`, key
// 0xFFFFFFFF gives `special`.
#ifndef MJ_STAR_U
#define MJ_STAR_U 4
#endif
constexpr int STAR_U = MJ_STAR_U;   // rows per thread per step
__device__ __forceinline__ void star_lookup4(const DirEntry& e, const uint2* __restrict__ tab,
                                             uint32_t slot_seed, const uint32_t (&key)[STAR_U],
                                             const bool (&live)[STAR_U], uint32_t none,
                                             uint32_t special, uint32_t (&out)[STAR_U]) {
    const uint32_t mask = (1u << e.log2cap) - 1u;
    const uint2* base = tab + e.offset;
    uint32_t s[STAR_U];
    uint2 kv[STAR_U];
#pragma unroll
    for (int u = 0; u < STAR_U; ++u) {
        s[u] = slot_hash(key[u], slot_seed) & mask;
        kv[u] = live[u] && key[u] != EMPTY_KEY ? base[s[u]] : make_uint2(EMPTY_KEY, 0u);
    }
#pragma unroll
    for (int u = 0; u < STAR_U; ++u) {
        if (!live[u]) { out[u] = none; continue; }
        if (key[u] == EMPTY_KEY) { out[u] = special; continue; }
        out[u] = probe_from(base, mask, key[u], kv[u], s[u], none);
    }
}

// LDS copies of the dimension tables: STAR_LDS_SLOTS packed (key, value)
// slots, rebuilt by every workgroup from a table region with a cheaper
// hash than the global tables' (one multiply; a poor spread only lengthens
// probes).  Every table copied holds at most STAR_LDS_SLOTS / 2 keys.
__device__ __forceinline__ uint32_t lds_hash(uint32_t key) {
    uint32_t h = key * 0x9E3779B1u;
    return h ^ (h >> 15);
}

__device__ __forceinline__ void lds_build(uint2* tab, const uint2* region, uint32_t cap) {
    constexpr uint32_t mask = STAR_LDS_SLOTS - 1u;
    for (uint32_t s = threadIdx.x; s < STAR_LDS_SLOTS; s += blockDim.x) tab[s] = make_uint2(EMPTY_KEY, 0u);
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < cap; s += blockDim.x) {
        const uint2 kv = region[s];
        if (kv.x == EMPTY_KEY) continue;
        uint32_t h = lds_hash(kv.x) & mask;
        while (atomicCAS(&tab[h].x, EMPTY_KEY, kv.x) != EMPTY_KEY) h = (h + 1u) & mask;   // keys are distinct
        tab[h].y = kv.y;
    }
}

// STAR_U LDS lookups at once: every row's first slot is read together (a
// hit or an empty slot costs one round trip), collisions walk further.
__device__ __forceinline__ void lds_get4(const uint2* tab, const uint32_t (&key)[STAR_U],
                                         const bool (&live)[STAR_U], uint32_t none, uint32_t special,
                                         uint32_t (&out)[STAR_U]) {
    constexpr uint32_t mask = STAR_LDS_SLOTS - 1u;
    uint32_t h[STAR_U];
    uint2 kv[STAR_U];
#pragma unroll
    for (int u = 0; u < STAR_U; ++u) {
        h[u] = lds_hash(key[u]) & mask;
        kv[u] = tab[h[u]];
    }
#pragma unroll
    for (int u = 0; u < STAR_U; ++u) {
        if (!live[u]) { out[u] = none; continue; }
        if (key[u] == EMPTY_KEY) { out[u] = special; continue; }
        out[u] = probe_from(tab, mask, key[u], kv[u], h[u], none);
    }
}

// The rows of this workgroup's chunk, STAR_U per thread per step, with the
// next step's rows loaded before the current ones are processed.
template <typename F>
__device__ __forceinline__ void star_stream(const uint32_t* col0, const uint32_t* col1, int64_t stride,
                                            uint64_t n, VGrid vg, F&& body) {
    uint64_t beg, end;
    star_chunk(n, vg, beg, end);
    const uint64_t nthr = blockDim.x, step = STAR_U * nthr;
    uint2 cur[STAR_U], nxt[STAR_U];
#pragma unroll
    for (int u = 0; u < STAR_U; ++u) {
        const uint64_t idx = beg + threadIdx.x + u * nthr;
        cur[u] = idx < end ? star_row(col0, col1, stride, idx) : make_uint2(0u, 0u);
    }
    for (uint64_t q = beg + threadIdx.x; q < end; q += step) {
#pragma unroll
        for (int u = 0; u < STAR_U; ++u) {
            const uint64_t idx = q + step + u * nthr;
            nxt[u] = idx < end ? star_row(col0, col1, stride, idx) : make_uint2(0u, 0u);
        }
        uint32_t key[STAR_U], c[STAR_U];
        bool live[STAR_U];
#pragma unroll
        for (int u = 0; u < STAR_U; ++u) {
            live[u] = q + u * nthr < end;
            key[u] = cur[u].x;
            c[u] = cur[u].y;
        }
        body(q, key, c, live);
#pragma unroll
        for (int u = 0; u < STAR_U; ++u) cur[u] = nxt[u];
    }
}

MJ_KERNEL(k_star_occ, 256, StarOccArgs) {
    const uint64_t cursor = *A.cursor;
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i <= A.R.pool_slots;
         i += (uint64_t)vg.nblk * blockDim.x) {
        uint32_t o;
        if (i == A.R.pool_slots) o = A.R.dir[0].special ? 1u : 0u;
        else o = (i < cursor && A.R.pool[i].x != EMPTY_KEY) ? 1u : 0u;
        A.occ[i] = o;
    }
}

MJ_KERNEL(k_star_ids, 256, StarIdArgs) {
    const uint32_t ps = A.R.pool_slots;
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < ps;
         i += (uint64_t)vg.nblk * blockDim.x) {
        const bool occ = A.rid[i + 1] != A.rid[i];
        A.idtab[i] = make_uint2(occ ? A.R.pool[i].x : EMPTY_KEY, occ ? (uint32_t)A.rid[i] : 0u);
    }
}

// Group-by of S = (b, c) rows by B, weight mult_T(c): the star three-way
// join's one pass over the fact relation.
MJ_KERNEL(k_star_group_b, STAR_THREADS, StarGroupArgs) {
    __shared__ uint2 ttab[STAR_LDS_SLOTS];
    __shared__ uint2 rtab[STAR_LDS_SLOTS];
    __shared__ unsigned long long acc[STAR_LDS_SLOTS / 2];
    const DirEntry re = A.R.dir[0];
    const DirEntry te = A.T.dir[0];
    const uint32_t rcap = 1u << re.log2cap, tcap = 1u << te.log2cap;
    const uint32_t k = (uint32_t)A.rid[A.R.pool_slots + 1];
    // both tables (and the k sums) in LDS; uniform over the launch
    const bool lds = rcap <= STAR_LDS_SLOTS && tcap <= STAR_LDS_SLOTS && k <= STAR_LDS_SLOTS / 2;
    const uint32_t rspecial = re.special ? (uint32_t)A.rid[A.R.pool_slots] : STAR_NONE;
    const int nthr = blockDim.x;
    if (lds) {
        lds_build(ttab, A.T.pool + te.offset, tcap);
        lds_build(rtab, A.idtab + re.offset, rcap);
        for (uint32_t i = threadIdx.x; i < k; i += nthr) acc[i] = 0;
    }
    __syncthreads();
    star_stream(A.col0, A.col1, A.stride, A.n, vg,
                [&](uint64_t, const uint32_t (&key)[STAR_U], const uint32_t (&c)[STAR_U],
                    const bool (&live)[STAR_U]) {
        uint32_t w[STAR_U], id[STAR_U];
        bool need[STAR_U];
        if (lds) {
            lds_get4(ttab, c, live, 0u, te.special, w);
#pragma unroll
            for (int u = 0; u < STAR_U; ++u) need[u] = w[u] != 0;
            lds_get4(rtab, key, need, STAR_NONE, rspecial, id);
#pragma unroll
            for (int u = 0; u < STAR_U; ++u)                 // an absent b is not in R
                if (id[u] != STAR_NONE) atomicAdd(&acc[id[u]], (unsigned long long)w[u]);
        } else {
            star_lookup4(te, A.T.pool, A.T.slot_seed, c, live, 0u, te.special, w);
#pragma unroll
            for (int u = 0; u < STAR_U; ++u) need[u] = w[u] != 0;
            star_lookup4(re, A.idtab, A.R.slot_seed, key, need, STAR_NONE, rspecial, id);
#pragma unroll
            for (int u = 0; u < STAR_U; ++u)
                if (id[u] != STAR_NONE) atomicAdd(&A.out[id[u]], (unsigned long long)w[u]);
        }
    });
    __syncthreads();
    if (lds)
        for (uint32_t i = threadIdx.x; i < k; i += nthr)
            A.partial[uint64_t(vg.bid) * STAR_STRIDE + i] = acc[i];
}

// Group-by of (a, c) rows by A value, weight mult_T(c): the star cascade's
// second join.  T's table in LDS when it fits, the sums in LDS while
// a_domain <= STAR_GROUPS.
MJ_KERNEL(k_star_group_a, STAR_THREADS, StarGroupArgs) {
    __shared__ uint2 ttab[STAR_LDS_SLOTS];
    __shared__ unsigned long long acc[STAR_GROUPS];
    const DirEntry te = A.T.dir[0];
    const uint32_t tcap = 1u << te.log2cap;
    const bool tlds = tcap <= STAR_LDS_SLOTS;            // uniform over the launch
    const uint32_t ngroups = A.ngroups_max;
    const bool local = ngroups <= STAR_GROUPS;
    const int nthr = blockDim.x;
    if (tlds) lds_build(ttab, A.T.pool + te.offset, tcap);
    if (local)
        for (uint32_t i = threadIdx.x; i < ngroups; i += nthr) acc[i] = 0;
    __syncthreads();
    star_stream(A.col0, A.col1, A.stride, A.n, vg,
                [&](uint64_t, const uint32_t (&key)[STAR_U], const uint32_t (&c)[STAR_U],
                    const bool (&live)[STAR_U]) {
        uint32_t w[STAR_U];
        if (tlds) lds_get4(ttab, c, live, 0u, te.special, w);
        else star_lookup4(te, A.T.pool, A.T.slot_seed, c, live, 0u, te.special, w);
#pragma unroll
        for (int u = 0; u < STAR_U; ++u) {
            if (w[u] == 0) continue;
            if (key[u] >= ngroups) { atomicExch(A.err, 1u); continue; }
            if (local) atomicAdd(&acc[key[u]], (unsigned long long)w[u]);
            else atomicAdd(&A.out[key[u]], (unsigned long long)w[u]);
        }
    });
    __syncthreads();
    if (local)
        for (uint32_t i = threadIdx.x; i < ngroups; i += nthr)
            A.partial[uint64_t(vg.bid) * STAR_STRIDE + i] = acc[i];
}

// out[g] = sum over blocks of partial[block][g] (LDS modes only): a block
// takes 64 groups, its 16 rows of threads each sum every 16th block's
// partials (64 consecutive groups per load), then the rows are added in LDS.
MJ_KERNEL(k_star_reduce, STAR_REDUCE_THREADS, StarReduceArgs) {
    __shared__ unsigned long long part[STAR_REDUCE_THREADS / 64][64];
    uint32_t ngroups;
    if (A.by_b) {
        const bool lds = (1u << A.rdir[0].log2cap) <= STAR_LDS_SLOTS &&
                         (1u << A.tdir[0].log2cap) <= STAR_LDS_SLOTS;
        ngroups = lds ? (uint32_t)A.rid[A.pool_slots + 1] : 0u;
    } else {
        ngroups = A.ngroups_max <= STAR_GROUPS ? A.ngroups_max : 0u;
    }
    constexpr uint32_t ROWS = STAR_REDUCE_THREADS / 64;
    const uint32_t col = threadIdx.x & 63u, row = threadIdx.x >> 6;
    for (uint32_t g0 = vg.bid * 64; g0 < ngroups; g0 += vg.nblk * 64) {
        const uint32_t g = g0 + col;
        unsigned long long s = 0;
        if (g < ngroups)
            for (uint32_t b = row; b < A.nblocks; b += ROWS) s += A.partial[uint64_t(b) * STAR_STRIDE + g];
        part[row][col] = s;
        __syncthreads();
        if (row == 0 && g < ngroups) {
            unsigned long long t = 0;
#pragma unroll
            for (uint32_t r = 0; r < ROWS; ++r) t += part[r][col];
            A.out[g] = t;
        }
        __syncthreads();
    }
}

MJ_KERNEL(k_star_count, 256, StarCountArgs) {
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)vg.nblk * blockDim.x) {
        const uint2 r = star_row(A.col0, A.col1, A.stride, i);
        const uint32_t sl = star_slot(A.R, r.y);
        if (sl == STAR_NONE) continue;
        const unsigned long long w = A.W[A.rid[sl]];
        if (w == 0) continue;
        if (r.x < A.a_domain) atomicAdd(&A.count[r.x], w);
        else atomicExch(A.err, 1u);
    }
}

// --------------------------------------------------------------- cascade
MJ_KERNEL(k_star_rmult, 256, StarRMultArgs) {
    const StarRIndexArgs& X = A.x;
    const uint32_t ps = X.R.pool_slots;
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i <= ps;
         i += (uint64_t)vg.nblk * blockDim.x) {
        if (X.rid[i + 1] == X.rid[i]) continue;        // not occupied
        A.mult[X.rid[i]] = i == ps ? X.R.dir[0].special : X.R.pool[i].y;
    }
}

MJ_KERNEL(k_star_rfill, 256, StarRIndexArgs) {
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)vg.nblk * blockDim.x) {
        const uint2 r = star_row(A.col0, A.col1, A.stride, i);
        const uint32_t sl = star_slot(A.R, r.y);      // every b of R is in its table
        if (sl == STAR_NONE) continue;                // (unless its pool ran out: reported)
        const unsigned long long id = A.rid[sl];
        const uint32_t k = atomicAdd(&A.rcur[id], 1u);
        A.ra[A.roff[id] + k] = r.x;
    }
}

// Join 1 of the cascade in two passes over S (pairs per tuple, then the
// pairs themselves at prefix-sum positions), R's (key, id) table and the
// group offsets in LDS when they fit.
template <bool WRITE>
__device__ void star_join1(const StarExpandArgs& A, VGrid vg, uint2* rtab, unsigned long long* roffs) {
    const DirEntry re = A.R.dir[0];
    const uint32_t rcap = 1u << re.log2cap;
    const uint32_t k = (uint32_t)A.rid[A.R.pool_slots + 1];
    const bool lds = rcap <= STAR_LDS_SLOTS && k < STAR_STRIDE;   // uniform over the launch
    const uint32_t rspecial = re.special ? (uint32_t)A.rid[A.R.pool_slots] : STAR_NONE;
    if (lds) {
        lds_build(rtab, A.idtab + re.offset, rcap);
        for (uint32_t i = threadIdx.x; i <= k; i += blockDim.x) roffs[i] = A.roff[i];
    }
    __syncthreads();
    const uint64_t nthr = blockDim.x;
    star_stream(A.col0, A.col1, A.stride, A.n, vg,
                [&](uint64_t q, const uint32_t (&key)[STAR_U], const uint32_t (&c)[STAR_U],
                    const bool (&live)[STAR_U]) {
        uint32_t id[STAR_U];
        if (lds) {
            lds_get4(rtab, key, live, STAR_NONE, rspecial, id);
        } else {
#pragma unroll
            for (int u = 0; u < STAR_U; ++u) id[u] = live[u] ? star_id(A.R, A.idtab, A.rid, key[u]) : STAR_NONE;
        }
#pragma unroll
        for (int u = 0; u < STAR_U; ++u) {
            if (!live[u]) continue;
            const uint64_t i = q + u * nthr;
            if (!WRITE) {
                A.icnt[i] = id[u] == STAR_NONE ? 0u
                            : (uint32_t)(lds ? roffs[id[u] + 1] - roffs[id[u]] : A.roff[id[u] + 1] - A.roff[id[u]]);
                continue;
            }
            const unsigned long long o = A.ioff[i], cnt = A.ioff[i + 1] - o;
            if (cnt == 0) continue;
            if (o + cnt > A.i_cap) { atomicExch(A.err, 1u); continue; }   // relations other than planned
            const unsigned long long base = lds ? roffs[id[u]] : A.roff[id[u]];
            for (unsigned long long j = 0; j < cnt; ++j) A.I[o + j] = make_uint2(A.ra[base + j], c[u]);
        }
    });
}

MJ_KERNEL(k_star_icount, STAR_THREADS, StarExpandArgs) {
    __shared__ uint2 rtab[STAR_LDS_SLOTS];
    __shared__ unsigned long long roffs[STAR_STRIDE + 1];
    star_join1<false>(A, vg, rtab, roffs);
}

MJ_KERNEL(k_star_expand, STAR_THREADS, StarExpandArgs) {
    __shared__ uint2 rtab[STAR_LDS_SLOTS];
    __shared__ unsigned long long roffs[STAR_STRIDE + 1];
    star_join1<true>(A, vg, rtab, roffs);
}

}  // namespace mj
