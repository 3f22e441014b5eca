// Star three-way join (Sec. 6, "linear star 3-way join"): the linear query
// R(A,B) |x| S(B,C) |x| T(C,D) counted per A when R and T are small
// dimension relations and S is a large fact relation.  The paper loads R and
// T on chip and streams S once past them; no partitioning of S is needed.
//
// On MI355X the dimension tables are one-bucket multiplicity tables (built
// by the partitioner and k_dbuild of the linear path) that stay L2-resident,
// and streaming S is a group-by on B weighted by mult_T(C):
//   W[b] = sum over s(b, c) in S of mult_T(c),   count[a] = sum over r(a, b) of W[b].
// R's distinct B values are numbered 0..k-1 (a prefix sum over the occupied
// slots of R's table), so a workgroup can keep W in an LDS array indexed by
// that number when k <= STAR_GROUPS; each workgroup then writes its sums
// once and k_star_reduce adds them up.  With more groups the sums go to the
// global array with atomics (correct at any size; the planner only picks the
// star plans when the groups fit LDS).
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

// multiplicity of `key` in a one-bucket table (0 when absent)
__device__ __forceinline__ uint32_t star_mult(const StarTable& T, uint32_t key) {
    const DirEntry e = T.dir[0];
    if (key == EMPTY_KEY) return e.special;
    const uint32_t mask = (1u << e.log2cap) - 1u;
    uint32_t s = slot_hash(key, T.slot_seed) & mask;
    while (true) {
        const uint2 kv = T.pool[e.offset + s];
        if (kv.x == key) return kv.y;
        if (kv.x == EMPTY_KEY) return 0u;
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

__global__ void k_star_occ(StarOccArgs A) {
    const uint64_t cursor = *A.cursor;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i <= A.R.pool_slots;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t o;
        if (i == A.R.pool_slots) o = A.R.dir[0].special ? 1u : 0u;
        else o = (i < cursor && A.R.pool[i].x != EMPTY_KEY) ? 1u : 0u;
        A.occ[i] = o;
    }
}

// Group-by of a stream of (key, c) rows, weight mult_T(c).  Each workgroup
// takes one contiguous chunk of the rows (coalesced reads, four rows per
// thread in flight).
__global__ void __launch_bounds__(STAR_THREADS)
k_star_group(StarGroupArgs A) {
    __shared__ unsigned long long acc[STAR_GROUPS];
    const uint32_t ngroups = A.by_rid ? (uint32_t)A.rid[A.R.pool_slots + 1] : A.ngroups_max;
    const bool local = ngroups <= STAR_GROUPS;           // uniform over the launch
    const int nthr = blockDim.x;
    if (local)
        for (uint32_t i = threadIdx.x; i < ngroups; i += nthr) acc[i] = 0;
    __syncthreads();
    const uint64_t per = (A.n + gridDim.x - 1) / gridDim.x;
    const uint64_t beg = uint64_t(blockIdx.x) * per;
    const uint64_t end = min<uint64_t>(A.n, beg + per);
    for (uint64_t q = beg + threadIdx.x; q < end; q += 4 * (uint64_t)nthr) {
        uint2 row[4];
        uint32_t w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t idx = q + u * (uint64_t)nthr;
            row[u] = idx < end ? star_row(A.col0, A.col1, A.stride, idx) : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            w[u] = q + u * (uint64_t)nthr < end ? star_mult(A.T, row[u].y) : 0u;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (w[u] == 0) continue;
            uint32_t id;
            if (A.by_rid) {
                const uint32_t sl = star_slot(A.R, row[u].x);
                if (sl == STAR_NONE) continue;                   // b not in R
                id = (uint32_t)A.rid[sl];
            } else {
                id = row[u].x;
            }
            if (id >= ngroups) { atomicExch(A.err, 1u); continue; }
            if (local) atomicAdd(&acc[id], (unsigned long long)w[u]);
            else atomicAdd(&A.out[id], (unsigned long long)w[u]);
        }
    }
    __syncthreads();
    if (local)
        for (uint32_t i = threadIdx.x; i < ngroups; i += nthr)
            A.partial[uint64_t(blockIdx.x) * STAR_GROUPS + i] = acc[i];
}

// out[id] = sum over blocks of partial[block][id] (LDS mode only)
__global__ void k_star_reduce(StarReduceArgs A) {
    const uint32_t ngroups = A.by_rid ? (uint32_t)A.rid[A.pool_slots + 1] : A.ngroups_max;
    if (ngroups > STAR_GROUPS) return;                  // the sums are already global
    for (uint32_t id = blockIdx.x * blockDim.x + threadIdx.x; id < ngroups;
         id += gridDim.x * blockDim.x) {
        unsigned long long s = 0;
        for (uint32_t b = 0; b < A.nblocks; ++b) s += A.partial[uint64_t(b) * STAR_GROUPS + id];
        A.out[id] = s;
    }
}

__global__ void k_star_count(StarCountArgs A) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)gridDim.x * blockDim.x) {
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
__global__ void k_star_rmult(StarRIndexArgs A, uint32_t* mult) {
    const uint32_t ps = A.R.pool_slots;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i <= ps;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (A.rid[i + 1] == A.rid[i]) continue;        // not occupied
        mult[A.rid[i]] = i == ps ? A.R.dir[0].special : A.R.pool[i].y;
    }
}

__global__ void k_star_rfill(StarRIndexArgs A) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint2 r = star_row(A.col0, A.col1, A.stride, i);
        const uint32_t sl = star_slot(A.R, r.y);      // every b of R is in its table
        if (sl == STAR_NONE) continue;                // (unless its pool ran out: reported)
        const unsigned long long id = A.rid[sl];
        const uint32_t k = atomicAdd(&A.rcur[id], 1u);
        A.ra[A.roff[id] + k] = r.x;
    }
}

__global__ void k_star_icount(StarExpandArgs A) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint2 s = star_row(A.col0, A.col1, A.stride, i);
        const uint32_t sl = star_slot(A.R, s.x);
        uint32_t c = 0;
        if (sl != STAR_NONE) {
            const unsigned long long id = A.rid[sl];
            c = (uint32_t)(A.roff[id + 1] - A.roff[id]);
        }
        A.icnt[i] = c;
    }
}

__global__ void k_star_expand(StarExpandArgs A) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long o = A.ioff[i], cnt = A.ioff[i + 1] - o;
        if (cnt == 0) continue;
        const uint2 s = star_row(A.col0, A.col1, A.stride, i);
        if (o + cnt > A.i_cap) { atomicExch(A.err, 1u); continue; }   // relations other than planned
        const unsigned long long base = A.roff[A.rid[star_slot(A.R, s.x)]];
        for (unsigned long long k = 0; k < cnt; ++k) A.I[o + k] = make_uint2(A.ra[base + k], s.y);
    }
}

}  // namespace mj
