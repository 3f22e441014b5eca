// Hash partitioner (Sec. 4 and Fig. 2 of the paper: relations are split by
// radix digits of robust hashes of their join columns; the paper leaves the
// partitioner's implementation open).
//
// Three launches per group of relations, none with a global atomic:
//   k_part_hist    : per tile, an LDS histogram of bucket ids, stored as
//                    column `tile` of a bucket-major matrix hist[d][tile]
//   k_part_rowscan : per bucket, the exclusive prefix of its row over tiles
//                    (in place) and the row total
//   k_part_scan    : per relation, the exclusive prefix of the bucket totals
//                    (bucket starts)
//   k_part_scatter : per tile, tuples are grouped by bucket in LDS (local
//                    rank by LDS atomics), then the staged tile is written
//                    out linearly: lane p stores element p of the tile's
//                    bucket-sorted order at starts[d] + hist[d][tile] + rank,
//                    so consecutive lanes store consecutive addresses inside
//                    every (tile, bucket) run.
// Tiles hold PART_TILE tuples; with at most 2^PART_MAX_BITS buckets a
// (tile, bucket) run averages >= 8 tuples.  Packed [n, 2] inputs are read
// with 16-byte loads.  Order inside a bucket is not specified.
#include "mj_kernels.h"

namespace mj {

__device__ __forceinline__ uint32_t part_bucket(const PartJob& J, uint32_t x0, uint32_t x1) {
    uint32_t k0 = J.key0_col ? x1 : x0;
    if (J.range_on) return min(k0 >> J.range_shift, (1u << J.bits0) - 1u);
    uint32_t d = top_bits(mix32(k0, J.seed0), J.bits0);
    if (J.bits1) {
        uint32_t k1 = J.key1_col ? x1 : x0;
        d = (d << J.bits1) | top_bits(mix32(k1, J.seed1), J.bits1);
    }
    return d;
}

#ifndef MJ_PART_NT_STORE
#define MJ_PART_NT_STORE 0
#endif
#ifndef MJ_PART_XCD_REMAP
#define MJ_PART_XCD_REMAP 1
#endif

// Output stores.  Plain stores let an XCD's write-back L2 merge the two
// halves of a cache line that adjacent tiles' runs share; nontemporal ones
// stream past it.
template <typename T>
__device__ __forceinline__ void part_store(T v, T* p) {
    if constexpr (MJ_PART_NT_STORE) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// The tile a block works on: tiles of one XCD are contiguous, so the runs
// adjacent tiles write into one bucket (adjacent in the output) meet in the
// same L2.
__device__ __forceinline__ uint32_t part_block(VGrid vg) {
    return MJ_PART_XCD_REMAP ? xcd_remap(vg.bid, vg.nblk) : vg.bid;
}

__device__ __forceinline__ int find_job(const PartLaunch& L, uint32_t blk) {
    int j = 0;
#pragma unroll
    for (int q = 1; q < MJ_PART_MAX_JOBS; ++q)
        if (q < L.njobs && blk >= L.job[q].tile_begin) j = q;
    return j;
}

// Load the tile's tuples into registers: item k of thread t is tuple
// beg + t*2 + (k&1) + (k>>1)*2*blockDim for packed inputs (two tuples per
// 16-byte load), beg + t + k*blockDim otherwise.
template <int ITEMS>
__device__ __forceinline__ void load_tile(const PartJob& J, uint64_t beg, uint32_t cnt,
                                          uint32_t (&x0)[ITEMS], uint32_t (&x1)[ITEMS],
                                          uint32_t (&idx)[ITEMS]) {
    const uint32_t t = threadIdx.x, B = blockDim.x;
    if (J.packed) {
        const u32x4* src = reinterpret_cast<const u32x4*>(J.col0 + 2 * beg);
#pragma unroll
        for (int k = 0; k < ITEMS; k += 2) {
            const uint32_t i = 2 * t + (k >> 1) * 2 * B;   // first of two tuples
            idx[k] = i;
            idx[k + 1] = i + 1;
            if (i + 1 < cnt) {
                u32x4 v = __builtin_nontemporal_load(src + (i >> 1));
                x0[k] = v.x; x1[k] = v.y; x0[k + 1] = v.z; x1[k + 1] = v.w;
            } else if (i < cnt) {
                x0[k] = J.col0[2 * (beg + i)];
                x1[k] = J.col0[2 * (beg + i) + 1];
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t i = t + k * B;
            idx[k] = i;
            if (i < cnt) {
                x0[k] = ld_col(J.col0, beg + i, J.stride);
                x1[k] = ld_col(J.col1, beg + i, J.stride);
            }
        }
    }
}

MJ_KERNEL(k_part_hist, PART_THREADS, PartLaunch) {
    const PartLaunch& L = A;
    extern __shared__ uint32_t lhist[];
    const uint32_t blk = part_block(vg);
    const int jid = find_job(L, blk);
    const PartJob& J = L.job[jid];
    const uint32_t nb = 1u << (J.bits0 + J.bits1);
    if (vg.bid == 0) {                               // before the next launches of the group
        for (uint32_t w = threadIdx.x; w < L.nclear; w += blockDim.x) L.clear[w] = 0;
    }
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) lhist[d] = 0;
    __syncthreads();
    const uint32_t tile = blk - J.tile_begin;
    const uint64_t beg = uint64_t(tile) * PART_TILE;
    const uint32_t cnt = (uint32_t)min<uint64_t>(PART_TILE, J.n - beg);
    constexpr int ITEMS = PART_TILE / PART_THREADS;
    uint32_t x0[ITEMS], x1[ITEMS], idx[ITEMS];
    load_tile<ITEMS>(J, beg, cnt, x0, x1, idx);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (idx[k] < cnt) atomicAdd(&lhist[part_bucket(J, x0[k], x1[k])], 1u);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x)
        J.hist[uint64_t(d) * J.ntiles + tile] = lhist[d];
}

// grid = sum over jobs of nb; block = one bucket row of one job.
MJ_KERNEL(k_part_rowscan, PART_THREADS, PartLaunch) {
    const PartLaunch& L = A;
    __shared__ uint32_t wave_tmp[PART_THREADS / WAVE + 1];
    __shared__ uint32_t carry;
    int jid = 0;
    uint32_t row = vg.bid;
    for (int q = 0; q < L.njobs; ++q) {
        const uint32_t nbq = 1u << (L.job[q].bits0 + L.job[q].bits1);
        if (row < nbq) { jid = q; break; }
        row -= nbq;
    }
    const PartJob& J = L.job[jid];
    uint32_t* h = J.hist + uint64_t(row) * J.ntiles;
    extern __shared__ uint32_t chunk[];           // PART_SCAN_CHUNK entries
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t c0 = 0; c0 < J.ntiles; c0 += PART_SCAN_CHUNK) {
        const uint32_t m = min<uint32_t>(PART_SCAN_CHUNK, J.ntiles - c0);
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) chunk[i] = h[c0 + i];
        __syncthreads();
        const uint32_t tot = block_exclusive_scan(chunk, m, wave_tmp);
        const uint32_t base = carry;
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) h[c0 + i] = chunk[i] + base;
        __syncthreads();
        if (threadIdx.x == 0) carry = base + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) J.counts[row] = carry;
}

// Bucket starts of one job: starts[d] = exclusive prefix of counts,
// starts[nb] = n; then, when the job asks, the work items of its buckets:
// first the pieces of the split buckets (so the longest work starts first;
// piece p of bucket d is item and scratch row hrow[d] + p), then the other
// buckets in bucket order.  All threads of the block call it.
__device__ void part_scan_job(const PartJob& J, uint32_t* lds, uint32_t* wave_tmp) {
    const uint32_t* counts = J.counts;
    const uint32_t nb = 1u << (J.bits0 + J.bits1);
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) lds[d] = counts[d];
    __syncthreads();
    uint32_t total = block_exclusive_scan(lds, nb, wave_tmp);
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) J.starts[d] = lds[d];
    if (threadIdx.x == 0) J.starts[nb] = total;
    if (!J.split.items) return;                      // uniform over the block
    const BucketItems& B = J.split;
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) {
        const uint32_t pcs = split_pieces(counts[d], B.chunk);
        lds[d] = pcs > 1 ? pcs : 0u;
    }
    __syncthreads();
    const uint32_t heavy = block_exclusive_scan(lds, nb, wave_tmp);
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) {
        const uint32_t pcs = split_pieces(counts[d], B.chunk);
        if (pcs == 1) continue;
        B.hrow[d] = lds[d];
        B.done[d] = 0;
        for (uint32_t p = 0; p < pcs; ++p) B.items[lds[d] + p] = d | (p << 12);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) lds[d] = split_pieces(counts[d], B.chunk) == 1 ? 1u : 0u;
    __syncthreads();
    const uint32_t light = block_exclusive_scan(lds, nb, wave_tmp);
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x)
        if (split_pieces(counts[d], B.chunk) == 1) B.items[heavy + lds[d]] = d;
    if (threadIdx.x == 0) *B.nitems = heavy + light;
}

// One block per job.
MJ_KERNEL(k_part_scan, PART_THREADS, PartLaunch) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wave_tmp[PART_THREADS / WAVE + 1];
    part_scan_job(A.job[vg.bid], lds, wave_tmp);
}

MJ_KERNEL(k_part_scatter, PART_SCATTER_THREADS, PartLaunch) {
    const PartLaunch& L = A;
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t wave_tmp[PART_SCATTER_THREADS / WAVE + 1];
    const uint32_t blk = part_block(vg);
    const int jid = find_job(L, blk);
    const PartJob& J = L.job[jid];
    const uint32_t nb = 1u << (J.bits0 + J.bits1);
    uint32_t* lcount = smem;                 // [nb]  counts, then local starts
    uint32_t* gbase = smem + nb;             // [nb]  global run start per bucket
    uint32_t* stage = smem + 2 * nb;         // [PART_TILE] (x2 words for pairs)

    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) lcount[d] = 0;
    __syncthreads();
    const uint32_t tile = blk - J.tile_begin;
    const uint64_t beg = uint64_t(tile) * PART_TILE;
    const uint32_t cnt = (uint32_t)min<uint64_t>(PART_TILE, J.n - beg);

    constexpr int ITEMS = PART_TILE / PART_SCATTER_THREADS;
    uint32_t x0[ITEMS], x1[ITEMS], idx[ITEMS], rk[ITEMS];
    load_tile<ITEMS>(J, beg, cnt, x0, x1, idx);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        if (idx[k] < cnt) {
            const uint32_t d = part_bucket(J, x0[k], x1[k]);
            rk[k] = (d << 16) | atomicAdd(&lcount[d], 1u);   // PART_TILE <= 2^16
        }
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x)
        gbase[d] = J.starts[d] + J.hist[uint64_t(d) * J.ntiles + tile];
    block_exclusive_scan(lcount, nb, wave_tmp);
    const bool pair = J.out_pair != nullptr;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        if (idx[k] < cnt) {
            const uint32_t d = rk[k] >> 16;
            const uint32_t p = lcount[d] + (rk[k] & 0xFFFFu);
            if (pair) {
                reinterpret_cast<uint2*>(stage)[p] = make_uint2(x0[k], x1[k]);
            } else {
                stage[p] = J.single_col ? x1[k] : x0[k];
            }
        }
    }
    __syncthreads();
    // write out in bucket-sorted order; the bucket of element p is recomputed
    // from its key (a binary search over lcount would cost as much)
    if (pair) {
        const uint2* st = reinterpret_cast<const uint2*>(stage);
        for (uint32_t p = threadIdx.x; p < cnt; p += blockDim.x) {
            const uint2 v = st[p];
            const uint32_t d = part_bucket(J, v.x, v.y);
            u32x2 w;
            w.x = J.swap_out ? v.y : v.x;
            w.y = J.swap_out ? v.x : v.y;
            part_store(w, reinterpret_cast<u32x2*>(J.out_pair) + gbase[d] + (p - lcount[d]));
        }
    } else {
        // single-column payloads are only used with a one-column bucket id
        // (bits1 = 0) computed from that same column, so the staged value
        // alone gives its bucket, hashed or by range as when it was staged
        for (uint32_t p = threadIdx.x; p < cnt; p += blockDim.x) {
            const uint32_t v = stage[p];
            const uint32_t d = part_bucket(J, v, v);
            part_store(v, J.out_single + gbase[d] + (p - lcount[d]));
        }
    }
}

size_t part_scatter_smem(uint32_t max_bits) {
    size_t nb = size_t(1) << max_bits;
    return nb * 8 + size_t(PART_TILE) * 8;
}

}  // namespace mj
