// Hash partitioner (Sec. 4 and Fig. 2 of the paper: relations are split by
// radix digits of robust hashes of their join columns; the paper leaves the
// partitioner's implementation open).
//
// Two passes over each relation, both coalesced:
//   k_part_hist    : per-tile LDS histogram of bucket ids -> global bucket counts
//   k_part_scan    : exclusive scan of the bucket counts -> bucket starts, cursors
//   k_part_scatter : per tile, tuples are placed in LDS grouped by bucket
//                    (local rank from LDS atomics), one global atomic per
//                    bucket reserves the tile's run, then the staged tile is
//                    written out linearly, so consecutive lanes store
//                    consecutive addresses inside each bucket run.
// Order inside a bucket is not specified (the joins are order-insensitive).
// Up to MJ_PART_MAX_JOBS relations are partitioned by one launch.
#include "mj_kernels.h"

namespace mj {

__device__ __forceinline__ uint32_t part_bucket(const PartJob& J, uint32_t x0, uint32_t x1) {
    uint32_t k0 = J.key0_col ? x1 : x0;
    uint32_t d = top_bits(mix32(k0, J.seed0), J.bits0);
    if (J.bits1) {
        uint32_t k1 = J.key1_col ? x1 : x0;
        d = (d << J.bits1) | top_bits(mix32(k1, J.seed1), J.bits1);
    }
    return d;
}

__device__ __forceinline__ int find_job(const PartLaunch& L, uint32_t blk) {
    int j = 0;
#pragma unroll
    for (int q = 1; q < MJ_PART_MAX_JOBS; ++q)
        if (q < L.njobs && blk >= L.job[q].tile_begin) j = q;
    return j;
}

__global__ void __launch_bounds__(PART_THREADS)
k_part_hist(PartLaunch L) {
    extern __shared__ uint32_t lhist[];
    const int jid = find_job(L, blockIdx.x);
    const PartJob& J = L.job[jid];
    const uint32_t nb = 1u << (J.bits0 + J.bits1);
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) lhist[d] = 0;
    __syncthreads();
    const uint64_t tile = blockIdx.x - J.tile_begin;
    const uint64_t beg = tile * PART_TILE;
    const uint64_t end = min<uint64_t>(beg + PART_TILE, J.n);
    for (uint64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        uint32_t x0 = ld_col(J.col0, i, J.stride);
        uint32_t x1 = ld_col(J.col1, i, J.stride);
        atomicAdd(&lhist[part_bucket(J, x0, x1)], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) {
        uint32_t c = lhist[d];
        if (c) atomicAdd(&J.counts[d], c);
    }
}

// Block-wide exclusive scan of lds[0..n) (n <= PART_THREADS * 32), in place;
// returns the total.  All threads of the block must call it.
__device__ uint32_t block_exclusive_scan(uint32_t* lds, uint32_t n, uint32_t* wave_tmp) {
    const uint32_t t = threadIdx.x;
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t b = min(n, t * per), e = min(n, b + per);
    uint32_t s = 0;
    for (uint32_t i = b; i < e; ++i) s += lds[i];
    // inclusive scan of s over the block
    uint32_t v = s;
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        uint32_t y = __shfl_up(v, off, WAVE);
        if (lane >= off) v += y;
    }
    const int w = t / WAVE, nw = blockDim.x / WAVE;
    if (lane == WAVE - 1) wave_tmp[w] = v;
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (int q = 0; q < nw; ++q) { uint32_t x = wave_tmp[q]; wave_tmp[q] = run; run += x; }
        wave_tmp[nw] = run;
    }
    __syncthreads();
    uint32_t excl = v - s + wave_tmp[w];
    for (uint32_t i = b; i < e; ++i) { uint32_t x = lds[i]; lds[i] = excl; excl += x; }
    __syncthreads();
    uint32_t total = wave_tmp[nw];
    __syncthreads();
    return total;
}

// One block per job: starts[d] = exclusive prefix of counts, starts[nb] = n,
// cursor[d] = starts[d].
__global__ void __launch_bounds__(PART_THREADS)
k_part_scan(PartLaunch L) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wave_tmp[PART_THREADS / WAVE + 1];
    const PartJob& J = L.job[blockIdx.x];
    const uint32_t nb = 1u << (J.bits0 + J.bits1);
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) lds[d] = J.counts[d];
    __syncthreads();
    uint32_t total = block_exclusive_scan(lds, nb, wave_tmp);
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) {
        J.starts[d] = lds[d];
        J.cursor[d] = lds[d];
    }
    if (threadIdx.x == 0) J.starts[nb] = total;
}

__global__ void __launch_bounds__(PART_THREADS)
k_part_scatter(PartLaunch L) {
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t wave_tmp[PART_THREADS / WAVE + 1];
    const int jid = find_job(L, blockIdx.x);
    const PartJob& J = L.job[jid];
    const uint32_t nb = 1u << (J.bits0 + J.bits1);
    uint32_t* lcount = smem;                 // [nb]  counts, then local starts
    uint32_t* gbase = smem + nb;             // [nb]  global run start per bucket
    uint2* stage = reinterpret_cast<uint2*>(smem + 2 * nb);          // [PART_TILE]
    uint16_t* stage_d = reinterpret_cast<uint16_t*>(stage + PART_TILE);  // [PART_TILE]

    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) lcount[d] = 0;
    __syncthreads();
    const uint64_t tile = blockIdx.x - J.tile_begin;
    const uint64_t beg = tile * PART_TILE;
    const uint32_t cnt = (uint32_t)min<uint64_t>(PART_TILE, J.n - beg);

    constexpr int ITEMS = PART_TILE / PART_THREADS;
    uint32_t x0[ITEMS], x1[ITEMS], dd[ITEMS], rk[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        uint32_t i = threadIdx.x + k * PART_THREADS;
        if (i < cnt) {
            x0[k] = ld_col(J.col0, beg + i, J.stride);
            x1[k] = ld_col(J.col1, beg + i, J.stride);
        }
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        uint32_t i = threadIdx.x + k * PART_THREADS;
        if (i < cnt) {
            dd[k] = part_bucket(J, x0[k], x1[k]);
            rk[k] = atomicAdd(&lcount[dd[k]], 1u);
        }
    }
    __syncthreads();
    // reserve this tile's run in every non-empty bucket, then turn counts
    // into local starts
    for (uint32_t d = threadIdx.x; d < nb; d += blockDim.x) {
        uint32_t c = lcount[d];
        gbase[d] = c ? atomicAdd(&J.cursor[d], c) : 0u;
    }
    block_exclusive_scan(lcount, nb, wave_tmp);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        uint32_t i = threadIdx.x + k * PART_THREADS;
        if (i < cnt) {
            uint32_t p = lcount[dd[k]] + rk[k];
            stage[p] = make_uint2(x0[k], x1[k]);
            stage_d[p] = (uint16_t)dd[k];
        }
    }
    __syncthreads();
    if (J.out_pair) {
        uint2* out = J.out_pair;
        for (uint32_t p = threadIdx.x; p < cnt; p += blockDim.x) {
            uint32_t d = stage_d[p];
            out[gbase[d] + (p - lcount[d])] = stage[p];
        }
    } else {
        uint32_t* out = J.out_single;
        const bool second = J.single_col != 0;
        for (uint32_t p = threadIdx.x; p < cnt; p += blockDim.x) {
            uint32_t d = stage_d[p];
            uint2 v = stage[p];
            out[gbase[d] + (p - lcount[d])] = second ? v.y : v.x;
        }
    }
}

size_t part_scatter_smem(uint32_t max_bits) {
    size_t nb = size_t(1) << max_bits;
    return nb * 8 + size_t(PART_TILE) * 10;
}

}  // namespace mj
