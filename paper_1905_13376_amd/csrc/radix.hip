// Stable LSD radix sort of 64-bit keys (8-bit digits), the repeated radix
// partitioning that groups each relation of the cyclic join by its join key
// (Fig. 3 partitions by radix digits of A, B and C).
//
//   k_rs_hist    : per tile, digit histogram -> column `tile` of hist[d][tile]
//   (k_part_rowscan / k_part_scan give every (digit, tile) its output start)
//   k_rs_scatter : per tile, stable ranks: the tile is walked in rounds of
//                  blockDim keys in input order; inside a round the rank of a
//                  key among equal digits is its position among the wave's
//                  matching lanes (found with eight ballots) plus the counts
//                  of earlier waves and earlier rounds.
#include "mj_kernels.h"

namespace mj {

__global__ void __launch_bounds__(RS_THREADS)
k_rs_hist(RsArgs A) {
    __shared__ uint32_t lh[256];
    const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
    for (uint32_t d = threadIdx.x; d < 256; d += blockDim.x) lh[d] = 0;
    __syncthreads();
    const uint64_t beg = uint64_t(tile) * RS_TILE;
    const uint64_t end = min<uint64_t>(beg + RS_TILE, A.n);
    for (uint64_t i = beg + threadIdx.x; i < end; i += blockDim.x)
        atomicAdd(&lh[(uint32_t)(A.in[i] >> A.shift) & 255u], 1u);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < 256; d += blockDim.x)
        A.hist[uint64_t(d) * A.ntiles + tile] = lh[d];
}

__global__ void __launch_bounds__(RS_THREADS)
k_rs_scatter(RsArgs A) {
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[RS_THREADS / WAVE][256];
    // adjacent tiles write adjacent runs of every digit: keep them on one XCD
    const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = lane_id();
    const int w = threadIdx.x / WAVE;
    constexpr int NW = RS_THREADS / WAVE;
    for (uint32_t d = threadIdx.x; d < 256; d += blockDim.x) {
        running[d] = A.starts[d] + A.hist[uint64_t(d) * A.ntiles + tile];
        for (int q = 0; q < NW; ++q) wcnt[q][d] = 0;
    }
    __syncthreads();
    const uint64_t beg = uint64_t(tile) * RS_TILE;
    const uint64_t end = min<uint64_t>(beg + RS_TILE, A.n);
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (uint64_t r0 = beg; r0 < end; r0 += RS_THREADS) {
        const uint64_t i = r0 + threadIdx.x;
        const bool live = i < end;
        const unsigned long long key = live ? A.in[i] : 0ull;
        const uint32_t d = (uint32_t)(key >> A.shift) & 255u;
        // lanes of this wave holding the same digit
        unsigned long long peers = __ballot(live);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long bal = __ballot(live && ((d >> bit) & 1u));
            peers &= ((d >> bit) & 1u) ? bal : ~bal;
        }
        const uint32_t rank_w = __popcll(peers & lt_mask);
        const bool leader = live && rank_w == 0;
        if (leader) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (live) {
            uint32_t before = 0;
            for (int q = 0; q < w; ++q) before += wcnt[q][d];
            A.out[running[d] + before + rank_w] = key;
        }
        __syncthreads();
        if (leader) {
            // the last wave holding digit d in this round advances running[d]
            bool last = true;
            for (int q = w + 1; q < NW; ++q) last = last && wcnt[q][d] == 0;
            if (last) {
                uint32_t tot = 0;
                for (int q = 0; q < NW; ++q) tot += wcnt[q][d];
                running[d] += tot;
            }
        }
        __syncthreads();
        if (leader) wcnt[w][d] = 0;
        __syncthreads();
    }
}

}  // namespace mj
