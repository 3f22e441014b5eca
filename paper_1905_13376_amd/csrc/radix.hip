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
//   k_rs_scan1   : with few tiles, one workgroup does both scans of a pass
//   k_rs_small   : arrays of at most RS_SMALL keys are sorted whole in one
//                  workgroup's LDS, in one launch instead of four per pass.
#include "mj_kernels.h"

namespace mj {

MJ_KERNEL(k_rs_hist, RS_THREADS, RsArgs) {
    __shared__ uint32_t lh[256];
    const uint32_t tile = xcd_remap(vg.bid, vg.nblk);
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

MJ_KERNEL(k_rs_scatter, RS_THREADS, RsArgs) {
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[RS_THREADS / WAVE][256];
    // adjacent tiles write adjacent runs of every digit: keep them on one XCD
    const uint32_t tile = xcd_remap(vg.bid, vg.nblk);
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

// One workgroup, at most RS_SCAN1_TILES tiles: every digit's row of the
// histogram becomes its exclusive prefix over tiles (in place), and the
// digits' totals their exclusive prefix (starts, with starts[256] = n):
// what k_part_rowscan and k_part_scan write, in one launch.
MJ_KERNEL(k_rs_scan1, 256, RsScan1Args) {
    (void)vg;
    const RsArgs& R = A.rs;
    uint32_t* starts = A.starts;
    __shared__ uint32_t h[256 * RS_SCAN1_TILES];
    __shared__ uint32_t tot[256];
    __shared__ uint32_t wave_tmp[256 / WAVE + 1];
    const uint32_t nt = R.ntiles, m = 256 * nt;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) h[i] = R.hist[i];
    __syncthreads();
    {
        const uint32_t d = threadIdx.x;          // one digit per thread
        uint32_t run = 0;
        for (uint32_t t = 0; t < nt; ++t) {
            const uint32_t c = h[d * nt + t];
            h[d * nt + t] = run;
            run += c;
        }
        tot[d] = run;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) R.hist[i] = h[i];
    const uint32_t total = block_exclusive_scan(tot, 256, wave_tmp);
    starts[threadIdx.x] = tot[threadIdx.x];
    if (threadIdx.x == 0) starts[256] = total;
}

// The keys ordered on their bits from `shift` up, ties in input order: the
// order the passes from `shift` up produce.  With shift = 0 the keys are
// sorted as they are (equal keys cannot be told apart).  Otherwise each key's
// digits are packed above its index, which makes every composite distinct,
// the composites are sorted, and each position takes the key its index names
// (kept in LDS beside them).  A bitonic network over the next power of two,
// padded with the largest value; pads sort after every real entry.
MJ_KERNEL(k_rs_small, RS_SMALL_THREADS, RsSmallArgs) {
    (void)vg;
    unsigned long long* keys = A.keys;
    const uint32_t n = A.n, shift = A.shift;
    extern __shared__ unsigned long long rs_lds[];
    uint32_t P = 2;
    while (P < n) P <<= 1;
    unsigned long long* v = rs_lds;
    // sorting on the bits above `shift` only: the sort key is those bits
    // with the element's index below them, so equal keys keep their order
    for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
        unsigned long long x = ~0ull;
        if (i < n) {
            const unsigned long long k = keys[i];
            x = shift ? (((k >> shift) << RS_SMALL_BITS) | i) : k;
        }
        v[i] = x;
    }
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const uint32_t lo = 2 * t - (t & (j - 1));   // t with a 0 bit inserted at j
                const uint32_t hi = lo + j;
                const unsigned long long a = v[lo], b = v[hi];
                if ((a > b) == ((lo & k) == 0)) {
                    v[lo] = b;
                    v[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    if (shift) {                      // the original keys, in sorted order, gathered before any is overwritten
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) v[i] = keys[uint32_t(v[i]) & (RS_SMALL - 1u)];
        __syncthreads();
    }
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) keys[i] = v[i];
}

}  // namespace mj
