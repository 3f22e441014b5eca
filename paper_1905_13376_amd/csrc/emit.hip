// The linear join with its result written out: the tuples (a, b, c, d) of
// R |x| S |x| T in nested-loop order (the join of Sec. 4, whose result the
// paper's experiments aggregate instead of storing, Sec. 6).
//
// S and T are grouped by a stable sort on their mixed join key, so each run
// keeps its relation's order.  For every S element the run of its C value in
// T is found once (k_emit_sdeg), and for every R tuple the run of its B
// value in S (k_emit_rdeg); prefix sums then give each R tuple the position
// of its first (r, s) pair and of its first result tuple.
//
// k_emit gives each workgroup one tile of EMIT_TILE consecutive output
// positions, so a hub's long block of results is spread over many
// workgroups and every workgroup writes the same amount; k_emit_tiles finds
// beforehand, one thread per tile, the first and last (r, s) pair of each.
// Inside a tile the (r, s) pairs that reach it are taken 256 at a time: each
// thread places one
// pair (its R tuple found by a binary search over the tile's pair starts in
// LDS), and then all threads write the pairs' result tuples in order, each
// finding its pair by a binary search over the batch in LDS.  Writes are
// 16-byte, consecutive across the workgroup, and nontemporal.
#include "mj_kernels.h"

namespace mj {

__global__ void __launch_bounds__(256)
k_emit_sdeg(EmitSArgs A) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x * 4;
    for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x * 4 + threadIdx.x; q < A.ns; q += stride) {
        uint32_t key[4], t[4];
        bool live[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t i = q + uint64_t(u) * blockDim.x;
            live[u] = i < A.ns;
            key[u] = live[u] ? mix32(A.sc[i], A.seed) : 0u;
        }
        run_find4(A.T, key, live, t);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (!live[u]) continue;
            const uint64_t i = q + uint64_t(u) * blockDim.x;
            uint32_t st = 0, len = 0;
            if (t[u] != 0xFFFFFFFFu) {
                st = A.T.run_start[t[u]];
                len = A.T.run_start[t[u] + 1] - st;
            }
            A.tst[i] = st;
            A.tdeg[i] = len;
        }
    }
}

__global__ void __launch_bounds__(256)
k_emit_rdeg(EmitRArgs A) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x * 4;
    for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x * 4 + threadIdx.x; q < A.nr; q += stride) {
        uint32_t key[4], w[4];
        bool live[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t j = q + uint64_t(u) * blockDim.x;
            live[u] = j < A.nr;
            key[u] = live[u] ? mix32(ld_col(A.r1, j, A.rstride), A.seed) : 0u;
        }
        run_find4(A.S, key, live, w);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (!live[u]) continue;
            const uint64_t j = q + uint64_t(u) * blockDim.x;
            uint32_t sb = 0, n = 0;
            unsigned long long wo = 0;
            if (w[u] != 0xFFFFFFFFu) {
                sb = A.S.run_start[w[u]];
                n = A.S.run_start[w[u] + 1] - sb;
                wo = A.P_S[sb + n] - A.P_S[sb];
            }
            A.sst[j] = sb;
            A.pdeg[j] = n;
            A.wout[j] = wo;
        }
    }
}

// last j in [lo, hi) with v[j] <= x, given v[lo] <= x (v non-decreasing)
template <class V>
__device__ __forceinline__ uint64_t last_le(const V* v, uint64_t lo, uint64_t hi, unsigned long long x) {
    while (hi - lo > 1) {
        const uint64_t m = lo + (hi - lo) / 2;
        if (v[m] <= x) lo = m; else hi = m;
    }
    return lo;
}

// the (r, s) pair holding output position p: its global pair index, and r
__device__ __forceinline__ unsigned long long pair_of(const EmitArgs& A, unsigned long long p, uint64_t jlo,
                                                      uint64_t& j) {
    j = last_le(A.O_R, jlo, A.nr, p);
    const uint32_t sb = A.sst[j];
    const uint32_t n = (uint32_t)(A.O_I[j + 1] - A.O_I[j]);
    const unsigned long long k = p - A.O_R[j] + A.P_S[sb];
    const uint64_t i = last_le(A.P_S, sb, uint64_t(sb) + n, k);      // s of that result
    return A.O_I[j] + (i - sb);
}

// Where each tile of the launch's chunk begins and ends: (first pair, last
// pair, R tuple of the first, R tuple of the last).  One thread per tile, so
// the dependent searches of all tiles overlap.
__global__ void __launch_bounds__(256)
k_emit_tiles(EmitArgs A, uint32_t ntiles) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const unsigned long long total = A.O_R[A.nr];
    const unsigned long long hi = min<unsigned long long>(A.first + A.cap, total);
    const unsigned long long p0 = A.first + uint64_t(t) * EMIT_TILE;
    if (p0 >= hi) return;                                // k_emit skips this tile too
    const unsigned long long p1 = min<unsigned long long>(p0 + EMIT_TILE, hi);
    uint64_t j0, j1;
    const unsigned long long g0 = pair_of(A, p0, 0, j0);
    const unsigned long long g1 = pair_of(A, p1 - 1, j0, j1);
    A.tiles[t] = make_ulonglong4(g0, g1, j0, j1);
}

__global__ void __launch_bounds__(EMIT_THREADS)
k_emit(EmitArgs A) {
    __shared__ unsigned long long oi[EMIT_JWIN];       // O_I over the tile's R tuples
    __shared__ uint32_t pstart[EMIT_THREADS];          // batch: first tile offset of each pair
    __shared__ uint4 prec[EMIT_THREADS];               // batch: (a, b, c, first t) of each pair
    __shared__ uint32_t s_qend;

    const unsigned long long total = A.O_R[A.nr];
    const unsigned long long hi = min<unsigned long long>(A.first + A.cap, total);
    const unsigned long long p0 = A.first + uint64_t(blockIdx.x) * EMIT_TILE;
    if (p0 >= hi) return;                                // uniform over the workgroup
    const unsigned long long p1 = min<unsigned long long>(p0 + EMIT_TILE, hi);

    const ulonglong4 tl = A.tiles[blockIdx.x];
    const unsigned long long g0 = tl.x, g1 = tl.y;
    const uint64_t j0 = tl.z, j1 = tl.w;
    const bool win = j1 - j0 < EMIT_JWIN;
    if (win)
        for (uint64_t k = threadIdx.x; k <= j1 - j0; k += blockDim.x) oi[k] = A.O_I[j0 + k];
    __syncthreads();

    for (unsigned long long gb = g0; gb <= g1; gb += EMIT_THREADS) {
        const uint32_t nvalid = (uint32_t)min<unsigned long long>(EMIT_THREADS, g1 - gb + 1);
        if (threadIdx.x < nvalid) {
            const unsigned long long g = gb + threadIdx.x;
            const uint64_t j = win ? j0 + last_le(oi, 0, j1 - j0 + 1, g) : last_le(A.O_I, j0, j1 + 1, g);
            const uint32_t sb = A.sst[j];
            const uint64_t i = sb + (g - A.O_I[j]);
            const unsigned long long ps = A.O_R[j] + (A.P_S[i] - A.P_S[sb]);
            const unsigned long long pe = ps + (A.P_S[i + 1] - A.P_S[i]);
            const unsigned long long s_abs = max(ps, p0);
            const unsigned long long e_abs = min(pe, p1);
            pstart[threadIdx.x] = (uint32_t)(s_abs - p0);
            prec[threadIdx.x] = make_uint4(ld_col(A.r0, j, A.rstride), ld_col(A.r1, j, A.rstride), A.sc[i],
                                           A.tst[i] + (uint32_t)(s_abs - ps));
            if (threadIdx.x == nvalid - 1) s_qend = (uint32_t)(e_abs - p0);
        }
        __syncthreads();
        const uint32_t qend = s_qend;
        // four outputs per thread and step: their searches and loads overlap
        for (uint32_t q0 = pstart[0] + threadIdx.x; q0 < qend; q0 += 4 * blockDim.x) {
            uint32_t d[4];
            uint4 r[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t q = min(q0 + u * blockDim.x, qend - 1);      // clamped: stays in range
                const uint32_t k = (uint32_t)last_le(pstart, 0, nvalid, q);
                r[u] = prec[k];
                r[u].w += q - pstart[k];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) d[u] = A.td[r[u].w];
            // streaming stores: the output is not read again here, and keeping
            // it out of the caches leaves them to T's runs
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t q = q0 + u * blockDim.x;
                if (q < qend) {
                    u32x4 v;
                    v.x = r[u].x; v.y = r[u].y; v.z = r[u].z; v.w = d[u];
                    __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(A.out) + (p0 - A.first + q));
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace mj
