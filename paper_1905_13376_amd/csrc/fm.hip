// Distinct count of the linear join's D values per A with Flajolet-Martin
// sketches (the footnotes to Example 1 and to Sec. 4's step list: friends of
// friends of friends per person, a union of large overlapping sets that a
// few bytes per set approximate).
//
// The sketch of a set holds FM_WORDS bitmaps; a value x with hash
// h = mix(x) sets bit (trailing zeros of h >> 4, or 28 when h >> 4 is 0) of
// bitmap h & 15, and the estimate is (16 / 0.77351) 2^(mean lowest zero
// bit).  Sketches merge by OR, so the per-A sketch follows the linear join
// with OR in place of the count's sum and product:
//   Tsk[c] = OR over t(c, d) of bit(d)
//   Wsk[b] = OR over s(b, c) of Tsk[c]
//   sketch[a] = OR over r(a, b) of Wsk[b]
// T and S are grouped by sorting their mixed keys (runs of equal high words
// with a prefix directory, as in the cyclic join); one thread builds the
// sketch of a short run in registers, one wave that of a long run.  R is partitioned by ranges of A, and one
// workgroup ORs its range's sketches in LDS and writes them with their
// estimates.
#include "mj_kernels.h"

namespace mj {

__device__ __forceinline__ void fm_bit(uint32_t h, uint32_t (&sk)[FM_WORDS]) {
    const uint32_t rest = h >> 4;
    const uint32_t bit = 1u << (rest ? __builtin_ctz(rest) : 28u);
    const uint32_t j = h & 15u;
#pragma unroll
    for (int k = 0; k < FM_WORDS; ++k) sk[k] |= (uint32_t)k == j ? bit : 0u;
}

// (16 / 0.77351) * 2^(sum / 16): exact powers of two times 2^(1/16) taken
// (sum mod 16) times, the same sequence of double multiplications the
// definition's reference uses, so that estimates agree bit for bit
__device__ __forceinline__ double fm_estimate(const uint32_t* sk) {
    bool any = false;
    uint32_t sum = 0;
    for (int j = 0; j < FM_WORDS; ++j) {
        any = any || sk[j] != 0;
        sum += sk[j] == 0xFFFFFFFFu ? 32u : (uint32_t)__builtin_ctz(~sk[j]);
    }
    if (!any) return 0.0;
    double p = 1.0;
    for (uint32_t i = 0; i < sum / 16; ++i) p *= 2.0;
    double f = 1.0;
    for (uint32_t i = 0; i < sum % 16; ++i) f *= 1.0442737824274138;   // 2^(1/16)
    return 16.0 / 0.77351 * p * f;
}

__device__ __forceinline__ void fm_store(uint32_t* dst, const uint32_t (&sk)[FM_WORDS]) {
    uint4* d = reinterpret_cast<uint4*>(dst);
#pragma unroll
    for (int q = 0; q < FM_WORDS / 4; ++q) d[q] = make_uint4(sk[4 * q], sk[4 * q + 1], sk[4 * q + 2], sk[4 * q + 3]);
}

__device__ __forceinline__ void fm_or(const uint32_t* src, uint32_t (&sk)[FM_WORDS]) {
    const uint4* s = reinterpret_cast<const uint4*>(src);
#pragma unroll
    for (int q = 0; q < FM_WORDS / 4; ++q) {
        const uint4 v = s[q];
        sk[4 * q] |= v.x; sk[4 * q + 1] |= v.y; sk[4 * q + 2] |= v.z; sk[4 * q + 3] |= v.w;
    }
}

// OR of the lanes' sketches, left in every lane
__device__ __forceinline__ void fm_wave_or(uint32_t (&sk)[FM_WORDS]) {
#pragma unroll
    for (int k = 0; k < FM_WORDS; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sk[k] |= (uint32_t)__shfl_xor((int)sk[k], off, WAVE);
}

// Runs are sketched by one thread when short and by one wave when long
// (hub values), so that a hub's list does not serialise its kernel.
__device__ __forceinline__ void fm_t_elem(const FmTArgs& A, uint32_t i, uint32_t (&sk)[FM_WORDS]) {
    fm_bit((uint32_t)A.Tk[i], sk);
}


__global__ void __launch_bounds__(FM_THREADS)
k_fm_tsketch(FmTArgs A) {
    const uint64_t nruns = *A.T.nruns;
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < nruns;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = A.T.run_start[r], e = A.T.run_start[r + 1];
        if (e - b > FM_SHORT) continue;
        uint32_t sk[FM_WORDS] = {};
        for (uint32_t i = b; i < e; ++i) fm_t_elem(A, i, sk);
        fm_store(A.tsk + r * FM_WORDS, sk);
    }
}

__global__ void __launch_bounds__(FM_THREADS)
k_fm_tsketch_long(FmTArgs A) {
    const uint64_t nruns = *A.T.nruns;
    const uint64_t nw = uint64_t(gridDim.x) * (blockDim.x / WAVE);
    const int lane = lane_id();
    for (uint64_t r = blockIdx.x * (uint64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; r < nruns; r += nw) {
        const uint32_t b = A.T.run_start[r], e = A.T.run_start[r + 1];
        if (e - b <= FM_SHORT) continue;                              // wave-uniform
        uint32_t sk[FM_WORDS] = {};
        for (uint32_t i = b + lane; i < e; i += WAVE) fm_t_elem(A, i, sk);
        fm_wave_or(sk);
        if (lane == 0) fm_store(A.tsk + r * FM_WORDS, sk);
    }
}

// OR into sk T's sketches of the C values of S's elements i0, i0 + step, ...
// (four of them, those below e), with the four lookups in flight together
__device__ __forceinline__ void fm_w_elem4(const FmWArgs& A, uint32_t i0, uint32_t step, uint32_t e,
                                           uint32_t (&sk)[FM_WORDS]) {
    uint32_t key[4], t[4];
    bool live[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t i = i0 + u * step;
        live[u] = i < e;
        key[u] = live[u] ? (uint32_t)A.Sk[i] : 0u;
    }
    run_find4(A.T, key, live, t);
    uint4 v[4][FM_WORDS / 4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < FM_WORDS / 4; ++q)
            v[u][q] = t[u] != FM_NONE ? reinterpret_cast<const uint4*>(A.tsk + uint64_t(t[u]) * FM_WORDS)[q]
                                      : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < FM_WORDS / 4; ++q) {
            sk[4 * q] |= v[u][q].x; sk[4 * q + 1] |= v[u][q].y;
            sk[4 * q + 2] |= v[u][q].z; sk[4 * q + 3] |= v[u][q].w;
        }
}

__global__ void __launch_bounds__(FM_THREADS)
k_fm_wsketch(FmWArgs A) {
    const uint64_t nruns = *A.S.nruns;
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < nruns;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = A.S.run_start[r], e = A.S.run_start[r + 1];
        if (e - b > FM_SHORT) continue;
        uint32_t sk[FM_WORDS] = {};
        for (uint32_t i = b; i < e; i += 4) fm_w_elem4(A, i, 1, e, sk);
        fm_store(A.wsk + r * FM_WORDS, sk);
    }
}

__global__ void __launch_bounds__(FM_THREADS)
k_fm_wsketch_long(FmWArgs A) {
    const uint64_t nruns = *A.S.nruns;
    const uint64_t nw = uint64_t(gridDim.x) * (blockDim.x / WAVE);
    const int lane = lane_id();
    for (uint64_t r = blockIdx.x * (uint64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; r < nruns; r += nw) {
        const uint32_t b = A.S.run_start[r], e = A.S.run_start[r + 1];
        if (e - b <= FM_SHORT) continue;                              // wave-uniform
        uint32_t sk[FM_WORDS] = {};
        for (uint32_t i = b + lane; i < e; i += 4 * WAVE) fm_w_elem4(A, i, WAVE, e, sk);
        fm_wave_or(sk);
        if (lane == 0) fm_store(A.wsk + r * FM_WORDS, sk);
    }
}

__global__ void __launch_bounds__(FM_THREADS)
k_fm_asketch(FmAArgs A) {
    __shared__ uint32_t acc[(1u << FM_RANGE_MAX_SHIFT) * FM_WORDS];
    const uint32_t k = blockIdx.x;
    const uint64_t base = uint64_t(k) << A.a_shift;
    // ranges past a_domain only receive keys out of range (reported)
    const uint32_t span = base < A.a_domain
                              ? (uint32_t)min<uint64_t>(uint64_t(1) << A.a_shift, A.a_domain - base) : 0u;
    for (uint32_t i = threadIdx.x; i < span * FM_WORDS; i += blockDim.x) acc[i] = 0;
    __syncthreads();
    // four R tuples per thread and step, their lookups and gathers in flight together
    const uint32_t qe = A.rstarts[k + 1];
    for (uint32_t q0 = A.rstarts[k] + threadIdx.x; q0 < qe; q0 += 4 * blockDim.x) {
        uint32_t key[4], w[4], off[4];
        bool live[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t q = q0 + u * blockDim.x;
            live[u] = false;
            key[u] = off[u] = 0;
            if (q < qe) {
                const uint2 r = A.R[q];
                const uint64_t o = uint64_t(r.x) - base;
                if (r.x >= A.a_domain || o >= span) { atomicExch(A.err, 1u); continue; }
                live[u] = true;
                off[u] = (uint32_t)o;
                key[u] = mix32(r.y, A.seed);
            }
        }
        run_find4(A.S, key, live, w);                                 // b's run in S, if any
        uint4 v[4][FM_WORDS / 4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q4 = 0; q4 < FM_WORDS / 4; ++q4)
                v[u][q4] = w[u] != FM_NONE ? reinterpret_cast<const uint4*>(A.wsk + uint64_t(w[u]) * FM_WORDS)[q4]
                                           : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uint32_t* dst = acc + off[u] * FM_WORDS;
#pragma unroll
            for (int q4 = 0; q4 < FM_WORDS / 4; ++q4) {
                if (v[u][q4].x) atomicOr(dst + 4 * q4, v[u][q4].x);
                if (v[u][q4].y) atomicOr(dst + 4 * q4 + 1, v[u][q4].y);
                if (v[u][q4].z) atomicOr(dst + 4 * q4 + 2, v[u][q4].z);
                if (v[u][q4].w) atomicOr(dst + 4 * q4 + 3, v[u][q4].w);
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < span * FM_WORDS; i += blockDim.x) A.sketch[base * FM_WORDS + i] = acc[i];
    if (A.est)
        for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) A.est[base + i] = fm_estimate(acc + i * FM_WORDS);
}

__global__ void k_fm_asketch_global(FmAArgs A) {
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < A.n;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint2 r = A.R[q];
        if (r.x >= A.a_domain) { atomicExch(A.err, 1u); continue; }
        const uint32_t w = run_find(A.S, mix32(r.y, A.seed));
        if (w == FM_NONE) continue;
        for (int j = 0; j < FM_WORDS; ++j) {
            const uint32_t v = A.wsk[uint64_t(w) * FM_WORDS + j];
            if (v) atomicOr(A.sketch + uint64_t(r.x) * FM_WORDS + j, v);
        }
    }
}

__global__ void k_fm_estimate(FmAArgs A) {
    if (!A.est) return;
    for (uint64_t a = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; a < A.a_domain;
         a += (uint64_t)gridDim.x * blockDim.x)
        A.est[a] = fm_estimate(A.sketch + a * FM_WORDS);
}

}  // namespace mj
