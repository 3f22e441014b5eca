// Cascade of two binary hash joins (Sec. 6.3): the first join R(A,B) |x|
// S(B,C) materialises the intermediate I(A,C) in HBM, the second joins I
// with T on C and aggregates per A.  (The paper's I(ABC) also carries B;
// B takes no part in the second join or in the count, so I holds (a, c).)
//
//   k_cas_index  : per b-bucket i, R_i is grouped by B in LDS (counting sort
//                  written back as R_grp) and every S tuple of S_i receives
//                  its match count ecnt[s] and the start elist[s] of its list
//   k_scan_*     : exclusive scan of ecnt -> eoff (u64), |I| = eoff[|S|]
//   k_cas_expand : one workgroup per range of OUTPUT positions, so a hub key
//                  whose list is joined with thousands of S tuples is spread
//                  over many workgroups; writes I[p] = (a, c) coalesced
//   k_cas_probe  : for every (a, c) of I, count[a] += mult_T(c), probing the
//                  bucketed multiplicity tables of T (the paper's on-chip T
//                  partitions of the second join); a wave sums each run of
//                  equal a before one atomic
// I can be produced and consumed in chunks of the workspace.
#include "mj_kernels.h"

namespace mj {

__device__ __forceinline__ uint32_t cas_pass_of(uint32_t b, uint32_t seed, uint32_t level) {
    return top_bits(mix32(b, seed ^ 0x1B56C4E9u), level);
}

MJ_KERNEL(k_cas_index, CAS_THREADS, CasIndexArgs) {
    __shared__ uint32_t tkeys[CAS_CAP];
    __shared__ uint32_t tcnt[CAS_CAP];
    __shared__ uint32_t toff[CAS_CAP];
    __shared__ uint32_t wave_tmp[CAS_THREADS / WAVE + 1];
    __shared__ uint32_t s_distinct, s_over, s_spcnt, s_spoff, s_base;
    __shared__ uint32_t st_level[64], st_pass[64];
    __shared__ int s_sp;

    const uint32_t i = vg.bid;
    const uint32_t r0 = A.rstarts[i], r1 = A.rstarts[i + 1];
    const uint32_t s0 = A.sstarts[i], s1 = A.sstarts[i + 1];
    const uint32_t mask = CAS_CAP - 1;
    const int nthr = blockDim.x;
    if (r0 == r1) {                          // no R tuples: every S tuple joins nothing
        for (uint32_t q = s0 + threadIdx.x; q < s1; q += nthr) { A.ecnt[q] = 0; A.elist[q] = 0; }
        return;
    }
    if (threadIdx.x == 0) { s_sp = 1; st_level[0] = 0; st_pass[0] = 0; s_base = 0; }
    while (true) {
        __syncthreads();
        const int sp = s_sp;
        if (sp == 0) break;
        const uint32_t level = st_level[sp - 1], pass = st_pass[sp - 1];
        for (uint32_t s = threadIdx.x; s < CAS_CAP; s += nthr) { tkeys[s] = EMPTY_KEY; tcnt[s] = 0; }
        __syncthreads();
        if (threadIdx.x == 0) { s_distinct = 0; s_over = 0; s_spcnt = 0; s_sp = sp - 1; }
        __syncthreads();
        // 1. count R tuples per B value of this pass
        for (uint32_t q = r0 + threadIdx.x; q < r1; q += nthr) {
            if (*(volatile uint32_t*)&s_over) break;
            const uint32_t b = A.R[q].y;
            if (level && cas_pass_of(b, A.seed, level) != pass) continue;
            if (b == EMPTY_KEY) { atomicAdd(&s_spcnt, 1u); continue; }
            uint32_t s = slot_hash(b, A.seed) & mask;
            for (uint32_t step = 0;; ++step) {
                uint32_t cur = tkeys[s];
                if (cur == b) { atomicAdd(&tcnt[s], 1u); break; }
                if (cur == EMPTY_KEY || step >= CAS_CAP) {
                    if (*(volatile uint32_t*)&s_over || step >= CAS_CAP) { s_over = 1; break; }
                    uint32_t old = atomicCAS(&tkeys[s], EMPTY_KEY, b);
                    if (old == EMPTY_KEY || old == b) {
                        if (old == EMPTY_KEY && atomicAdd(&s_distinct, 1u) + 1 >= CAS_LIMIT) s_over = 1;
                        atomicAdd(&tcnt[s], 1u);
                        break;
                    }
                }
                s = (s + 1u) & mask;
            }
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
        // 2. list starts inside this bucket's region of R_grp
        for (uint32_t s = threadIdx.x; s < CAS_CAP; s += nthr) toff[s] = tcnt[s];
        __syncthreads();
        const uint32_t in_pass = block_exclusive_scan(toff, CAS_CAP, wave_tmp);
        const uint32_t base = s_base;
        if (threadIdx.x == 0) s_spoff = in_pass;      // the 0xFFFFFFFF list goes last
        __syncthreads();
        // 3. counting sort: A values of R into their lists
        for (uint32_t q = r0 + threadIdx.x; q < r1; q += nthr) {
            const uint2 rv = A.R[q];
            const uint32_t b = rv.y;
            if (level && cas_pass_of(b, A.seed, level) != pass) continue;
            uint32_t pos;
            if (b == EMPTY_KEY) {
                pos = atomicAdd(&s_spoff, 1u);
            } else {
                uint32_t s = slot_hash(b, A.seed) & mask;
                while (tkeys[s] != b) s = (s + 1u) & mask;
                pos = atomicAdd(&toff[s], 1u);
            }
            A.Rgrp[r0 + base + pos] = rv.x;
        }
        __syncthreads();
        // 4. each S tuple of this pass: its list (after step 3, toff[s] is the end)
        for (uint32_t q = s0 + threadIdx.x; q < s1; q += nthr) {
            const uint32_t b = A.S[q].x;
            if (level && cas_pass_of(b, A.seed, level) != pass) continue;
            uint32_t cnt = 0, start = 0;
            if (b == EMPTY_KEY) {
                cnt = s_spcnt;
                start = in_pass;
            } else {
                uint32_t s = slot_hash(b, A.seed) & mask;
                while (true) {
                    const uint32_t cur = tkeys[s];
                    if (cur == b) { cnt = tcnt[s]; start = toff[s] - cnt; break; }
                    if (cur == EMPTY_KEY) break;
                    s = (s + 1u) & mask;
                }
            }
            A.ecnt[q] = cnt;
            A.elist[q] = cnt ? r0 + base + start : 0u;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_base = base + in_pass + s_spcnt;
    }
}

// ------------------------------------------------------------- u32/u64 -> u64 scan
// out[i] = sum of in[0..i) for i in [0, n]; three launches.
template <class In>
__device__ __forceinline__ void scan_reduce(const In* in, uint64_t n, unsigned long long* partial, VGrid vg) {
    const uint64_t beg = uint64_t(vg.bid) * SCAN_TILE;
    const uint64_t end = min<uint64_t>(beg + SCAN_TILE, n);
    unsigned long long s = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += blockDim.x) s += in[i];
    s = wave_sum_u64(s);
    __shared__ unsigned long long ws[SCAN_THREADS / WAVE];
    if (lane_id() == 0) ws[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < SCAN_THREADS / WAVE; ++w) t += ws[w];
        partial[vg.bid] = t;
    }
}

MJ_KERNEL(k_scan_reduce, SCAN_THREADS, ScanArgs) { scan_reduce(A.in, A.n, A.partial, vg); }

MJ_KERNEL(k_scan_reduce64, SCAN_THREADS, Scan64Args) { scan_reduce(A.in, A.n, A.partial, vg); }

// exclusive scan of the partials in place (one block); partial[nblk] = total
MJ_KERNEL(k_scan_partials, SCAN_THREADS, ScanArgs) {
    unsigned long long* partial = A.partial;
    const uint32_t nblk = A.nblk;
    __shared__ unsigned long long carry;
    __shared__ unsigned long long ws[SCAN_THREADS / WAVE + 1];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t c0 = 0; c0 < nblk; c0 += SCAN_THREADS) {
        const uint32_t i = c0 + threadIdx.x;
        const unsigned long long x = i < nblk ? partial[i] : 0ull;
        unsigned long long v = x;
        const int lane = lane_id();
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            unsigned long long y = __shfl_up(v, off, WAVE);
            if (lane >= off) v += y;
        }
        const int w = threadIdx.x / WAVE;
        if (lane == WAVE - 1) ws[w] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long run = 0;
            for (int q = 0; q < SCAN_THREADS / WAVE; ++q) { unsigned long long t = ws[q]; ws[q] = run; run += t; }
            ws[SCAN_THREADS / WAVE] = run;
        }
        __syncthreads();
        const unsigned long long base = carry;
        if (i < nblk) partial[i] = base + ws[w] + v - x;
        __syncthreads();
        if (threadIdx.x == 0) carry = base + ws[SCAN_THREADS / WAVE];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[nblk] = carry;
}

template <class In>
__device__ __forceinline__ void scan_apply(const In* in, uint64_t n, const unsigned long long* partial,
                                           unsigned long long* out, VGrid vg) {
    __shared__ unsigned long long ws[SCAN_THREADS / WAVE + 1];
    const uint64_t beg = uint64_t(vg.bid) * SCAN_TILE;
    const uint64_t end = min<uint64_t>(beg + SCAN_TILE, n);
    unsigned long long carry = partial[vg.bid];
    for (uint64_t c0 = beg; c0 < end; c0 += SCAN_THREADS) {
        const uint64_t i = c0 + threadIdx.x;
        const unsigned long long x = i < end ? in[i] : 0ull;
        unsigned long long v = x;
        const int lane = lane_id();
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            unsigned long long y = __shfl_up(v, off, WAVE);
            if (lane >= off) v += y;
        }
        const int w = threadIdx.x / WAVE;
        if (lane == WAVE - 1) ws[w] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long run = 0;
            for (int q = 0; q < SCAN_THREADS / WAVE; ++q) { unsigned long long t = ws[q]; ws[q] = run; run += t; }
            ws[SCAN_THREADS / WAVE] = run;
        }
        __syncthreads();
        if (i < end) out[i] = carry + ws[w] + v - x;
        carry += ws[SCAN_THREADS / WAVE];
        __syncthreads();
    }
    if (vg.bid == vg.nblk - 1 && threadIdx.x == 0) out[n] = partial[vg.nblk];
}

MJ_KERNEL(k_scan_apply, SCAN_THREADS, ScanArgs) { scan_apply(A.in, A.n, A.partial, A.out, vg); }

// At most SCAN_TILE elements: the whole scan in one workgroup, one launch.
template <class In>
__device__ __forceinline__ void scan_one(const In* in, uint64_t n, unsigned long long* out) {
    __shared__ unsigned long long ws[SCAN_THREADS / WAVE + 1];
    unsigned long long carry = 0;
    for (uint64_t c0 = 0; c0 < n; c0 += SCAN_THREADS) {
        const uint64_t i = c0 + threadIdx.x;
        const unsigned long long x = i < n ? in[i] : 0ull;
        unsigned long long v = x;
        const int lane = lane_id();
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            unsigned long long y = __shfl_up(v, off, WAVE);
            if (lane >= off) v += y;
        }
        const int w = threadIdx.x / WAVE;
        if (lane == WAVE - 1) ws[w] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long run = 0;
            for (int q = 0; q < SCAN_THREADS / WAVE; ++q) { unsigned long long t = ws[q]; ws[q] = run; run += t; }
            ws[SCAN_THREADS / WAVE] = run;
        }
        __syncthreads();
        if (i < n) out[i] = carry + ws[w] + v - x;
        carry += ws[SCAN_THREADS / WAVE];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

MJ_KERNEL(k_scan_one, SCAN_THREADS, ScanArgs) { scan_one(A.in, A.n, A.out); }

MJ_KERNEL(k_scan_one64, SCAN_THREADS, Scan64Args) { scan_one(A.in, A.n, A.out); }

MJ_KERNEL(k_scan_apply64, SCAN_THREADS, Scan64Args) { scan_apply(A.in, A.n, A.partial, A.out, vg); }

// ------------------------------------------------------------- expansion
// Block b writes I positions [lo + b*EXP_TILE, ...) of the chunk [lo, hi).
MJ_KERNEL(k_cas_expand, EXP_THREADS, CasExpandArgs) {
    __shared__ uint64_t s_first, s_last;
    const unsigned long long p0 = A.lo + uint64_t(vg.bid) * EXP_TILE;
    if (p0 >= A.hi) return;
    const unsigned long long p1 = min<unsigned long long>(p0 + EXP_TILE, A.hi);
    if (threadIdx.x == 0) {
        // last s with eoff[s] <= p0, and last s with eoff[s] <= p1 - 1
        uint64_t lo = 0, hi = A.ns;           // search over eoff[0..ns)
        while (lo < hi) { uint64_t m = (lo + hi) >> 1; if (A.eoff[m] <= p0) lo = m + 1; else hi = m; }
        s_first = lo - 1;
        lo = s_first; hi = A.ns;
        while (lo < hi) { uint64_t m = (lo + hi) >> 1; if (A.eoff[m] <= p1 - 1) lo = m + 1; else hi = m; }
        s_last = lo - 1;
    }
    __syncthreads();
    const uint64_t sf = s_first, sl = s_last;
    // the tile's list starts in LDS when they fit (the usual case)
    __shared__ unsigned long long woff[EXP_WIN];
    const bool win = sl - sf < EXP_WIN;
    if (win)
        for (uint64_t k = threadIdx.x; k <= sl - sf; k += blockDim.x) woff[k] = A.eoff[sf + k];
    __syncthreads();
    const unsigned long long total = A.eoff[A.ns];
    // four positions per thread and step, their list reads in flight together
    for (unsigned long long p00 = p0 + threadIdx.x; p00 < p1; p00 += 4ull * blockDim.x) {
        uint64_t sidx[4];
        unsigned long long base[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const unsigned long long p = min<unsigned long long>(p00 + uint64_t(u) * blockDim.x, p1 - 1);
            uint64_t lo = 0, hi = sl - sf + 1;    // last s in [sf, sl] with eoff[s] <= p
            if (win) {
                while (hi - lo > 1) { uint64_t m = (lo + hi) >> 1; if (woff[m] <= p) lo = m; else hi = m; }
                base[u] = woff[lo];
            } else {
                while (hi - lo > 1) { uint64_t m = (lo + hi) >> 1; if (A.eoff[sf + m] <= p) lo = m; else hi = m; }
                base[u] = A.eoff[sf + lo];
            }
            sidx[u] = sf + lo;
        }
        uint32_t g[4], v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const unsigned long long p = min<unsigned long long>(p00 + uint64_t(u) * blockDim.x, p1 - 1);
            const bool ok = p < total;
            g[u] = ok ? A.Rgrp[A.elist[sidx[u]] + (uint32_t)(p - base[u])] : EMPTY_KEY;
            v[u] = ok ? A.S[sidx[u]].y : EMPTY_KEY;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const unsigned long long p = p00 + uint64_t(u) * blockDim.x;
            if (p >= p1) continue;
            // a position past the intermediate's end only comes with a plan
            // made for other data: marked, not joined
            A.I[p - A.lo] = A.swap ? make_uint2(v[u], g[u]) : make_uint2(g[u], v[u]);
        }
    }
}

// ------------------------------------------------------------- second join
MJ_KERNEL(k_cas_probe, 256, CasProbeArgs) {
    const int lane = lane_id();
    const bool wide = A.deg && *A.use_wide != 0;           // uniform over the launch
    const uint64_t stride = uint64_t(vg.nblk) * blockDim.x * 4;
    // the loop runs on the block's base so that every lane of a wave takes
    // part in the cross-lane steps of every round, the tail round included
    for (uint64_t q0 = uint64_t(vg.bid) * blockDim.x * 4; q0 < A.n; q0 += stride) {
        const uint64_t q = q0 + threadIdx.x;
        uint2 iv[4];
        uint32_t c[4], w[4];
        bool live[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t idx = q + uint64_t(u) * blockDim.x;
            live[u] = idx < A.n;
            iv[u] = live[u] ? A.I[idx] : make_uint2(0xFFFFFFFFu, 0u);
            c[u] = iv[u].y;
        }
        if (A.deg) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                w[u] = (live[u] && c[u] < A.c_domain) ? (wide ? A.deg[c[u]] : (uint32_t)A.deg16[c[u]]) : 0u;
        } else {
            dtab_lookup4(A.ddir, A.dpool, c, live, A.c_seed, A.c_bits, A.slot_seed, w);
        }
        // a wave holds 64 consecutive pairs per u: sum each run of equal a
        // (segments by ballot, not by value, so two runs of one a stay apart)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t a = iv[u].x;
            unsigned long long v = live[u] ? (unsigned long long)w[u] : 0ull;
            const uint32_t a_up = (uint32_t)__shfl_up((int)a, 1, WAVE);
            const bool live_up = __shfl_up((int)live[u], 1, WAVE) != 0;
            const bool head = lane == 0 || a_up != a || live_up != live[u];
            const unsigned long long heads = __ballot(head);
            const unsigned long long upto = lane == WAVE - 1 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
            const int seg = __popcll(heads & upto);
#pragma unroll
            for (int off = 1; off < WAVE; off <<= 1) {
                const unsigned long long y = __shfl_up(v, off, WAVE);
                const int sy = __shfl_up(seg, off, WAVE);
                if (lane >= off && sy == seg) v += y;
            }
            const int seg_next = __shfl_down(seg, 1, WAVE);
            const bool tail = lane == WAVE - 1 || seg_next != seg;
            if (!tail || !live[u]) continue;
            if (a >= A.a_domain) { atomicExch(A.err, 1u); continue; }
            if (v) atomicAdd(&A.count[a], v);
        }
    }
}

}  // namespace mj
