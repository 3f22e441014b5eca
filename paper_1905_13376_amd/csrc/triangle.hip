// Cyclic three-way join R(A,B) |x| S(B,C) |x| T(C,A), total count (Sec. 5).
//
// Every relation is turned into 64-bit keys of mixed 32-bit values and
// sorted (radix.hip):  R -> (m(b), m(a)),  T -> (m(c), m(a)),  S -> (m(b), m(c))
// and a second copy S' -> (m(c), m(b)).  m is a bijection of the 32-bit keys,
// so equal mixed values mean equal keys and every join predicate can be
// evaluated on mixed values.  After sorting, R's tuples with one B value form
// a contiguous list ordered by m(a), and so do T's tuples with one C value.
//
// The paper keeps a partition R' of R on chip and streams S' and T' past it
// (Sec. 5.1).  Here the unit kept on chip is one relation's list for one
// join value, and every S tuple is handled once, by its shorter list:
//   * pass 1 stages R's list of b and, for the s(b, c) whose T list is
//     strictly shorter, streams T's list of c past it;
//   * pass 2 stages T's list of c and, for the remaining s (R's list not
//     longer), streams R's list of b past it.
// In each pass:
//   * k_tri_light : one wave per group whose staged list has at most
//                   TRI_LIGHT_X tuples (its LDS table maps m(a) to a
//                   multiplicity);
//   * k_tri_heavy : staged lists of hub values are cut into slices of at
//                   most TRI_HEAVY_X tuples by ranges of m(a) -- the share on
//                   A -- and the groups into ranges; one workgroup per
//                   (slice, range) streams the part of each iterated list that
//                   falls in the slice's A range.
// Work items come from device queues filled by k_tri_classify.  Each wave
// sums its counts in registers and adds them to the total once.
#include "mj_kernels.h"

namespace mj {

// --------------------------------------------------------------- key forms
MJ_KERNEL(k_tri_keys, 256, TriKeyArgs) {
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)vg.nblk * blockDim.x) {
        const uint32_t hi = ld_col(A.key_col, i, A.stride);
        const uint32_t lo = ld_col(A.val_col, i, A.stride);
        A.out[i] = ((unsigned long long)mix32(hi, A.seed) << 32) | (A.raw_low ? lo : mix32(lo, A.seed));
    }
}

// ------------------------------------------------------- runs of equal keys
// (and, when `low` is given, the low words: the joins read only those once
// the runs of the high words are indexed)
MJ_KERNEL(k_run_flags, 256, RunFlagsArgs) {
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)vg.nblk * blockDim.x) {
        const unsigned long long k = A.keys[i];
        A.flags[i] = (i == 0 || (k >> 32) != (A.keys[i - 1] >> 32)) ? 1u : 0u;
        if (A.low) A.low[i] = (uint32_t)k;
    }
}

// run r starts at element i for every head i (ridx = exclusive scan of flags)
MJ_KERNEL(k_run_compact, 256, RunCompactArgs) {
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)vg.nblk * blockDim.x) {
        if (A.flags[i]) {
            const uint64_t r = A.ridx[i];
            A.run_key[r] = (uint32_t)(A.keys[i] >> 32);
            A.run_start[r] = (uint32_t)i;
        }
    }
    if (vg.bid == 0 && threadIdx.x == 0) {
        A.run_start[A.ridx[A.n]] = (uint32_t)A.n;
        *A.nruns = A.ridx[A.n];
    }
}

// dir[p] = first run whose key prefix (top `bits` bits) is >= p, p in [0, 2^bits]
MJ_KERNEL(k_run_dir, 256, RunDirArgs) {
    const uint64_t nruns = *A.nruns;
    const uint64_t np = uint64_t(1) << A.bits;
    for (uint64_t r = vg.bid * (uint64_t)blockDim.x + threadIdx.x; r <= nruns;
         r += (uint64_t)vg.nblk * blockDim.x) {
        const uint64_t lo = r == 0 ? 0 : uint64_t(top_bits(A.run_key[r - 1], A.bits)) + 1;
        const uint64_t hi = r == nruns ? np : uint64_t(top_bits(A.run_key[r], A.bits));
        for (uint64_t p = lo; p <= hi; ++p) A.dir[p] = (uint32_t)r;
    }
}

// --------------------------------------------------------------- classify
// Light: R list of b short and S group small -> one wave.  Heavy: otherwise
// -> (slice of R's list) x (range of the S group) workgroup items, counted
// per group here and enumerated through a scan of the counts.
__device__ __forceinline__ void heavy_shape(uint32_t x, uint32_t gn, uint32_t share,
                                            uint32_t& nsl, uint32_t& nsr) {
    nsl = (x + TRI_HEAVY_X - 1) / TRI_HEAVY_X;
    nsl = max(nsl, min(share, (x + 63) / 64));
    nsr = (gn + TRI_HEAVY_S - 1) / TRI_HEAVY_S;
}

MJ_KERNEL(k_tri_classify, 256, TriClassifyArgs) {
    const uint64_t ng = *A.Grp.nruns;
    for (uint64_t g = vg.bid * (uint64_t)blockDim.x + threadIdx.x; g < ng;
         g += (uint64_t)vg.nblk * blockDim.x) {
        uint32_t rs, x;
        if (!run_lookup(A.Stg, A.Grp.run_key[g], rs, x)) continue;
        const uint32_t gn = A.Grp.run_start[g + 1] - A.Grp.run_start[g];
        if (x <= TRI_LIGHT_X && gn <= TRI_LIGHT_S) {
            const uint32_t q = atomicAdd(A.nlight, 1u);
            A.light[q] = (uint32_t)g;
        } else {
            uint32_t nsl, nsr;
            heavy_shape(x, gn, A.share, nsl, nsr);
            const uint32_t h = atomicAdd(A.nheavy_groups, 1u);
            A.heavy_group[h] = (uint32_t)g;
            A.heavy_items[h] = nsl * nsr;
        }
    }
}

// ------------------------------------------------------------ LDS A-tables
// open addressing on m(a); value = multiplicity; m(a) = 0xFFFFFFFF in `spec`
__device__ __forceinline__ void atab_add(uint32_t* keys, uint32_t* vals, uint32_t mask,
                                         uint32_t* spec, uint32_t a) {
    if (a == EMPTY_KEY) { atomicAdd(spec, 1u); return; }
    uint32_t s = a & mask;                    // m(a) is already a hash
    while (true) {
        const uint32_t cur = keys[s];
        if (cur == a) { atomicAdd(&vals[s], 1u); return; }
        if (cur == EMPTY_KEY) {
            const uint32_t old = atomicCAS(&keys[s], EMPTY_KEY, a);
            if (old == EMPTY_KEY || old == a) { atomicAdd(&vals[s], 1u); return; }
        }
        s = (s + 1u) & mask;
    }
}

__device__ __forceinline__ uint32_t atab_get(const uint32_t* keys, const uint32_t* vals,
                                             uint32_t mask, uint32_t spec, uint32_t a) {
    if (a == EMPTY_KEY) return spec;
    uint32_t s = a & mask;
    while (true) {
        const uint32_t cur = keys[s];
        if (cur == a) return vals[s];
        if (cur == EMPTY_KEY) return 0u;
        s = (s + 1u) & mask;
    }
}

// number of entries of sorted low words keys[lo, hi) equal to a
__device__ __forceinline__ uint32_t count_low(const unsigned long long* keys, uint32_t lo,
                                              uint32_t hi, uint32_t a) {
    uint32_t l = lo, h = hi;
    while (l < h) { uint32_t m = (l + h) >> 1; if ((uint32_t)keys[m] < a) l = m + 1; else h = m; }
    uint32_t l2 = l, h2 = hi;
    while (l2 < h2) { uint32_t m = (l2 + h2) >> 1; if ((uint32_t)keys[m] <= a) l2 = m + 1; else h2 = m; }
    return l2 - l;
}

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------- streaming lists
// First index in [lo, hi) of a sorted list whose value is not below v (or,
// with `upper`, above v).  The wave probes 64 evenly spaced pivots per
// round, so a list of n entries takes about log_65(n) rounds of independent
// loads instead of log_2(n) dependent ones.
__device__ __forceinline__ uint32_t wave_bound(const uint32_t* keys, uint32_t lo, uint32_t hi,
                                               uint32_t v, bool upper) {
    const int lane = lane_id();
    while (hi - lo > WAVE) {
        const uint32_t n = hi - lo;                   // n >= 65: pivots strictly increase
        const uint32_t p = lo + (uint32_t)((uint64_t)n * (lane + 1) / (WAVE + 1));
        const uint32_t k = keys[p];
        const int below = __popcll(__ballot(upper ? k <= v : k < v));
        const uint32_t nlo = below == 0 ? lo : lo + (uint32_t)((uint64_t)n * below / (WAVE + 1)) + 1;
        const uint32_t nhi = below == WAVE ? hi : lo + (uint32_t)((uint64_t)n * (below + 1) / (WAVE + 1));
        lo = nlo;
        hi = nhi;
    }
    bool in = false;
    if (lo + lane < hi) {
        const uint32_t k = keys[lo + lane];
        in = upper ? k <= v : k < v;
    }
    return lo + (uint32_t)__popcll(__ballot(in));
}

// One chunk of up to 64 S tuples of a group, lane j holding tuple si (when
// `valid`): each tuple's iterated list streams past the staged table.  Lists
// of at most TRI_SHORT_LIST entries are walked by their own lane; longer
// ones one after another by the whole wave (64 consecutive entries per load,
// UNROLL loads in flight per lane), so a long list is read with coalesced
// loads.  When the staged list is a slice, only the part of a long list in
// the slice's A range [alo, ahi] is read (a short list's other entries find
// nothing).  Returns the lane's partial sum.
__device__ __forceinline__ unsigned long long stream_chunk(const TriJoinArgs& A, uint32_t si, bool valid,
                                                           uint32_t x, const uint32_t* keys,
                                                           const uint32_t* vals, uint32_t mask, uint32_t sp,
                                                           bool sliced, uint32_t alo, uint32_t ahi) {
    const int lane = lane_id();
    constexpr int UNROLL = 4;
    unsigned long long acc = 0;
    uint32_t ts = 0, y = 0;
    if (!(valid && run_lookup(A.Itr, A.Grpl[si], ts, y)) ||
        (A.strict ? y >= x : y > x))                  // the other pass owns this s
        y = 0;
    if (y <= TRI_SHORT_LIST) {                        // UNROLL loads in flight, then their probes
        const uint32_t te = ts + y;
        for (uint32_t t0 = ts; t0 < te; t0 += UNROLL) {
            uint32_t key[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) key[u] = t0 + u < te ? A.Itrl[t0 + u] : 0u;
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
                if (t0 + u < te) acc += atab_get(keys, vals, mask, sp, key[u]);
        }
    }
    unsigned long long longm = __ballot(y > TRI_SHORT_LIST);
    while (longm) {                                   // wave-uniform
        const int j = __ffsll((long long)longm) - 1;
        longm &= longm - 1;
        uint32_t l = __shfl(ts, j, WAVE);
        uint32_t l2 = l + __shfl(y, j, WAVE);
        if (sliced && l2 - l > WAVE) {                // the part inside [alo, ahi]
            l = wave_bound(A.Itrl, l, l2, alo, false);
            l2 = wave_bound(A.Itrl, l, l2, ahi, true);
        }
        for (uint32_t t0 = l; t0 < l2; t0 += UNROLL * WAVE) {
            uint32_t key[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const uint32_t t = t0 + u * WAVE + lane;
                key[u] = t < l2 ? A.Itrl[t] : 0u;
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
                if (t0 + u * WAVE + lane < l2) acc += atab_get(keys, vals, mask, sp, key[u]);
        }
    }
    return acc;
}

// ------------------------------------------------------------- light groups
// One wave, one S group: R's list of b into the wave's LDS table, then every
// s(b,c) of the group streams T's list of c past it, 64 tuples at a time
// (stream_chunk).  Returns the lane's sum.
struct WaveTable {
    uint32_t* keys;
    uint32_t* vals;
    uint16_t* used;                   // slots taken (< TRI_LIGHT_CAP), for the clean-up
    uint32_t* nused;
    uint32_t* spec;
};

__device__ unsigned long long tri_light_group(const TriJoinArgs& A, uint32_t g, const WaveTable& W) {
    const int lane = lane_id();
    const uint32_t mask = TRI_LIGHT_CAP - 1;
    const uint32_t gkey = A.Grp.run_key[g];
    const uint32_t gs = A.Grp.run_start[g], ge = A.Grp.run_start[g + 1];
    uint32_t rs = 0, x = 0;
    run_lookup(A.Stg, gkey, rs, x);
    for (uint32_t q = lane; q < x; q += WAVE) {
        const uint32_t a = A.Stgl[rs + q];
        if (a == EMPTY_KEY) { atomicAdd(W.spec, 1u); continue; }
        uint32_t s = a & mask;
        while (true) {
            const uint32_t cur = W.keys[s];
            if (cur == a) { atomicAdd(&W.vals[s], 1u); break; }
            if (cur == EMPTY_KEY) {
                const uint32_t old = atomicCAS(&W.keys[s], EMPTY_KEY, a);
                if (old == EMPTY_KEY) { W.used[atomicAdd(W.nused, 1u)] = (uint16_t)s; atomicAdd(&W.vals[s], 1u); break; }
                if (old == a) { atomicAdd(&W.vals[s], 1u); break; }
            }
            s = (s + 1u) & mask;
        }
    }
    wave_fence();
    const uint32_t spec = *W.spec;
    unsigned long long acc = 0;
    for (uint32_t c0 = gs; c0 < ge; c0 += WAVE)
        acc += stream_chunk(A, c0 + lane, c0 + lane < ge, x, W.keys, W.vals, mask, spec, false, 0u, 0u);
    wave_fence();
    const uint32_t nu = *W.nused;
    for (uint32_t q = lane; q < nu; q += WAVE) { const uint32_t s = W.used[q]; W.keys[s] = EMPTY_KEY; W.vals[s] = 0; }
    wave_fence();
    if (lane == 0) { *W.spec = 0; *W.nused = 0; }
    wave_fence();
    return acc;
}

#define TRI_LIGHT_SETUP                                                              \
    constexpr int NW = TRI_THREADS / WAVE;                                           \
    __shared__ uint32_t tkeys[NW][TRI_LIGHT_CAP];                                    \
    __shared__ uint32_t tvals[NW][TRI_LIGHT_CAP];                                    \
    __shared__ uint16_t tused[NW][TRI_LIGHT_X];                                      \
    __shared__ uint32_t tnused[NW];                                                  \
    __shared__ uint32_t tspec[NW];                                                   \
    const int w = threadIdx.x / WAVE, lane = lane_id();                              \
    WaveTable W{tkeys[w], tvals[w], tused[w], &tnused[w], &tspec[w]};                \
    for (uint32_t s = lane; s < TRI_LIGHT_CAP; s += WAVE) { W.keys[s] = EMPTY_KEY; W.vals[s] = 0; } \
    if (lane == 0) { *W.spec = 0; *W.nused = 0; }                                    \
    wave_fence();

// Light items are taken a run at a time: the queue counter is one address,
// whose atomics are served one after another (about 12 ns each), so one
// atomic per item bounded the kernel once items numbered in the millions,
// and each atomic's round trip also stalls the wave that waits for it.  A
// run is a quarter of a wave's fair share, at least TRI_LIGHT_GRAB_MIN and
// at most TRI_LIGHT_GRAB items.
constexpr uint32_t TRI_LIGHT_GRAB = 16, TRI_LIGHT_GRAB_MIN = 4;

__device__ __forceinline__ uint32_t light_grab(unsigned long long nitems, unsigned long long waves) {
    const unsigned long long g = nitems / (4ull * waves);
    return (uint32_t)(g < TRI_LIGHT_GRAB_MIN ? TRI_LIGHT_GRAB_MIN : (g > TRI_LIGHT_GRAB ? TRI_LIGHT_GRAB : g));
}

MJ_KERNEL(k_tri_light, TRI_THREADS, TriJoinArgs) {
    TRI_LIGHT_SETUP
    const uint32_t nitems = *A.nlight;
    const uint32_t grab = light_grab(nitems, (unsigned long long)vg.nblk * (TRI_THREADS / WAVE));
    unsigned long long acc = 0;
    uint32_t it = 0, end = 0;
    while (true) {
        if (it >= end) {                              // wave-uniform
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(A.light_next, grab);
            it = __shfl(t, 0, WAVE);
            if (it >= nitems) break;
            end = min(it + grab, nitems);
        }
        acc += tri_light_group(A, A.light[it], W);
        ++it;
    }
    acc = wave_sum_u64(acc);
    if (lane == 0 && acc) atomicAdd(A.total, acc);
}

// ------------------------------------------------------------- heavy groups
// One workgroup, one item: a slice of a hub's R list into LDS, then the
// item's S tuples, one wave per S tuple, stream the slice's A range of T's list.
struct BlockTable {
    uint32_t* keys;
    uint32_t* vals;
    uint32_t* spec;
    uint32_t* chunk;                  // next chunk of 64 S tuples of the item
};

// One workgroup, one item: a slice of a staged list into LDS, then the
// item's S tuples stream their iterated lists past it (only the part in the
// slice's A range when the staged list is sliced).  Waves take chunks of 64
// S tuples from a workgroup counter and lane j looks up tuple j's list; lists of at most
// TRI_SHORT_LIST entries are then walked by their own lane, longer ones one
// after another by the whole wave (64 consecutive entries per load, several
// loads in flight per lane).
__device__ unsigned long long tri_heavy_item(const TriJoinArgs& A, uint32_t it, const BlockTable& B) {
    const int lane = lane_id();
    const uint32_t mask = TRI_HEAVY_CAP - 1;
    // item -> (heavy group, slice of the staged list, range of the group)
    uint32_t lo = 0, hi = A.n_heavy_cap;              // last h with off[h] <= it
    while (hi - lo > 1) { uint32_t m = (lo + hi) >> 1; if (A.heavy_off[m] <= it) lo = m; else hi = m; }
    const uint32_t g = A.heavy_group[lo];
    const uint32_t local = (uint32_t)(it - A.heavy_off[lo]);
    uint32_t rs = 0, x = 0;
    run_lookup(A.Stg, A.Grp.run_key[g], rs, x);
    const uint32_t gs = A.Grp.run_start[g], gn = A.Grp.run_start[g + 1] - gs;
    uint32_t nsl, nsr;
    heavy_shape(x, gn, A.share, nsl, nsr);
    const uint32_t sa = local / nsr, sb = local % nsr;
    TriHeavyItem H;
    H.r0 = rs + (uint32_t)((uint64_t)x * sa / nsl);
    H.r1 = rs + (uint32_t)((uint64_t)x * (sa + 1) / nsl);
    H.s0 = gs + sb * TRI_HEAVY_S;
    H.s1 = min(gs + gn, H.s0 + TRI_HEAVY_S);
    unsigned long long acc = 0;
    if (H.r0 == H.r1) return 0;                       // uniform across the block
    for (uint32_t q = H.r0 + threadIdx.x; q < H.r1; q += blockDim.x)
        atab_add(B.keys, B.vals, mask, B.spec, A.Stgl[q]);
    __syncthreads();
    const uint32_t sp = *B.spec;
    const bool sliced = nsl > 1;
    const uint32_t alo = A.Stgl[H.r0], ahi = A.Stgl[H.r1 - 1];
    while (true) {
        uint32_t c = 0;
        if (lane == 0) c = atomicAdd(B.chunk, 1u);
        const uint32_t c0 = H.s0 + __shfl(c, 0, WAVE) * WAVE;
        if (c0 >= H.s1) break;                        // wave-uniform
        const uint32_t si = c0 + lane;
        acc += stream_chunk(A, si, si < H.s1, x, B.keys, B.vals, mask, sp, sliced, alo, ahi);
    }
    return acc;
}

#define TRI_HEAVY_SETUP                                                   \
    __shared__ uint32_t hkeys[TRI_HEAVY_CAP];                             \
    __shared__ uint32_t hvals[TRI_HEAVY_CAP];                             \
    __shared__ uint32_t hspec;                                            \
    __shared__ uint32_t hchunk;                                           \
    __shared__ uint32_t s_item;                                           \
    BlockTable B{hkeys, hvals, &hspec, &hchunk};                          \
    const int lane = lane_id();

MJ_KERNEL(k_tri_heavy, TRI_HEAVY_THREADS, TriJoinArgs) {
    (void)vg;
    TRI_HEAVY_SETUP
    const uint32_t nitems = (uint32_t)A.heavy_off[A.n_heavy_cap];
    unsigned long long acc = 0;
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) { s_item = atomicAdd(A.heavy_next, 1u); hspec = 0; hchunk = 0; }
        for (uint32_t s = threadIdx.x; s < TRI_HEAVY_CAP; s += blockDim.x) { hkeys[s] = EMPTY_KEY; hvals[s] = 0; }
        __syncthreads();
        const uint32_t it = s_item;
        if (it >= nitems) break;
        acc += tri_heavy_item(A, it, B);
    }
    acc = wave_sum_u64(acc);
    if (lane == 0 && acc) atomicAdd(A.total, acc);
}

// ------------------------------------------------------------- batches
// Every cyclic join of a batch prepared its own queues; one persistent
// launch serves all of them.  Global item k -> (join j, local item) through
// the exclusive prefix of the per-join item counts.
__device__ __forceinline__ uint32_t batch_join_of(const unsigned long long* base, uint32_t njoins,
                                                  unsigned long long k) {
    uint32_t lo = 0, hi = njoins;                     // last j with base[j] <= k
    while (hi - lo > 1) { uint32_t m = (lo + hi) >> 1; if (base[m] <= k) lo = m; else hi = m; }
    return lo;
}

__global__ void __launch_bounds__(TRI_THREADS)
k_tri_light_batch(TriBatchArgs Bt) {
    TRI_LIGHT_SETUP
    const unsigned long long nitems = Bt.light_base[Bt.njoins];
    const unsigned long long grab = light_grab(nitems, (unsigned long long)gridDim.x * (TRI_THREADS / WAVE));
    unsigned long long it = 0, end = 0, acc = 0;
    uint32_t cur = 0;                                 // the join whose count acc holds
    while (true) {
        if (it >= end) {                              // wave-uniform
            unsigned long long t = 0;
            if (lane == 0) t = atomicAdd(Bt.next, grab);
            it = __shfl(t, 0, WAVE);
            if (it >= nitems) break;
            end = min(it + grab, nitems);
        }
        const uint32_t j = batch_join_of(Bt.light_base, Bt.njoins, it);
        if (j != cur) {                               // a run may span joins: add the last one's count
            acc = wave_sum_u64(acc);
            if (lane == 0 && acc) atomicAdd(Bt.joins[cur].total, acc);
            acc = 0;
            cur = j;
        }
        const TriJoinArgs& A = Bt.joins[j];
        acc += tri_light_group(A, A.light[it - Bt.light_base[j]], W);
        ++it;
    }
    acc = wave_sum_u64(acc);
    if (lane == 0 && acc) atomicAdd(Bt.joins[cur].total, acc);
}

__global__ void __launch_bounds__(TRI_HEAVY_THREADS)
k_tri_heavy_batch(TriBatchArgs Bt) {
    TRI_HEAVY_SETUP
    __shared__ unsigned long long s_bitem;
    __shared__ unsigned long long s_sum;
    const unsigned long long nitems = Bt.heavy_base[Bt.njoins];
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) { s_bitem = atomicAdd(Bt.next + 1, 1ull); hspec = 0; hchunk = 0; s_sum = 0; }
        for (uint32_t s = threadIdx.x; s < TRI_HEAVY_CAP; s += blockDim.x) { hkeys[s] = EMPTY_KEY; hvals[s] = 0; }
        __syncthreads();
        const unsigned long long it = s_bitem;
        if (it >= nitems) break;
        const uint32_t j = batch_join_of(Bt.heavy_base, Bt.njoins, it);
        const TriJoinArgs& A = Bt.joins[j];
        unsigned long long acc = tri_heavy_item(A, (uint32_t)(it - Bt.heavy_base[j]), B);
        acc = wave_sum_u64(acc);
        if (lane == 0 && acc) atomicAdd(&s_sum, acc);
        __syncthreads();
        if (threadIdx.x == 0 && s_sum) atomicAdd(A.total, s_sum);
    }
    (void)s_item;
}

// per-join item counts of a batch -> exclusive prefixes (one block)
__global__ void k_tri_batch_prefix(TriBatchArgs Bt) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long l = 0, h = 0;
    for (uint32_t j = 0; j < Bt.njoins; ++j) {
        Bt.light_base[j] = l;
        Bt.heavy_base[j] = h;
        l += *Bt.joins[j].nlight;
        h += Bt.joins[j].heavy_off[Bt.joins[j].n_heavy_cap];
    }
    Bt.light_base[Bt.njoins] = l;
    Bt.heavy_base[Bt.njoins] = h;
    Bt.next[0] = 0;
    Bt.next[1] = 0;
}

// ----------------------------------------------- cascade, cyclic second join
// For every (a, c) of I = R |x| S: the multiplicity of (c, a) in T, found in
// T's sorted list of m(c) by binary search on m(a).
MJ_KERNEL(k_cas_probe_tri, 256, CasProbeTriArgs) {
    unsigned long long acc = 0;
    for (uint64_t q = vg.bid * (uint64_t)blockDim.x + threadIdx.x; q < A.n;
         q += (uint64_t)vg.nblk * blockDim.x) {
        const uint2 iv = A.I[q];
        uint32_t ts, y;
        if (!run_lookup(A.T, mix32(iv.y, A.seed), ts, y)) continue;
        acc += count_low(A.Tk, ts, ts + y, mix32(iv.x, A.seed));
    }
    acc = wave_sum_u64(acc);
    if (lane_id() == 0 && acc) atomicAdd(A.total, acc);
}

}  // namespace mj
