// The cyclic join of one symmetric relation without duplicates or loops
// (R = S = T = the edges of a simple graph, both directions) counted with
// every triangle once: each edge is kept in one direction only, from the
// endpoint of lower (degree, mixed id) rank to the higher one, and the
// cyclic join of R' = the kept edges reversed, S' = T' = the kept edges
//   #{ (x, y, w) : x -> y, x -> w, y -> w }
// counts every triangle exactly once, by intersecting the out-lists of x and
// y, which degree order keeps short (at most about sqrt(2m)).  The full
// join's total is six times that.  The planner checks the property
// (k_sym_check) before it offers this algorithm.
#include "mj_kernels.h"

namespace mj {

// keep[i] = 1 when edge i = (u, v) points up in (degree, mixed id) order;
// a loop, or a v that never appears as an edge's first end, means the
// relation is not what the plan certified
MJ_KERNEL(k_orient_flags, 256, OrientArgs) {
    const uint64_t stride = uint64_t(vg.nblk) * blockDim.x * 2;
    for (uint64_t q = uint64_t(vg.bid) * blockDim.x * 2 + threadIdx.x; q < A.n; q += stride) {
        uint32_t key[4], run[4];
        bool live[4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint64_t i = q + uint64_t(u) * blockDim.x;
            const bool ok = i < A.n;
            live[2 * u] = live[2 * u + 1] = ok;
            key[2 * u] = ok ? mix32(ld_col(A.c0, i, A.stride), A.seed) : 0u;
            key[2 * u + 1] = ok ? mix32(ld_col(A.c1, i, A.stride), A.seed) : 0u;
        }
        run_find4(A.U, key, live, run);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint64_t i = q + uint64_t(u) * blockDim.x;
            if (i >= A.n) continue;
            const uint32_t mu = key[2 * u], mv = key[2 * u + 1];
            const uint32_t ru = run[2 * u], rv = run[2 * u + 1];
            if (mu == mv || ru == 0xFFFFFFFFu || rv == 0xFFFFFFFFu) {
                atomicOr(A.err, 1u);
                A.flags[i] = 0;
                continue;
            }
            const uint32_t du = A.U.run_start[ru + 1] - A.U.run_start[ru];
            const uint32_t dv = A.U.run_start[rv + 1] - A.U.run_start[rv];
            A.flags[i] = (du < dv || (du == dv && mu < mv)) ? 1u : 0u;
        }
    }
}

// The same rule with vertex ids below vdom: the degrees are read from a
// direct-indexed array.  An id at or above vdom, a loop, or a v of degree 0
// (never an edge's first end) means the relation is not what the plan
// certified.
MJ_KERNEL(k_orient_flags_dense, 256, OrientArgs) {
    const uint64_t stride = uint64_t(vg.nblk) * blockDim.x * 4;
    for (uint64_t q = uint64_t(vg.bid) * blockDim.x * 4 + threadIdx.x; q < A.n; q += stride) {
        uint32_t u[4], v[4], du[4], dv[4];
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t i = q + uint64_t(k) * blockDim.x;
            const bool live = i < A.n;
            u[k] = live ? ld_col(A.c0, i, A.stride) : 0u;
            v[k] = live ? ld_col(A.c1, i, A.stride) : 0u;
            ok[k] = live && u[k] != v[k] && u[k] < A.vdom && v[k] < A.vdom;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {                 // the reads in flight together
            du[k] = ok[k] ? A.deg[u[k]] : 0u;
            dv[k] = ok[k] ? A.deg[v[k]] : 0u;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t i = q + uint64_t(k) * blockDim.x;
            if (i >= A.n) continue;
            if (!ok[k] || dv[k] == 0) {
                atomicOr(A.err, 1u);
                A.flags[i] = 0;
                continue;
            }
            const uint32_t mu = mix32(u[k], A.seed), mv = mix32(v[k], A.seed);
            A.flags[i] = (du[k] < dv[k] || (du[k] == dv[k] && mu < mv)) ? 1u : 0u;
        }
    }
}

MJ_KERNEL(k_orient_compact, 256, OrientArgs) {
    for (uint64_t i = vg.bid * (uint64_t)blockDim.x + threadIdx.x; i < A.n;
         i += (uint64_t)vg.nblk * blockDim.x) {
        if (!A.flags[i]) continue;
        A.E[A.ridx[i]] = make_uint2(ld_col(A.c0, i, A.stride), ld_col(A.c1, i, A.stride));
    }
}

// total = 6 x triangles, or all ones when the relation was not symmetric
// and simple after all (the oriented edges must be exactly half of them)
MJ_KERNEL(k_orient_finish, 64, OrientFinishArgs) {
    const OrientArgs& O = A.o;
    if (vg.bid == 0 && threadIdx.x == 0)
        *O.total = (*O.err || O.ridx[O.n] != A.expect) ? ~0ull : *O.total * 6ull;
}

// over the sorted (m(u), m(v)) and (m(v), m(u)) keys of one relation: equal
// arrays mean it is symmetric, repeats mean duplicates, equal halves loops
__global__ void __launch_bounds__(256)
k_sym_check(const unsigned long long* K1, const unsigned long long* K2, uint64_t n, uint32_t* bad) {
    bool b = false;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = K1[i];
        b = b || k != K2[i] || (uint32_t)(k >> 32) == (uint32_t)k || (i > 0 && K1[i - 1] == k);
    }
    if (b) atomicOr(bad, 1u);
}

}  // namespace mj
