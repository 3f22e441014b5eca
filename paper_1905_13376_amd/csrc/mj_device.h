// Device-side building blocks shared by the libmj kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mj {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;
constexpr uint32_t EMPTY_KEY = 0xFFFFFFFFu;   // LDS/global table sentinel; the real
                                              // key 0xFFFFFFFF is kept in a side slot

// 32-bit finaliser of MurmurHash3 applied to key ^ seed: a bijection of the
// 32-bit keys, so distinct keys never collide in the full hash value.  The
// paper asks only for "robust" hash functions (Sec. 4); bucket numbers are
// the top bits (radix digits of the hash), table slots the low bits.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t k, uint32_t seed) {
    uint32_t h = k ^ seed;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Bucket from the top `bits` bits of a hash (bits may be 0: one bucket).
__host__ __device__ __forceinline__ uint32_t top_bits(uint32_t h, uint32_t bits) {
    return bits == 0 ? 0u : (bits >= 32 ? h : (h >> (32u - bits)));
}

// Second, independent hash for table slots inside a bucket.
__host__ __device__ __forceinline__ uint32_t slot_hash(uint32_t k, uint32_t seed) {
    return mix32(k, seed ^ 0x68E31DA4u);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Workgroups of a launch are handed to the 8 XCDs of the chip in turn
// (block b runs on XCD b % 8), and each XCD has its own L2.  xcd_remap maps
// the launch order onto a work index so that every XCD receives one
// contiguous range of work items: neighbouring items (adjacent output runs,
// shared table regions) then meet in the same L2.  It is a bijection on
// [0, n) for any n; only locality depends on the hardware's hand-out order.
constexpr uint32_t NUM_XCD = 8;
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t n) {
    const uint32_t x = b % NUM_XCD, local = b / NUM_XCD;
    const uint32_t per = n / NUM_XCD, tall = n % NUM_XCD;   // first `tall` XCDs get per + 1
    return x < tall ? x * (per + 1) + local : tall * (per + 1) + (x - tall) * per + local;
}

// Wave-wide sum of a 64-bit value (a butterfly of cross-lane permutes,
// __shfl_xor, six steps).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) { return wave_sum_u64(v); }
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return wave_sum_u32(v); }

// Heavy keys: the active lanes of the wave whose key equals the first
// active lane's key fold their values into that lane, which then adds the
// sum once (a hub's tuples cost one atomic per wave instead of one per
// lane).  Every lane of the wave must call it.  Returns true for a lane
// whose value was folded into another (it skips its own add); the first
// lane's v becomes the sum.  With fewer than two such lanes nothing changes.
template <class T>
__device__ __forceinline__ bool wave_fold_first(uint32_t key, bool act, T& v) {
    const unsigned long long live = __ballot(act);
    if (live == 0) return false;                                   // uniform over the wave
    const int first = __ffsll((long long)live) - 1;
    const uint32_t k0 = __shfl(key, first, WAVE);
    const bool same = act && key == k0;
    if (__popcll(__ballot(same)) < 2) return false;                // uniform over the wave
    const T sum = wave_sum(same ? v : T(0));
    if (!same) return false;
    if (lane_id() == first) { v = sum; return false; }
    return true;
}

// Hand-off between workgroups through a ticket atomic (the last of a
// bucket's pieces adds up the others' rows): the writers' release makes
// their stores visible at device scope before their ticket add, and the
// last workgroup's acquire after its ticket add makes them visible to its
// loads.  Each XCD has its own L2: the release writes the XCD's dirty lines
// back, the acquire invalidates the XCD's L2, so the writers do only the
// former (a full fence in every piece also threw away the gathered arrays
// the other workgroups of its XCD were reading).
__device__ __forceinline__ void handoff_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void handoff_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Read tuple component from a strided column.
__device__ __forceinline__ uint32_t ld_col(const uint32_t* __restrict__ col, uint64_t i,
                                           int64_t stride) {
    return __builtin_nontemporal_load(col + i * (uint64_t)stride);
}

__device__ __forceinline__ unsigned long long atomic_add_u64(unsigned long long* p,
                                                             unsigned long long v) {
    return atomicAdd(p, v);
}

// Block-wide exclusive scan of lds[0..n), in place; returns the total.
// All threads of the block must call it.
__device__ inline uint32_t block_exclusive_scan(uint32_t* lds, uint32_t n, uint32_t* wave_tmp) {
    const uint32_t t = threadIdx.x;
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t b = min(n, t * per), e = min(n, b + per);
    uint32_t s = 0;
    for (uint32_t i = b; i < e; ++i) s += lds[i];
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

// ----------------------------------------------------------- merged launches
// Launches of one kernel, each with its own argument struct and grid, can
// run as one grid: `base` holds each launch's first block, a workgroup finds
// its launch by a search over it, and the kernel's body sees that launch's
// block index and grid size in a VGrid.  Kernels written with MJ_KERNEL read
// their block index and grid size only from there, so that they compute the
// same alone and merged.
struct VGrid { uint32_t bid, nblk; };
struct MultiGrid {
    const void* args;        // [njobs] argument structs of the kernel's type
    const uint32_t* base;    // [njobs + 1] first block of each launch; base[njobs] = the grid
    uint32_t njobs;
};

// The launch holding block b: the last j with base[j] <= b (every launch has
// at least one block, so base increases).  Each round compares one entry per
// lane and keeps the segment of the last lane whose entry is at most b: two
// rounds for up to 4096 launches.  Every lane of the wave calls it, at the
// kernel's start, with the same b; the result is the same in every lane.
__device__ inline uint32_t multi_job(const MultiGrid& M, uint32_t b) {
    const uint32_t nl = (uint32_t)__popcll(__ballot(1));   // the wave's lanes (the low ones)
    const uint32_t lane = lane_id();
    uint32_t lo = 0, hi = M.njobs;
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + nl - 1) / nl;
        const uint32_t k = lo + lane * step;
        const unsigned long long bal = __ballot(k < hi && M.base[k] <= b);
        lo += (uint32_t)(63 - __clzll((long long)bal)) * step;   // lane 0's entry always qualifies
        hi = min(hi, lo + step);
    }
    return lo;
}

// Launch j's argument struct.  The table is not written while the kernel
// runs, so it is read as constant memory (like a kernel's own arguments):
// uniform loads of its fields, also at indices known only at run time.
#ifndef MJ_CONSTANT_AS
#define MJ_CONSTANT_AS __attribute__((address_space(4)))
#endif
template <class Args>
__device__ __forceinline__ const Args& merged_args(const void* table, uint32_t j) {
    const MJ_CONSTANT_AS Args* t = (const MJ_CONSTANT_AS Args*)table;
    return *(const Args*)(t + j);
}

}  // namespace mj

// A kernel that runs alone (`name`, its grid is the launch's) or merged with
// other launches of itself (`name##_multi`, one MultiGrid argument).  The
// body follows the macro; it names its argument struct A and its grid vg.
// Alone, the body takes the struct by value (the kernel's own argument, so
// the code is that of a plain kernel); merged, by reference into the
// constant table (a private copy would put an indexed array of the struct in
// scratch memory).
#define MJ_KERNEL(name, T, Args)                                                            \
    template <class P_>                                                                     \
    __device__ __forceinline__ void name##_body(P_ A, ::mj::VGrid vg);                      \
    __global__ void __launch_bounds__(T) name(Args A) {                                     \
        name##_body<const Args>(A, ::mj::VGrid{blockIdx.x, gridDim.x});                     \
    }                                                                                       \
    __global__ void __launch_bounds__(T) name##_multi(::mj::MultiGrid M) {                  \
        const uint32_t j_ = ::mj::multi_job(M, blockIdx.x);                                 \
        name##_body<const Args&>(::mj::merged_args<Args>(M.args, j_),                       \
                                 ::mj::VGrid{blockIdx.x - M.base[j_], M.base[j_ + 1] - M.base[j_]}); \
    }                                                                                       \
    template <class P_>                                                                     \
    __device__ __forceinline__ void name##_body(P_ A, ::mj::VGrid vg)

// Declarations of both forms, and the name of the argument struct.
#define MJ_KERNEL_DECL(name, Args)    \
    typedef Args name##_args;         \
    __global__ void name(Args A);     \
    __global__ void name##_multi(::mj::MultiGrid M)
