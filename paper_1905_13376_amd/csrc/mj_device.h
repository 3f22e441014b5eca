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

}  // namespace mj
