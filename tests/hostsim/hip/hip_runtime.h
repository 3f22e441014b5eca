// Host build of libmj's kernels (test infrastructure only).
//
// This header stands in for <hip/hip_runtime.h> when the library's sources
// are compiled for the CPU by tests/hostsim/build.py.  It is never used by
// the product: libmj.so is built by hipcc for gfx950 only, and the Python
// package loads nothing else.  The host build exists to run the kernels
// under AddressSanitizer / UndefinedBehaviorSanitizer, so that an access
// outside a buffer, a read of memory no kernel wrote, or a deadlock at a
// barrier is reported with its kernel and source line.
//
// Execution model emulated (the parts of it the kernels use):
//   - a workgroup's threads are fibers on one OS thread; __syncthreads()
//     waits for every thread of the workgroup that has not returned;
//   - a wavefront is 64 consecutive threads; every cross-lane operation
//     (__shfl*, __ballot) is a rendezvous of the wave's live lanes;
//   - __shared__ variables are per-OS-thread statics (one workgroup runs on
//     an OS thread at a time), dynamic LDS is a per-workgroup buffer;
//   - workgroups of one launch run on a pool of OS threads, launches run to
//     completion in order (streams and events are ordered trivially).
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <type_traits>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
#define __shared__ static thread_local
#define __restrict__ __restrict
#define __align__(n) __attribute__((aligned(n)))
// merged launches' argument tables are plain memory on the host
#define MJ_CONSTANT_AS

struct dim3 {
    uint32_t x, y, z;
    constexpr dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};

struct __attribute__((aligned(8))) uint2 { uint32_t x, y; };
struct __attribute__((aligned(16))) uint4 { uint32_t x, y, z, w; };
struct __attribute__((aligned(8))) int2 { int32_t x, y; };
struct __attribute__((aligned(16))) ulonglong2 { unsigned long long x, y; };
struct __attribute__((aligned(16))) ulonglong4 { unsigned long long x, y, z, w; };
inline ulonglong2 make_ulonglong2(unsigned long long a, unsigned long long b) { return ulonglong2{a, b}; }
inline ulonglong4 make_ulonglong4(unsigned long long a, unsigned long long b, unsigned long long c,
                                  unsigned long long d) { return ulonglong4{a, b, c, d}; }
struct __attribute__((aligned(8))) float2 { float x, y; };
struct __attribute__((aligned(16))) float4 { float x, y, z, w; };
inline uint2 make_uint2(uint32_t a, uint32_t b) { return uint2{a, b}; }
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return uint4{a, b, c, d}; }
inline int2 make_int2(int32_t a, int32_t b) { return int2{a, b}; }
inline float2 make_float2(float a, float b) { return float2{a, b}; }

namespace hipsim {

struct ThreadIdx { uint32_t x, y, z; };

// the fiber (GPU thread) running on this OS thread
struct Lane;
extern thread_local Lane* cur;
const ThreadIdx& thread_idx();
const dim3& block_idx();
const dim3& block_dim();
const dim3& grid_dim();
unsigned lane();
void* dyn_smem();
void syncthreads();
uint64_t wave_exchange(uint64_t v, int op, int arg, int width);   // op: see sim.cpp
enum { OP_SHFL = 0, OP_UP = 1, OP_DOWN = 2, OP_XOR = 3, OP_BALLOT = 4 };

void launch(const char* name, dim3 grid, dim3 block, size_t smem, const std::function<void()>& body);

template <class T>
inline uint64_t to_bits(T v) {
    static_assert(sizeof(T) <= 8, "shuffle of a value wider than 64 bits");
    uint64_t b = 0;
    memcpy(&b, &v, sizeof(T));
    return b;
}
template <class T>
inline T from_bits(uint64_t b) {
    T v;
    memcpy(&v, &b, sizeof(T));
    return v;
}

}  // namespace hipsim

#define threadIdx (::hipsim::thread_idx())
#define blockIdx (::hipsim::block_idx())
#define blockDim (::hipsim::block_dim())
#define gridDim (::hipsim::grid_dim())

inline unsigned __lane_id() { return ::hipsim::lane(); }
inline void __syncthreads() { ::hipsim::syncthreads(); }
inline void __threadfence() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }
// the device's scoped fence builtin: a fence of the given order on the host
#define __builtin_amdgcn_fence(order, scope) __atomic_thread_fence(order)
// the wave's lanes meet (a ballot is a rendezvous of the wave's live lanes)
#define __builtin_amdgcn_wave_barrier() ((void)::hipsim::wave_exchange(0, ::hipsim::OP_BALLOT, 0, 64))
#define __builtin_amdgcn_fence(...) __atomic_thread_fence(__ATOMIC_SEQ_CST)

template <class T>
inline T __shfl(T v, int src, int width = 64) {
    return ::hipsim::from_bits<T>(::hipsim::wave_exchange(::hipsim::to_bits(v), ::hipsim::OP_SHFL, src, width));
}
template <class T>
inline T __shfl_up(T v, unsigned d, int width = 64) {
    return ::hipsim::from_bits<T>(::hipsim::wave_exchange(::hipsim::to_bits(v), ::hipsim::OP_UP, (int)d, width));
}
template <class T>
inline T __shfl_down(T v, unsigned d, int width = 64) {
    return ::hipsim::from_bits<T>(::hipsim::wave_exchange(::hipsim::to_bits(v), ::hipsim::OP_DOWN, (int)d, width));
}
template <class T>
inline T __shfl_xor(T v, int m, int width = 64) {
    return ::hipsim::from_bits<T>(::hipsim::wave_exchange(::hipsim::to_bits(v), ::hipsim::OP_XOR, m, width));
}
inline unsigned long long __ballot(int pred) {
    return ::hipsim::wave_exchange(pred ? 1u : 0u, ::hipsim::OP_BALLOT, 0, 64);
}

inline int __popc(unsigned x) { return __builtin_popcount(x); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __clz(int x) { return x == 0 ? 32 : __builtin_clz((unsigned)x); }
inline int __clzll(long long x) { return x == 0 ? 64 : __builtin_clzll((unsigned long long)x); }
inline int __ffs(int x) { return __builtin_ffs(x); }
inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }

// min / max: the device library's overloads and templates
template <class T>
inline T min(T a, T b) { return a < b ? a : b; }
template <class T>
inline T max(T a, T b) { return a < b ? b : a; }
template <class A, class B>
inline typename std::common_type<A, B>::type min(A a, B b) {
    typedef typename std::common_type<A, B>::type C;
    return (C)a < (C)b ? (C)a : (C)b;
}
template <class A, class B>
inline typename std::common_type<A, B>::type max(A a, B b) {
    typedef typename std::common_type<A, B>::type C;
    return (C)a < (C)b ? (C)b : (C)a;
}

inline float __uint_as_float(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
inline uint32_t __float_as_uint(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
inline float __int_as_float(int32_t u) { float f; memcpy(&f, &u, 4); return f; }
inline int32_t __float_as_int(float f) { int32_t u; memcpy(&u, &f, 4); return u; }

// atomics (global and LDS memory alike)
template <class T>
inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
inline float atomicAdd(float* p, float v) {
    float old = *p;
    while (!__atomic_compare_exchange(p, &old, (float[]){old + v}, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {}
    return old;
}
template <class T>
inline T atomicOr(T* p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_RELAXED); }
template <class T>
inline T atomicAnd(T* p, T v) { return __atomic_fetch_and(p, v, __ATOMIC_RELAXED); }
template <class T>
inline T atomicExch(T* p, T v) { return __atomic_exchange_n(p, v, __ATOMIC_RELAXED); }
template <class T>
inline T atomicMax(T* p, T v) {
    T old = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (old < v && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {}
    return old;
}
template <class T>
inline T atomicMin(T* p, T v) {
    T old = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (v < old && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {}
    return old;
}
template <class T>
inline T atomicCAS(T* p, T cmp, T v) {
    __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
    return cmp;
}

// ------------------------------------------------------------ runtime API
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorNotReady = 600 };
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
enum hipStreamCaptureStatus { hipStreamCaptureStatusNone = 0, hipStreamCaptureStatusActive = 1 };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
enum { hipStreamDefault = 0, hipStreamNonBlocking = 1 };
enum { hipEventDefault = 0, hipEventDisableTiming = 2 };
enum { hipHostMallocDefault = 0 };

struct hipDeviceProp_t {
    char name[256];
    int multiProcessorCount;
    size_t sharedMemPerBlock;
    size_t totalGlobalMem;
};

hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags = 0);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s = nullptr);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t s = nullptr);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetDevice(int* d);
hipError_t hipSetDevice(int d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute a, int v);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus* st);
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol);
#define HIP_SYMBOL(x) reinterpret_cast<const void*>(&(x))

#define hipLaunchKernelGGL(kern, grid, block, smem, stream, ...) \
    ::hipsim::launch(#kern, dim3(grid), dim3(block), (size_t)(smem), [&]() { kern(__VA_ARGS__); })
