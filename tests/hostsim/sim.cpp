// Host build of libmj's kernels (test infrastructure only): the fiber
// scheduler that runs a workgroup's threads, the wave rendezvous behind the
// cross-lane operations, and the runtime calls the library's host code
// makes.  See hip/hip_runtime.h in this directory for the model.
#include "hip/hip_runtime.h"

#include <sys/mman.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define HIPSIM_ASAN 1
#endif
#endif
#ifdef HIPSIM_ASAN
#include <sanitizer/asan_interface.h>
#endif

extern "C" void hipsim_switch(void** save_sp, void* new_sp);
// x86-64 System V: save the callee-saved registers on the old stack, switch
// stacks, restore them from the new one.
asm(R"(
.text
.globl hipsim_switch
.type hipsim_switch,@function
hipsim_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
.size hipsim_switch, .-hipsim_switch
)");

namespace hipsim {

namespace {

constexpr size_t STACK_BYTES = 256 * 1024;
constexpr int MAX_THREADS = 1024;
constexpr int WAVE = 64;

enum State { RUNNABLE = 0, AT_BARRIER = 1, AT_WAVE = 2, DONE = 3 };

struct Wave {
    int live = 0;
    int arrived[2] = {0, 0};
    uint64_t val[2][WAVE];
    uint64_t seq[2][WAVE];
};

struct Worker;

}  // namespace

struct Lane {
    void* sp = nullptr;
    char* stack = nullptr;
    ThreadIdx tidx{};
    uint32_t tid = 0;
    int state = RUNNABLE;
    uint64_t seq = 0;          // cross-lane operations done so far
    Worker* w = nullptr;
};

namespace {

struct Launch {
    const char* name;
    dim3 grid, block;
    size_t smem;
    const std::function<void()>* body;
    std::atomic<uint64_t> next{0};
    uint64_t nblocks;
};

struct Worker {
    std::vector<Lane> lanes;
    std::vector<Wave> waves;
    void* sched_sp = nullptr;
    dim3 bidx;
    char* dyn = nullptr;
    int live = 0;
    int at_barrier = 0;
    Launch* L = nullptr;
    std::thread th;
};

thread_local Worker* tw = nullptr;
std::atomic<int> g_error{0};
std::string g_last_kernel;

[[noreturn]] void die(const char* what) {
    std::fprintf(stderr, "hipsim: %s (kernel %s)\n", what, tw && tw->L ? tw->L->name : "?");
    std::fflush(stderr);
    std::abort();
}

void to_scheduler(Lane* l) {
    Worker* w = l->w;
    hipsim_switch(&l->sp, w->sched_sp);
}

void lane_entry() {
    Lane* l = cur;
    (*l->w->L->body)();
    l->state = DONE;
    Worker* w = l->w;
    w->live -= 1;
    Wave& wv = w->waves[l->tid / WAVE];
    wv.live -= 1;
    to_scheduler(l);
    die("a finished lane was resumed");
}

void* init_stack(Lane& l) {
#ifdef HIPSIM_ASAN
    // the frames a finished lane left (its entry and the switch) lie near the
    // top of its stack; deeper frames returned and cleared their own marks
    __asan_unpoison_memory_region(l.stack + STACK_BYTES - 16384, 16384);
#endif
    uintptr_t top = (reinterpret_cast<uintptr_t>(l.stack) + STACK_BYTES) & ~uintptr_t(15);
    uintptr_t* sp = reinterpret_cast<uintptr_t*>(top);
    *--sp = 0;                                            // return address of lane_entry
    *--sp = reinterpret_cast<uintptr_t>(&lane_entry);     // where hipsim_switch returns
    for (int i = 0; i < 6; ++i) *--sp = 0;                // callee-saved registers
    return sp;
}

void run_block(Worker& w, uint64_t b) {
    Launch& L = *w.L;
    const uint32_t nthr = L.block.x * L.block.y * L.block.z;
    w.bidx = dim3((uint32_t)(b % L.grid.x), (uint32_t)((b / L.grid.x) % L.grid.y),
                  (uint32_t)(b / (uint64_t(L.grid.x) * L.grid.y)));
    // exactly the bytes the launch asked for: an access past them is reported
    w.dyn = static_cast<char*>(std::malloc(L.smem));
    if (L.smem) std::memset(w.dyn, 0xCD, L.smem);        // LDS holds no zeros at start
    const uint32_t nwaves = (nthr + WAVE - 1) / WAVE;
    for (uint32_t q = 0; q < nwaves; ++q) {
        Wave& wv = w.waves[q];
        wv.live = (int)std::min<uint32_t>(WAVE, nthr - q * WAVE);
        wv.arrived[0] = wv.arrived[1] = 0;
        std::memset(wv.seq, 0xFF, sizeof wv.seq);
    }
    for (uint32_t t = 0; t < nthr; ++t) {
        Lane& l = w.lanes[t];
        l.tid = t;
        l.tidx = ThreadIdx{t % L.block.x, (t / L.block.x) % L.block.y, t / (L.block.x * L.block.y)};
        l.state = RUNNABLE;
        l.seq = 0;
        l.w = &w;
        l.sp = init_stack(l);
    }
    w.live = (int)nthr;
    w.at_barrier = 0;
    while (w.live > 0) {
        bool ran = false;
        for (uint32_t t = 0; t < nthr; ++t) {
            Lane& l = w.lanes[t];
            if (l.state != RUNNABLE) continue;
            ran = true;
            cur = &l;
            hipsim_switch(&w.sched_sp, l.sp);
            cur = nullptr;
        }
        // a barrier every live lane has reached opens
        if (w.at_barrier > 0 && w.at_barrier == w.live) {
            for (uint32_t t = 0; t < nthr; ++t)
                if (w.lanes[t].state == AT_BARRIER) w.lanes[t].state = RUNNABLE;
            w.at_barrier = 0;
            continue;
        }
        // a wave operation every live lane of the wave has reached completes
        bool opened = false;
        for (uint32_t q = 0; q < nwaves; ++q) {
            Wave& wv = w.waves[q];
            for (int buf = 0; buf < 2; ++buf) {
                if (wv.arrived[buf] > 0 && wv.arrived[buf] == wv.live) {
                    for (int i = 0; i < WAVE && q * WAVE + i < nthr; ++i) {
                        Lane& l = w.lanes[q * WAVE + i];
                        if (l.state == AT_WAVE && ((l.seq - 1) & 1) == (uint64_t)buf) l.state = RUNNABLE;
                    }
                    wv.arrived[buf] = 0;
                    opened = true;
                }
            }
        }
        if (opened) continue;
        if (!ran && w.live > 0) {
            int nb = 0, nw = 0;
            for (uint32_t t = 0; t < nthr; ++t) {
                nb += w.lanes[t].state == AT_BARRIER;
                nw += w.lanes[t].state == AT_WAVE;
            }
            std::fprintf(stderr, "hipsim: deadlock in block %llu: %d lanes at __syncthreads, %d at a wave "
                         "operation, %d live\n", (unsigned long long)b, nb, nw, w.live);
            die("deadlock");
        }
    }
    std::free(w.dyn);
    w.dyn = nullptr;
}

// ----------------------------------------------------------- worker pool
struct Pool {
    std::vector<Worker*> workers;
    std::mutex m;
    std::condition_variable cv_go, cv_done;
    Launch* job = nullptr;
    uint64_t epoch = 0;
    int busy = 0;

    explicit Pool(int n) {
        for (int i = 0; i < n; ++i) {
            Worker* w = new Worker();
            w->lanes.resize(MAX_THREADS);
            w->waves.resize(MAX_THREADS / WAVE);
            for (auto& l : w->lanes) {
                void* p = mmap(nullptr, STACK_BYTES, PROT_READ | PROT_WRITE,
                               MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
                if (p == MAP_FAILED) die("stack mmap");
                l.stack = static_cast<char*>(p);
            }
            workers.push_back(w);
            w->th = std::thread([this, w] { loop(w); });
        }
    }
    void loop(Worker* w) {
        tw = w;
        uint64_t seen = 0;
        while (true) {
            Launch* L;
            {
                std::unique_lock<std::mutex> lk(m);
                cv_go.wait(lk, [&] { return epoch != seen; });
                seen = epoch;
                L = job;
            }
            w->L = L;
            for (uint64_t b; (b = L->next.fetch_add(1)) < L->nblocks;) run_block(*w, b);
            w->L = nullptr;
            std::unique_lock<std::mutex> lk(m);
            if (--busy == 0) cv_done.notify_all();
        }
    }
    void run(Launch& L) {
        std::unique_lock<std::mutex> lk(m);
        job = &L;
        busy = (int)workers.size();
        ++epoch;
        cv_go.notify_all();
        cv_done.wait(lk, [&] { return busy == 0; });
    }
};

Pool& pool() {
    static Pool* p = [] {
        int n = 8;
        if (const char* e = std::getenv("HIPSIM_THREADS")) n = std::max(1, std::atoi(e));
        return new Pool(n);
    }();
    return *p;
}

std::atomic<int> g_last_error{hipSuccess};

std::mutex g_note_m;
std::vector<std::string> g_noted;
void note_inactive_read(const char* kernel) {
    std::lock_guard<std::mutex> lk(g_note_m);
    for (auto& k : g_noted) if (k == kernel) return;
    g_noted.push_back(kernel);
    std::fprintf(stderr, "hipsim: %s: a lane read a cross-lane value from an inactive lane\n", kernel);
}

}  // namespace

thread_local Lane* cur = nullptr;

const ThreadIdx& thread_idx() { return cur->tidx; }
const dim3& block_idx() { return cur->w->bidx; }
const dim3& block_dim() { return cur->w->L->block; }
const dim3& grid_dim() { return cur->w->L->grid; }
unsigned lane() { return cur->tid % WAVE; }
void* dyn_smem() { return cur->w->dyn; }

void syncthreads() {
    Lane* l = cur;
    l->state = AT_BARRIER;
    l->w->at_barrier += 1;
    to_scheduler(l);
}

uint64_t wave_exchange(uint64_t v, int op, int arg, int width) {
    Lane* l = cur;
    Worker* w = l->w;
    const uint32_t q = l->tid / WAVE, me = l->tid % WAVE;
    Wave& wv = w->waves[q];
    const uint64_t k = l->seq++;
    const int buf = (int)(k & 1);
    wv.val[buf][me] = v;
    wv.seq[buf][me] = k;
    wv.arrived[buf] += 1;
    l->state = AT_WAVE;
    to_scheduler(l);
    // every live lane of the wave has deposited its value for operation k
    if (width <= 0 || width > WAVE || (width & (width - 1))) die("bad shuffle width");
    const uint32_t seg = me & ~uint32_t(width - 1);
    // a lane that has left the loop or returned deposits nothing: the
    // hardware's permute returns 0 for it, and reading one is reported once
    // per kernel (the result then depends on which lanes are active)
    auto get = [&](uint32_t src, uint64_t) -> uint64_t {
        if (wv.seq[buf][src] != k) {
            note_inactive_read(w->L->name);
            return 0;
        }
        return wv.val[buf][src];
    };
    switch (op) {
        case OP_SHFL: {
            const uint32_t src = seg + ((uint32_t)arg & (width - 1));
            return get(src, v);
        }
        case OP_UP: {
            if ((int)(me - seg) < arg) return v;
            return get(me - arg, v);
        }
        case OP_DOWN: {
            if (me - seg + arg >= (uint32_t)width) return v;
            return get(me + arg, v);
        }
        case OP_XOR: {
            const uint32_t src = me ^ (uint32_t)arg;
            if ((src & ~uint32_t(width - 1)) != seg) return v;
            return get(src, v);
        }
        case OP_BALLOT: {
            uint64_t m = 0;
            for (int i = 0; i < WAVE; ++i)
                if (wv.seq[buf][i] == k && wv.val[buf][i]) m |= uint64_t(1) << i;
            return m;
        }
    }
    die("unknown wave operation");
}

void launch(const char* name, dim3 grid, dim3 block, size_t smem, const std::function<void()>& body) {
    const uint64_t nthr = uint64_t(block.x) * block.y * block.z;
    const uint64_t nblk = uint64_t(grid.x) * grid.y * grid.z;
    if (nthr == 0 || nthr > MAX_THREADS || nblk == 0 || grid.x > 0x7FFFFFFFu || smem > 160 * 1024) {
        std::fprintf(stderr, "hipsim: invalid launch of %s: grid %ux%ux%u block %ux%ux%u smem %zu\n", name,
                     grid.x, grid.y, grid.z, block.x, block.y, block.z, smem);
        g_last_error = hipErrorInvalidValue;
        return;
    }
    if (std::getenv("HIPSIM_TRACE"))
        std::fprintf(stderr, "hipsim: launch %s grid %u block %u smem %zu\n", name, grid.x, block.x, smem);
    Launch L;
    L.name = name;
    L.grid = grid;
    L.block = block;
    L.smem = smem;
    L.body = &body;
    L.nblocks = nblk;
    pool().run(L);
}

}  // namespace hipsim

// ------------------------------------------------------------ runtime API
namespace {
unsigned char fill_byte() {
    const char* e = std::getenv("HIPSIM_FILL");
    return e ? (unsigned char)std::strtoul(e, nullptr, 0) : 0xA5;
}
}  // namespace

hipError_t hipMalloc(void** p, size_t bytes) {
    *p = std::malloc(bytes ? bytes : 1);
    if (!*p) return hipErrorOutOfMemory;
    std::memset(*p, fill_byte(), bytes);
    return hipSuccess;
}
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
    if (bytes) std::memmove(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind k) {
    return hipMemcpyAsync(dst, src, bytes, k, nullptr);
}
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t) {
    std::memset(dst, v, bytes);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipsim::g_last_error.exchange(hipSuccess); }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "hipsim error"; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
    std::memset(p, 0, sizeof *p);
    std::strcpy(p->name, "hipsim");
    // HIPSIM_CUS: a smaller device, so that persistent grids are few and
    // each wave takes many work items
    const char* cus = std::getenv("HIPSIM_CUS");
    p->multiProcessorCount = cus ? std::max(1, std::atoi(cus)) : 256;
    p->sharedMemPerBlock = 160 * 1024;
    p->totalGlobalMem = size_t(288) << 30;
    return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }

struct ihipEvent_t { std::chrono::steady_clock::time_point t; };
struct ihipStream_t { int dummy; };
hipError_t hipEventCreate(hipEvent_t* e) { *e = new ihipEvent_t(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->t = std::chrono::steady_clock::now(); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new ihipStream_t(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus* st) {
    *st = hipStreamCaptureStatusNone;
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol) {
    *ptr = const_cast<void*>(symbol);
    return hipSuccess;
}
