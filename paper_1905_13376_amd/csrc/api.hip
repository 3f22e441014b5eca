// Host side of libmj: argument validation, workspace layout, planning and
// kernel launches behind the C ABI declared in include/mj.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "mj.h"
#include "mj_kernels.h"
#include "mj_host.h"
#include "mj_plan_model.h"

#include <functional>
#include <map>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

using namespace mj;

// One launch (or device copy) of a join's path, recorded instead of issued
// while a batch gathers its joins' work.  A kernel with a merged form
// (`multi`) runs in one grid with the same kernel's launches of other joins;
// anything else is issued alone, in its join's order.
struct LaunchRec {
    std::string name;
    const void* multi = nullptr;          // the kernel's merged form, or null
    uint32_t grid = 0, block = 0, smem = 0;
    uint32_t asz = 0;                     // bytes of its argument struct (merged form)
    size_t aoff = 0;                      // where they sit in the chain's `args`
    std::function<int(hipStream_t)> alone;
};
struct LaunchChain {                      // one join's work, in order
    std::vector<LaunchRec> recs;
    std::vector<unsigned char> args;
};

// Optional per-kernel timing with HIP events recorded on the launch stream.
struct Prof {
    LaunchChain* rec = nullptr;           // set: launches are recorded here, not issued
    bool on = false;
    struct Rec { std::string name; hipEvent_t a, b; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> free_ev;
    std::map<std::string, std::pair<double, long>> total;   // ms, launches
    hipEvent_t ev() {
        if (!free_ev.empty()) { hipEvent_t e = free_ev.back(); free_ev.pop_back(); return e; }
        hipEvent_t e = nullptr; (void)hipEventCreate(&e); return e;
    }
    void collect() {
        for (auto& r : pending) {
            (void)hipEventSynchronize(r.b);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, r.a, r.b);
            auto& t = total[r.name];
            t.first += ms; t.second += 1;
            free_ev.push_back(r.a); free_ev.push_back(r.b);
        }
        pending.clear();
    }
    ~Prof() {
        collect();
        for (auto e : free_ev) (void)hipEventDestroy(e);
    }
};

template <class... P, class... A>
static void record_alone(LaunchChain* c, const std::string& name, void (*kern)(P...), dim3 g, dim3 b,
                         uint32_t smem, A&&... a) {
    LaunchRec r;
    r.name = name;
    r.grid = g.x * g.y * g.z;
    r.block = b.x * b.y * b.z;
    r.smem = smem;
    std::tuple<typename std::decay<P>::type...> args(std::forward<A>(a)...);   // converted now
    r.alone = [=](hipStream_t st) -> int {
        std::apply([&](const auto&... x) { hipLaunchKernelGGL(kern, g, b, smem, st, x...); }, args);
        return hipGetLastError() == hipSuccess ? MJ_OK : MJ_ERR_HIP;
    };
    c->recs.push_back(std::move(r));
}

template <class Args>
static void record_merged(LaunchChain* c, const std::string& name, void (*multi)(MultiGrid), void (*kern)(Args),
                          dim3 g, dim3 b, uint32_t smem, const Args& a) {
    static_assert(std::is_trivially_copyable<Args>::value, "argument structs are copied as bytes");
    LaunchRec r;
    r.name = name;
    r.multi = reinterpret_cast<const void*>(multi);
    r.grid = g.x * g.y * g.z;
    r.block = b.x * b.y * b.z;
    r.smem = smem;
    r.asz = (uint32_t)sizeof(Args);
    r.aoff = c->args.size();
    const unsigned char* bytes = reinterpret_cast<const unsigned char*>(&a);
    c->args.insert(c->args.end(), bytes, bytes + sizeof(Args));
    r.alone = [=](hipStream_t st) -> int {
        hipLaunchKernelGGL(kern, g, b, smem, st, a);
        return hipGetLastError() == hipSuccess ? MJ_OK : MJ_ERR_HIP;
    };
    c->recs.push_back(std::move(r));
}

// Launch a kernel, bracketed by timing events when profiling is on (or
// record it, inside a batch).
#define MJ_LAUNCH(prof, name, kern, grid, block, smem, st, ...)                       \
    do {                                                                           \
        if ((prof) && (prof)->rec) {                                               \
            record_alone((prof)->rec, std::string(name), kern, dim3(grid), dim3(block), \
                         (uint32_t)(smem), __VA_ARGS__);                           \
            break;                                                                 \
        }                                                                          \
        hipEvent_t ea_ = nullptr, eb_ = nullptr;                                   \
        if ((prof) && (prof)->on) { ea_ = (prof)->ev(); eb_ = (prof)->ev();        \
                                    (void)hipEventRecord(ea_, st); }               \
        hipLaunchKernelGGL(kern, grid, block, smem, st, __VA_ARGS__);              \
        hipError_t le_ = hipGetLastError();                                        \
        if (le_ != hipSuccess) {                                                   \
            std::fprintf(stderr, "libmj: launch of %s failed: %s\n",              \
                         std::string(name).c_str(), hipGetErrorString(le_));       \
            return MJ_ERR_HIP;                                                     \
        }                                                                          \
        if (ea_) { (void)hipEventRecord(eb_, st);                                  \
                   (prof)->pending.push_back({std::string(name), ea_, eb_}); }     \
    } while (0)

// Launch a kernel written with MJ_KERNEL; the arguments initialise its
// argument struct.  Inside a batch the launch is recorded in its merged form.
#define MJ_LAUNCHM(prof, name, kern, grid, block, smem, st, ...)                      \
    do {                                                                           \
        const kern##_args ma_{__VA_ARGS__};                                        \
        if ((prof) && (prof)->rec) {                                               \
            record_merged((prof)->rec, std::string(name), kern##_multi, kern, dim3(grid), \
                          dim3(block), (uint32_t)(smem), ma_);                     \
            break;                                                                 \
        }                                                                          \
        MJ_LAUNCH(prof, name, kern, grid, block, smem, st, ma_);                   \
    } while (0)

// ------------------------------------------------------------------ context
struct mj_ctx {
    int device = 0;
    int num_cu = 256;
    Prof prof;
    DeviceModel model = default_model();
    std::map<std::string, mj_plan_t> tuned;     // autotuner cache per size class
    std::vector<void*> pinned;                  // captured batches' argument tables (kept alive)
    char* stage = nullptr;                      // eager batches' argument tables (pinned, reused)
    size_t stage_bytes = 0;
    hipEvent_t stage_read = nullptr;            // recorded after the last copy out of `stage`
    const void* planner = nullptr;              // learned planner parameters (device)
    // this device's copy of the file-scope scratch array (device address),
    // found once at context creation
    void* static_scratch = nullptr;
};

// Workspace of mj_linear3_count_static: one array per device, part of the
// library's code object, so that the call allocates nothing.  Every call on
// a device shares it (and finds what the last call left there).
constexpr size_t MJ_STATIC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[MJ_STATIC_SCRATCH_BYTES];

namespace {

#define MJ_HIP(call)                                                   \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) {                                        \
            std::fprintf(stderr, "libmj: %s failed: %s\n", #call,      \
                         hipGetErrorString(e_));                       \
            return MJ_ERR_HIP;                                         \
        }                                                              \
    } while (0)

#define MJ_LAUNCHED()                                                  \
    do {                                                               \
        hipError_t e_ = hipGetLastError();                             \
        if (e_ != hipSuccess) {                                        \
            std::fprintf(stderr, "libmj: launch failed: %s\n",         \
                         hipGetErrorString(e_));                       \
            return MJ_ERR_HIP;                                         \
        }                                                              \
    } while (0)

}  // namespace

// ============================================================ validation
namespace mj {

int check_rel(const mj_rel* r) {
    if (!r) return MJ_ERR_INVALID_ARG;
    if (r->n >= (uint64_t(1) << 32)) return MJ_ERR_INVALID_ARG;
    if (r->n > 0 && (!r->col0 || !r->col1 || r->stride < 1)) return MJ_ERR_INVALID_ARG;
    return MJ_OK;
}

bool same_rel(const mj_rel& x, const mj_rel& y) {
    return x.col0 == y.col0 && x.col1 == y.col1 && x.n == y.n && x.stride == y.stride;
}

// FNV-1a over the three relations' pointers, strides and sizes: the plan's
// fingerprint of the inputs it was made for.
uint64_t fingerprint(const mj_rel& R, const mj_rel& S, const mj_rel& T) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) { h ^= (v >> (8 * i)) & 0xFF; h *= 1099511628211ull; }
    };
    for (const mj_rel* r : {&R, &S, &T}) {
        mix(reinterpret_cast<uintptr_t>(r->col0));
        mix(reinterpret_cast<uintptr_t>(r->col1));
        mix(r->n);
        mix(static_cast<uint64_t>(r->stride));
    }
    return h;
}

uint32_t ceil_log2(uint64_t x) {
    uint32_t b = 0;
    while ((uint64_t(1) << b) < x) ++b;
    return b;
}

}  // namespace mj

// ================================================================ layouts
namespace {

struct Bump {
    char* base;
    size_t off = 0;
    explicit Bump(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

// Skew split of a per-bucket kernel: a bucket of more than `chunk` tuples
// (MJ_SPLIT_PCT percent of the mean bucket, at least SPLIT_MIN_CHUNK) runs
// as several workgroups.  items: at most nb + n / chunk + 1 of them;
// scratch rows: a split bucket has len > chunk, so its pieces number fewer
// than 2 len / chunk, and all split buckets fewer than 2 n / chunk + 1.
#ifndef MJ_SPLIT_PCT
#define MJ_SPLIT_PCT 200
#endif
uint32_t split_chunk(uint64_t n, uint32_t bits) {
    const uint64_t mean = (n + (uint64_t(1) << bits) - 1) >> bits;
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(SPLIT_MIN_CHUNK, mean * MJ_SPLIT_PCT / 100),
                                        uint64_t(1) << 31);
}
uint32_t split_grid(uint64_t n, uint32_t bits) { return (1u << bits) + (uint32_t)(n / split_chunk(n, bits)) + 1; }
// the work items of n tuples under a given split (its chunk may come from a
// larger relation's layout: then they are fewer)
uint32_t items_grid(const BucketItems& I, uint64_t n, uint32_t bits) {
    return (1u << bits) + (uint32_t)(n / I.chunk) + 1;
}
uint64_t split_rows(uint64_t n, uint32_t bits) { return 2 * (n / split_chunk(n, bits)) + 1; }
BucketItems take_items(Bump& B, uint64_t n, uint32_t bits) {
    BucketItems I{};
    const uint32_t nb = 1u << bits;
    I.chunk = split_chunk(n, bits);
    I.items = B.take<uint32_t>(split_grid(n, bits));
    I.nitems = B.take<uint32_t>(1);
    I.hrow = B.take<uint32_t>(nb);
    I.done = B.take<uint32_t>(nb);
    return I;
}

struct TableLayout {                 // bucketed multiplicity tables of one column
    uint32_t* hist;
    uint32_t* counts;
    uint32_t* starts;
    uint32_t* keys;                  // the partitioned column
    DirEntry* dir;
    uint2* pool;
    unsigned long long* pool_cursor;
    uint32_t* err;
    uint64_t pool_slots;
    BucketItems split;               // heavy buckets in pieces: their items,
    uint2* rows;                     // the pieces' (key, count) tables
    uint32_t* row_special;
};

uint32_t ntiles_of(uint64_t n) { return (uint32_t)((n + PART_TILE - 1) / PART_TILE); }

uint64_t pool_slots_for(uint64_t n, uint32_t nbkt) {
    return 4 * n + uint64_t(DB_MIN_CAP) * nbkt + DB_MIN_CAP;
}

void take_table(Bump& B, TableLayout& L, uint64_t n, uint32_t bits) {
    const uint32_t nb = 1u << bits;
    L.hist = B.take<uint32_t>(uint64_t(nb) * ntiles_of(n));
    L.counts = B.take<uint32_t>(nb);
    L.starts = B.take<uint32_t>(nb + 1);
    L.keys = B.take<uint32_t>(std::max<uint64_t>(n, 1));
    L.dir = B.take<DirEntry>(nb);
    L.pool_slots = pool_slots_for(n, nb);
    L.pool = B.take<uint2>(L.pool_slots);
    L.pool_cursor = B.take<unsigned long long>(1);
    L.err = B.take<uint32_t>(1);
    L.split = take_items(B, n, bits);
    const uint64_t nrows = split_rows(n, bits);
    L.rows = B.take<uint2>(nrows * DB_CAP);
    L.row_special = B.take<uint32_t>(nrows);
}

struct RelPart {                     // one relation partitioned into 2^bits buckets
    uint32_t* hist;
    uint32_t* counts;
    uint32_t* starts;
    uint2* pairs;
};

void take_part(Bump& B, RelPart& P, uint64_t n, uint32_t bits) {
    const uint32_t nb = 1u << bits;
    P.hist = B.take<uint32_t>(uint64_t(nb) * ntiles_of(n));
    P.counts = B.take<uint32_t>(nb);
    P.starts = B.take<uint32_t>(nb + 1);
    P.pairs = B.take<uint2>(std::max<uint64_t>(n, 1));
}

// Ranges of A for the per-A counts: about 32K R tuples per range, at most
// 2^PART_MAX_BITS ranges of at most 2^ACELL_MAX_SHIFT values.  False when
// a_domain needs more (the cells then add into the output with atomics).
bool a_ranges(const mj_plan_t& p, uint32_t& bits, uint32_t& shift) {
    if (p.a_domain == 0) return false;
    const uint32_t L = ceil_log2(p.a_domain);
    bits = std::min<uint32_t>({ceil_log2((p.n_r + 32767) / 32768), PART_MAX_BITS, L});
    if (L - bits > ACELL_MAX_SHIFT) bits = L - ACELL_MAX_SHIFT;
    shift = L - bits;
    return bits <= PART_MAX_BITS;
}

// Ranges of a key domain [0, domain): about 32K of n tuples per range, at
// most 2^PART_MAX_BITS ranges of at most 2^ACELL_MAX_SHIFT values; false
// when the domain needs more.
bool key_ranges(uint64_t n, uint32_t domain, uint32_t& bits, uint32_t& shift) {
    if (domain == 0) return false;
    const uint32_t L = ceil_log2(domain);
    bits = std::min<uint32_t>({ceil_log2((n + 32767) / 32768), PART_MAX_BITS, L});
    if (L - bits > ACELL_MAX_SHIFT) bits = L - ACELL_MAX_SHIFT;
    shift = L - bits;
    return bits <= PART_MAX_BITS;
}

// dense keys: B and C below these bounds, and not much sparser than the tuples
constexpr uint32_t DENSE_MAX_DOMAIN = 1u << 24;
bool dense_ok(uint64_t dom, uint64_t n) { return dom >= 1 && dom <= DENSE_MAX_DOMAIN && dom <= 2 * n + 4096; }

struct DenseLayout {                  // the linear join with direct-indexed tables
    RelPart T, S, R;                  // T.c by range of C (keys in T.pairs' space), S by B, R by A
    uint32_t* tkeys;
    uint32_t* deg;                    // [c_domain] multiplicity of each C value in T
    uint16_t* deg16;                  // [c_domain] the same, cut to 16 bits
    unsigned long long* w;            // [b_domain] W[b]
    uint16_t* w16;                    // [b_domain] W[b], or 0xFFFF where W[b] >= 0xFFFF (then read w)
    uint32_t* err;                    // [0]: a key out of its bound; [1]: unused;
                                      // [2]: some deg[c] >= 2^16
    uint32_t c_bits, c_shift, b_bits, b_shift, a_bits, a_shift;
    BucketItems Tsplit, Ssplit, Rsplit;  // skew split of each partition's ranges
    unsigned long long* rows;         // scratch rows of the split ranges (shared by the three sums)
    size_t bytes;
};

bool dense_plan(const mj_plan_t& p) {
    uint32_t x, y;
    return (p.flags & MJ_PLAN_DENSE_KEYS) && key_ranges(p.n_r, p.a_domain, x, y) &&
           key_ranges(p.n_s, p.b_domain, x, y) && key_ranges(p.n_t, p.c_domain, x, y);
}

DenseLayout dense_layout(void* ws, const mj_plan_t& p) {
    Bump B(ws);
    DenseLayout L{};
    key_ranges(p.n_t, p.c_domain, L.c_bits, L.c_shift);
    key_ranges(p.n_s, p.b_domain, L.b_bits, L.b_shift);
    key_ranges(p.n_r, p.a_domain, L.a_bits, L.a_shift);
    auto part = [&](RelPart& P, uint64_t n, uint32_t bits, bool pairs) {
        const uint32_t nb = 1u << bits;
        P.hist = B.take<uint32_t>(uint64_t(nb) * ntiles_of(n));
        P.counts = B.take<uint32_t>(nb);
        P.starts = B.take<uint32_t>(nb + 1);
        P.pairs = pairs ? B.take<uint2>(std::max<uint64_t>(n, 1)) : nullptr;
    };
    part(L.T, p.n_t, L.c_bits, false);
    L.tkeys = B.take<uint32_t>(std::max<uint64_t>(p.n_t, 1));
    part(L.S, p.n_s, L.b_bits, true);
    part(L.R, p.n_r, L.a_bits, true);
    L.Tsplit = take_items(B, p.n_t, L.c_bits);
    L.Ssplit = take_items(B, p.n_s, L.b_bits);
    L.Rsplit = take_items(B, p.n_r, L.a_bits);
    const uint64_t row_words = std::max({split_rows(p.n_t, L.c_bits) << L.c_shift,
                                         split_rows(p.n_s, L.b_bits) << L.b_shift,
                                         split_rows(p.n_r, L.a_bits) << L.a_shift});
    L.rows = B.take<unsigned long long>(row_words);
    L.deg = B.take<uint32_t>(std::max<uint32_t>(p.c_domain, 1));
    L.deg16 = B.take<uint16_t>(std::max<uint32_t>(p.c_domain, 1));
    L.w = B.take<unsigned long long>(std::max<uint32_t>(p.b_domain, 1));
    L.w16 = B.take<uint16_t>(std::max<uint32_t>(p.b_domain, 1));
    L.err = B.take<uint32_t>(3);
    L.bytes = B.off + 256;
    return L;
}

struct LinearLayout {
    RelPart R, S;                     // R and S by bucket of B (cells)
    RelPart Ra;                       // R by range of A (shares R's pair buffer)
    TableLayout T;
    WDirEntry* wdir;                  // W tables per bucket of B
    WSlot* wpool;
    unsigned long long* wcursor;
    uint64_t wslots;
    uint32_t a_bits, a_shift;
    bool by_range;                    // per-A counts by ranges of A (no atomics)
    BucketItems Rasplit;              // skew split of the ranges of A
    unsigned long long* rows;         // scratch rows of its split ranges
    BucketItems Ssplit;               // skew split of the buckets of S (W build)
    WSlot* wrows;                     // the pieces' W tables
    unsigned long long* wrow_special;
    // S-largest plans: R's B values as tables per part of R, a sum per slot
    TableLayout Rk;
    unsigned long long* wval;
    unsigned long long* wspecial;
    size_t bytes;
};

// S-largest plans partition S by (bucket of B, bucket of C)
uint32_t s_part_bits(const mj_plan_t& p) {
    return p.log2_nb + (p.algo == MJ_ALGO_SLARGE ? p.log2_nc : 0u);
}

// Workgroups per (part of R, part of T) of the S-largest plan: about 32K
// tuples of S each, and 512 workgroups at least in all.
uint32_t sl_pieces(const mj_plan_t& p) {
    const uint64_t cells = uint64_t(1) << (p.log2_nb + p.log2_nc);
    uint64_t k = std::max<uint64_t>(1, p.n_s / (cells * 32768));
    k = std::max<uint64_t>(k, (512 + cells - 1) / cells);
    return (uint32_t)std::min<uint64_t>(k, 64);
}

LinearLayout linear_layout(void* ws, const mj_plan_t& p) {
    Bump B(ws);
    LinearLayout L;
    take_part(B, L.R, p.n_r, p.log2_nb);
    take_part(B, L.S, p.n_s, s_part_bits(p));
    take_table(B, L.T, p.n_t, p.log2_nc);
    L.by_range = a_ranges(p, L.a_bits, L.a_shift);
    L.wdir = nullptr; L.wpool = nullptr; L.wcursor = nullptr; L.wslots = 0;
    L.Rasplit = BucketItems{}; L.rows = nullptr;
    L.Ssplit = BucketItems{}; L.wrows = nullptr; L.wrow_special = nullptr;
    L.Ra = L.R;
    if (L.by_range) {
        const uint32_t na = 1u << L.a_bits;
        L.Ra.hist = B.take<uint32_t>(uint64_t(na) * ntiles_of(p.n_r));
        L.Ra.counts = B.take<uint32_t>(na);
        L.Ra.starts = B.take<uint32_t>(na + 1);
        L.Rasplit = take_items(B, p.n_r, L.a_bits);
        L.rows = B.take<unsigned long long>(split_rows(p.n_r, L.a_bits) << L.a_shift);
        const uint32_t nb = 1u << p.log2_nb;
        L.wdir = B.take<WDirEntry>(nb);
        if (p.algo == MJ_ALGO_SLARGE) {
            // the W tables are R's B tables, slot for slot
            take_table(B, L.Rk, p.n_r, p.log2_nb);
            L.wval = B.take<unsigned long long>(L.Rk.pool_slots);
            L.wspecial = B.take<unsigned long long>(nb);
            L.wslots = L.Rk.pool_slots;
        } else {
            // a bucket's table holds at most 4 slots per S tuple (a power of
            // two >= twice its keys), plus the minimum per bucket and the
            // empty head
            L.wslots = 4 * p.n_s + uint64_t(W_MIN_CAP) * (nb + 1);
            L.Ssplit = take_items(B, p.n_s, p.log2_nb);
            const uint64_t nrows = split_rows(p.n_s, p.log2_nb);
            L.wrows = B.take<WSlot>(nrows * CELL_CAP);
            L.wrow_special = B.take<unsigned long long>(nrows);
        }
        L.wpool = B.take<WSlot>(L.wslots);
        L.wcursor = B.take<unsigned long long>(1);
    }
    L.bytes = B.off + 256;
    return L;
}



struct CascadeLayout {
    RelPart R, S;
    TableLayout T;
    // dense keys: T's C column by range and its multiplicities deg / deg16
    RelPart Tr;
    uint32_t* tkeys;
    uint32_t* deg;
    uint16_t* deg16;
    uint32_t* dflags;                 // [0]: a C value out of its bound; [1]: unused; [2]: some deg >= 2^16
    uint32_t c_bits, c_shift;
    uint32_t* Rgrp;
    uint32_t* ecnt;
    uint32_t* elist;
    unsigned long long* eoff;
    unsigned long long* partial;
    uint2* I;
    uint64_t i_cap;               // pairs of I that fit the workspace
    size_t base_bytes;            // everything but I
};

constexpr uint64_t CAS_DEFAULT_I_CAP = uint64_t(1) << 28;   // 2 GiB of (a, c) pairs

CascadeLayout cascade_layout(void* ws, const mj_plan_t& p, uint64_t ws_bytes) {
    Bump B(ws);
    CascadeLayout L;
    take_part(B, L.R, p.n_r, p.log2_nb);
    take_part(B, L.S, p.n_s, p.log2_nb);
    L.Tr = RelPart{}; L.tkeys = nullptr; L.deg = nullptr; L.deg16 = nullptr; L.dflags = nullptr;
    L.c_bits = L.c_shift = 0;
    if (dense_plan(p)) {
        key_ranges(p.n_t, p.c_domain, L.c_bits, L.c_shift);
        const uint32_t nb = 1u << L.c_bits;
        L.Tr.hist = B.take<uint32_t>(uint64_t(nb) * ntiles_of(p.n_t));
        L.Tr.counts = B.take<uint32_t>(nb);
        L.Tr.starts = B.take<uint32_t>(nb + 1);
        L.tkeys = B.take<uint32_t>(std::max<uint64_t>(p.n_t, 1));
        L.deg = B.take<uint32_t>(std::max<uint32_t>(p.c_domain, 1));
        L.deg16 = B.take<uint16_t>(std::max<uint32_t>(p.c_domain, 1));
        L.dflags = B.take<uint32_t>(3);
    } else {
        take_table(B, L.T, p.n_t, p.log2_nc);
    }
    // join 1 groups S's C values by B and probes with R's tuples
    L.Rgrp = B.take<uint32_t>(std::max<uint64_t>(p.n_s, 1));
    L.ecnt = B.take<uint32_t>(std::max<uint64_t>(p.n_r, 1));
    L.elist = B.take<uint32_t>(std::max<uint64_t>(p.n_r, 1));
    L.eoff = B.take<unsigned long long>(p.n_r + 1);
    const uint64_t nblk = (p.n_r + SCAN_TILE - 1) / SCAN_TILE;
    L.partial = B.take<unsigned long long>(nblk + 1);
    L.I = B.take<uint2>(0);
    L.base_bytes = B.off + 256;
    if (ws) {
        L.i_cap = ws_bytes > L.base_bytes ? (ws_bytes - L.base_bytes) / sizeof(uint2) : 0;
    } else {
        L.i_cap = std::max<uint64_t>(1, std::min<uint64_t>(p.join2_size, CAS_DEFAULT_I_CAP));
    }
    return L;
}

uint32_t seed_b(const mj_plan_t& p) { return p.seed; }
uint32_t seed_c(const mj_plan_t& p) { return p.seed ^ 0x9E3779B9u; }
uint32_t seed_slot(const mj_plan_t& p) { return p.seed ^ 0x7F4A7C15u; }
uint32_t seed_w(const mj_plan_t& p) { return p.seed ^ 0x2545F491u; }

uint32_t grid_for(uint64_t n, int threads, uint32_t cap = 65535) {
    uint64_t g = (n + threads - 1) / threads;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, cap));
}

PartJob make_job(const mj_rel& r, uint32_t* hist, uint32_t* counts, uint32_t* starts,
                 int key0, uint32_t seed0, uint32_t bits0, int key1, uint32_t seed1, uint32_t bits1) {
    PartJob J{};
    J.col0 = r.col0; J.col1 = r.col1; J.stride = r.stride; J.n = r.n;
    J.packed = (r.stride == 2 && r.col1 == r.col0 + 1 &&
                (reinterpret_cast<uintptr_t>(r.col0) & 15) == 0) ? 1u : 0u;
    J.key0_col = key0; J.seed0 = seed0; J.bits0 = bits0;
    J.key1_col = key1; J.seed1 = seed1; J.bits1 = bits1;
    J.hist = hist; J.counts = counts; J.starts = starts;
    J.ntiles = ntiles_of(r.n);
    return J;
}

// Partition up to MJ_PART_MAX_JOBS relations (four launches in all).
int launch_partition(Prof* prof, const char* tag, PartLaunch& P, hipStream_t st) {
    uint32_t tiles = 0, rows = 0, maxbits = 0;
    for (int q = 0; q < P.njobs; ++q) {
        const PartJob& J = P.job[q];
        // a one-column payload is re-bucketed from that column alone
        if (!J.out_pair && (J.bits1 != 0 || J.key0_col != J.single_col)) return MJ_ERR_INVALID_ARG;
        if ((J.out_pair != nullptr) == (J.out_single != nullptr)) return MJ_ERR_INVALID_ARG;
    }
    for (int q = 0; q < P.njobs; ++q) {
        P.job[q].tile_begin = tiles;
        tiles += P.job[q].ntiles;
        const uint32_t bits = P.job[q].bits0 + P.job[q].bits1;
        rows += 1u << bits;
        maxbits = std::max(maxbits, bits);
    }
    const std::string t(tag);
    // k_part_hist clears the caller's words first
    if (tiles) {
        MJ_LAUNCHM(prof, t + ":k_part_hist", k_part_hist, dim3(tiles), dim3(PART_THREADS),
                  (size_t(1) << maxbits) * 4, st, P);
    } else if (P.nclear) {
        MJ_LAUNCHM(prof, t + ":k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, st, P.clear, (uint64_t)P.nclear, 0u);
    }
    MJ_LAUNCHM(prof, t + ":k_part_rowscan", k_part_rowscan, dim3(rows), dim3(PART_THREADS),
              PART_SCAN_CHUNK * 4, st, P);
    MJ_LAUNCHM(prof, t + ":k_part_scan", k_part_scan, dim3(P.njobs), dim3(PART_THREADS),
              (size_t(1) << maxbits) * 4, st, P);
    if (tiles)
        MJ_LAUNCHM(prof, t + ":k_part_scatter", k_part_scatter, dim3(tiles), dim3(PART_SCATTER_THREADS),
                  part_scatter_smem(maxbits), st, P);
    return MJ_OK;
}

// Partition T.c (or any single column) by bucket and build its tables.
int launch_tables(Prof* prof, const TableLayout& L, const mj_rel& rel, int col, uint32_t bits,
                  uint32_t bseed, uint32_t sseed, hipStream_t st) {
    const uint32_t nb = 1u << bits;
    MJ_LAUNCHM(prof, "tab:k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(L.pool),
                       (uint64_t)(2 * DB_MIN_CAP), EMPTY_KEY);
    // pool[0..DB_MIN_CAP) stays empty (keys EMPTY); cursor = DB_MIN_CAP; err = 0
    MJ_LAUNCHM(prof, "tab:k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, st, L.pool_cursor, (uint64_t)1,
                       (unsigned long long)DB_MIN_CAP);
    MJ_LAUNCHM(prof, "tab:k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, st, L.err, (uint64_t)1, 0u);

    PartLaunch P{};
    P.njobs = 1;
    P.job[0] = make_job(rel, L.hist, L.counts, L.starts, col, bseed, bits, 0, 0, 0);
    P.job[0].out_single = L.keys;
    P.job[0].single_col = col;
    P.job[0].split = L.split;                    // heavy buckets in pieces
    int st2 = launch_partition(prof, "tab", P, st);
    if (st2) return st2;
    DBuildArgs D{};
    D.keys = L.keys; D.starts = L.starts; D.nbkt = nb; D.slot_seed = sseed;
    D.dir = L.dir; D.pool = L.pool; D.pool_cursor = L.pool_cursor; D.pool_cap = L.pool_slots;
    D.err = L.err;
    D.split = L.split; D.rows = L.rows; D.row_special = L.row_special;
    MJ_LAUNCHM(prof, "tab:k_dbuild", k_dbuild, dim3(items_grid(L.split, rel.n, bits)), dim3(DB_THREADS), 0, st, D);
    return MJ_OK;
}

struct RunBuf {
    uint32_t* run_key;
    uint32_t* run_start;
    uint32_t* dir;
    uint32_t bits;
    unsigned long long* nruns;
};

struct PassBuf {                      // work queues of one pass of the cyclic join
    uint32_t* light;
    uint32_t* ctr;                    // nlight, light_next, nheavy_groups, heavy_next
    uint32_t* heavy_group;
    uint32_t* heavy_items;
    unsigned long long* heavy_off;
    uint32_t n_heavy_cap;
};

struct TriLayout {
    unsigned long long* Rk;
    unsigned long long* Sk;           // S by (m(b), m(c))
    unsigned long long* Sk2;          // S by (m(c), m(b))
    unsigned long long* Tk;
    uint32_t* Rl;                     // low words of the sorted keys
    uint32_t* Sl;
    uint32_t* Sl2;
    uint32_t* Tl;
    unsigned long long* tmp;          // radix double buffer
    uint32_t* rs_hist;
    uint32_t* rs_counts;
    uint32_t* rs_starts;
    uint32_t* flags;
    unsigned long long* ridx;
    unsigned long long* partial;
    RunBuf R, S, S2, T;
    PassBuf P[2];
    size_t bytes;
};

uint32_t dir_bits(uint64_t n) { return std::min<uint32_t>(24, std::max<uint32_t>(1, ceil_log2(n))); }

void take_runs(Bump& B, RunBuf& X, uint64_t n, bool with_dir) {
    X.run_key = B.take<uint32_t>(std::max<uint64_t>(n, 1));
    X.run_start = B.take<uint32_t>(n + 1);
    X.bits = dir_bits(n);
    X.dir = with_dir ? B.take<uint32_t>((uint64_t(1) << X.bits) + 1) : nullptr;
    X.nruns = B.take<unsigned long long>(1);
}

void take_pass(Bump& B, PassBuf& P, uint64_t n_stage, uint64_t n_s) {
    P.light = B.take<uint32_t>(std::max<uint64_t>(n_s, 1));
    P.ctr = B.take<uint32_t>(4);
    P.n_heavy_cap = (uint32_t)(n_stage / (TRI_LIGHT_X + 1) + n_s / (TRI_LIGHT_S + 1) + 2);
    P.heavy_group = B.take<uint32_t>(P.n_heavy_cap);
    P.heavy_items = B.take<uint32_t>(P.n_heavy_cap);
    P.heavy_off = B.take<unsigned long long>(P.n_heavy_cap + 1);
}

TriLayout tri_layout(void* ws, const mj_plan_t& p) {
    Bump B(ws);
    TriLayout L;
    const uint64_t nmax = std::max<uint64_t>({p.n_r, p.n_s, p.n_t, 1});
    L.Rk = B.take<unsigned long long>(std::max<uint64_t>(p.n_r, 1));
    L.Sk = B.take<unsigned long long>(std::max<uint64_t>(p.n_s, 1));
    L.Sk2 = B.take<unsigned long long>(std::max<uint64_t>(p.n_s, 1));
    L.Tk = B.take<unsigned long long>(std::max<uint64_t>(p.n_t, 1));
    L.Rl = B.take<uint32_t>(std::max<uint64_t>(p.n_r, 1));
    L.Sl = B.take<uint32_t>(std::max<uint64_t>(p.n_s, 1));
    L.Sl2 = B.take<uint32_t>(std::max<uint64_t>(p.n_s, 1));
    L.Tl = B.take<uint32_t>(std::max<uint64_t>(p.n_t, 1));
    L.tmp = B.take<unsigned long long>(nmax);
    const uint64_t ntiles = (nmax + RS_TILE - 1) / RS_TILE;
    L.rs_hist = B.take<uint32_t>(256 * ntiles);
    L.rs_counts = B.take<uint32_t>(256);
    L.rs_starts = B.take<uint32_t>(257);
    L.flags = B.take<uint32_t>(nmax);
    L.ridx = B.take<unsigned long long>(nmax + 1);
    L.partial = B.take<unsigned long long>((nmax + SCAN_TILE - 1) / SCAN_TILE + 1);
    take_runs(B, L.R, p.n_r, true);
    take_runs(B, L.S, p.n_s, false);
    take_runs(B, L.S2, p.n_s, false);
    take_runs(B, L.T, p.n_t, true);
    take_pass(B, L.P[0], p.n_r, p.n_s);
    take_pass(B, L.P[1], p.n_t, p.n_s);
    L.bytes = B.off + 256;
    return L;
}

int launch_scan_u32(Prof* prof, const uint32_t* in, uint64_t n, unsigned long long* partial,
                    unsigned long long* out, hipStream_t s) {
    const uint32_t nblk = (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE);
    if (nblk == 0) {
        MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, out, (uint64_t)1, 0ull);
        return MJ_OK;
    }
    if (nblk == 1) {                         // one tile: one launch
        MJ_LAUNCHM(prof, "k_scan_one", k_scan_one, dim3(1), dim3(SCAN_THREADS), 0, s, in, n, partial, out, nblk);
        return MJ_OK;
    }
    MJ_LAUNCHM(prof, "k_scan_reduce", k_scan_reduce, dim3(nblk), dim3(SCAN_THREADS), 0, s, in, n, partial, out, nblk);
    MJ_LAUNCHM(prof, "k_scan_partials", k_scan_partials, dim3(1), dim3(SCAN_THREADS), 0, s, in, n, partial, out, nblk);
    MJ_LAUNCHM(prof, "k_scan_apply", k_scan_apply, dim3(nblk), dim3(SCAN_THREADS), 0, s, in, n, partial, out, nblk);
    return MJ_OK;
}

int launch_scan_u64(Prof* prof, const unsigned long long* in, uint64_t n, unsigned long long* partial,
                    unsigned long long* out, hipStream_t s) {
    const uint32_t nblk = (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE);
    if (nblk == 0) {
        MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, out, (uint64_t)1, 0ull);
        return MJ_OK;
    }
    if (nblk == 1) {
        MJ_LAUNCHM(prof, "k_scan_one64", k_scan_one64, dim3(1), dim3(SCAN_THREADS), 0, s, in, n, partial, out, nblk);
        return MJ_OK;
    }
    MJ_LAUNCHM(prof, "k_scan_reduce64", k_scan_reduce64, dim3(nblk), dim3(SCAN_THREADS), 0, s, in, n, partial, out,
               nblk);
    MJ_LAUNCHM(prof, "k_scan_partials", k_scan_partials, dim3(1), dim3(SCAN_THREADS), 0, s, nullptr, n, partial,
               out, nblk);
    MJ_LAUNCHM(prof, "k_scan_apply64", k_scan_apply64, dim3(nblk), dim3(SCAN_THREADS), 0, s, in, n, partial, out,
               nblk);
    return MJ_OK;
}

// Sort n 64-bit keys in place (8 stable passes of 8 bits; tmp is the other buffer).
// LSD radix sort of 64-bit keys on bytes first_pass..7 (first_pass = 4:
// grouped by the high word, stable in the low word); first_pass must be even
// so that the result is back in `keys`
int launch_radix_sort(Prof* prof, unsigned long long* keys, unsigned long long* tmp, uint64_t n,
                      uint32_t* hist, uint32_t* counts, uint32_t* starts, hipStream_t s,
                      uint32_t first_pass = 0) {
    if (n <= 1) return MJ_OK;
    if (first_pass & 1) return MJ_ERR_INVALID_ARG;
    if (first_pass >= 8) return MJ_OK;
    if (n <= RS_SMALL) {                 // the whole sort in one workgroup
        uint32_t P = 2;
        while (P < n) P <<= 1;
        const uint32_t shift = 8 * first_pass;
        const size_t smem = size_t(P) * sizeof(unsigned long long);
        MJ_LAUNCHM(prof, "k_rs_small", k_rs_small, dim3(1), dim3(RS_SMALL_THREADS), smem, s, keys, (uint32_t)n,
                  shift);
        return MJ_OK;
    }
    const uint32_t ntiles = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
    unsigned long long* src = keys;
    unsigned long long* dst = tmp;
    for (uint32_t pass = first_pass; pass < 8; ++pass) {
        RsArgs A;
        A.in = src; A.out = dst; A.n = n; A.shift = 8 * pass; A.ntiles = ntiles;
        A.hist = hist; A.starts = starts;
        MJ_LAUNCHM(prof, "k_rs_hist", k_rs_hist, dim3(ntiles), dim3(RS_THREADS), 0, s, A);
        if (ntiles <= RS_SCAN1_TILES) {
            MJ_LAUNCHM(prof, "k_rs_scan1", k_rs_scan1, dim3(1), dim3(256), 0, s, A, starts);
        } else {
            PartLaunch P{};
            P.njobs = 1;
            P.job[0].hist = hist; P.job[0].ntiles = ntiles; P.job[0].counts = counts;
            P.job[0].starts = starts; P.job[0].bits0 = 8; P.job[0].bits1 = 0;
            MJ_LAUNCHM(prof, "k_part_rowscan", k_part_rowscan, dim3(256), dim3(PART_THREADS),
                      PART_SCAN_CHUNK * 4, s, P);
            MJ_LAUNCHM(prof, "k_part_scan", k_part_scan, dim3(1), dim3(PART_THREADS), 256 * 4, s, P);
        }
        MJ_LAUNCHM(prof, "k_rs_scatter", k_rs_scatter, dim3(ntiles), dim3(RS_THREADS), 0, s, A);
        std::swap(src, dst);
    }
    return MJ_OK;            // an even number of passes: the result is back in `keys`
}

int launch_runs(Prof* prof, const TriLayout& L, const unsigned long long* keys, uint64_t n,
                const RunBuf& X, uint32_t* low, hipStream_t s) {
    if (n == 0) {
        MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, X.nruns, (uint64_t)1, 0ull);
        MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, X.run_start, (uint64_t)1, 0u);
    } else {
        MJ_LAUNCHM(prof, "k_run_flags", k_run_flags, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s,
                  keys, n, L.flags, low);
        int st = launch_scan_u32(prof, L.flags, n, L.partial, L.ridx, s);
        if (st) return st;
        MJ_LAUNCHM(prof, "k_run_compact", k_run_compact, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s,
                  keys, n, L.flags, L.ridx, X.run_key, X.run_start, X.nruns);
    }
    if (X.dir)
        MJ_LAUNCHM(prof, "k_run_dir", k_run_dir, dim3(grid_for(n + 1, 256, 16384)), dim3(256), 0, s,
                  X.run_key, X.nruns, X.bits, X.dir);
    return MJ_OK;
}

RunIndex run_index(const RunBuf& X) {
    RunIndex I;
    I.run_key = X.run_key; I.run_start = X.run_start; I.dir = X.dir; I.bits = X.bits;
    I.nruns = X.nruns;
    return I;
}

// (mix(key) << 32 | mix(other)), or the other value itself as low word
int tri_keys(Prof* prof, const mj_rel& r, int key_col, unsigned long long* out, uint32_t seed,
             hipStream_t s, bool raw_low = false) {
    if (r.n == 0) return MJ_OK;
    TriKeyArgs K;
    K.key_col = key_col ? r.col1 : r.col0;
    K.val_col = key_col ? r.col0 : r.col1;
    K.stride = r.stride; K.n = r.n; K.seed = seed; K.raw_low = raw_low ? 1u : 0u; K.out = out;
    MJ_LAUNCHM(prof, "k_tri_keys", k_tri_keys, dim3(grid_for(r.n, 256, 16384)), dim3(256), 0, s, K);
    return MJ_OK;
}

struct CasTriLayout {
    RelPart R, S;
    uint32_t* Rgrp;
    uint32_t* ecnt;
    uint32_t* elist;
    unsigned long long* eoff;
    unsigned long long* partial;
    unsigned long long* Tk;
    unsigned long long* tmp;
    uint32_t* rs_hist;
    uint32_t* rs_counts;
    uint32_t* rs_starts;
    uint32_t* flags;
    unsigned long long* ridx;
    RunBuf Trun;
    uint32_t* err;                    // set when |I| on the device is not the plan's
    uint2* I;
    uint64_t i_cap;
    size_t base_bytes;
};

CasTriLayout cas_tri_layout(void* ws, const mj_plan_t& p, uint64_t ws_bytes) {
    Bump B(ws);
    CasTriLayout L;
    take_part(B, L.R, p.n_r, p.log2_nb);
    take_part(B, L.S, p.n_s, p.log2_nb);
    L.Rgrp = B.take<uint32_t>(std::max<uint64_t>(p.n_r, 1));
    L.ecnt = B.take<uint32_t>(std::max<uint64_t>(p.n_s, 1));
    L.elist = B.take<uint32_t>(std::max<uint64_t>(p.n_s, 1));
    L.eoff = B.take<unsigned long long>(p.n_s + 1);
    const uint64_t nmax = std::max<uint64_t>({p.n_s, p.n_t, 1});
    L.partial = B.take<unsigned long long>((nmax + SCAN_TILE - 1) / SCAN_TILE + 1);
    L.Tk = B.take<unsigned long long>(std::max<uint64_t>(p.n_t, 1));
    L.tmp = B.take<unsigned long long>(std::max<uint64_t>(p.n_t, 1));
    L.rs_hist = B.take<uint32_t>(256 * ((std::max<uint64_t>(p.n_t, 1) + RS_TILE - 1) / RS_TILE));
    L.rs_counts = B.take<uint32_t>(256);
    L.rs_starts = B.take<uint32_t>(257);
    L.flags = B.take<uint32_t>(std::max<uint64_t>(p.n_t, 1));
    L.ridx = B.take<unsigned long long>(p.n_t + 1);
    take_runs(B, L.Trun, p.n_t, true);
    L.err = B.take<uint32_t>(1);
    L.I = B.take<uint2>(0);
    L.base_bytes = B.off + 256;
    if (ws) {
        L.i_cap = ws_bytes > L.base_bytes ? (ws_bytes - L.base_bytes) / sizeof(uint2) : 0;
    } else {
        L.i_cap = std::max<uint64_t>(1, std::min<uint64_t>(p.join2_size, CAS_DEFAULT_I_CAP));
    }
    return L;
}

int tri_prepare(Prof* prof, int num_cu, const mj_rel& R, const mj_rel& S, const mj_rel& T,
                const mj_plan_t& p, const TriLayout& L, unsigned long long* out, hipStream_t s) {
    (void)num_cu; (void)out;
    int st;
    const uint32_t seed = p.seed;
    // keys: R -> (m(b), m(a)), S -> (m(b), m(c)) and (m(c), m(b)), T -> (m(c), m(a)).
    // An array made from the same (key column, other column) as an earlier
    // one -- R = S = T as one symmetric relation gives two distinct arrays,
    // not four -- is copied from it instead of sorted again.
    struct KeySrc { const mj_rel* r; int key_col; unsigned long long* dst; };
    const KeySrc src[4] = {{&R, 1, L.Rk}, {&S, 0, L.Sk}, {&S, 1, L.Sk2}, {&T, 0, L.Tk}};
    auto cols = [](const KeySrc& k, const uint32_t*& kc, const uint32_t*& vc) {
        kc = k.key_col ? k.r->col1 : k.r->col0;
        vc = k.key_col ? k.r->col0 : k.r->col1;
    };
    for (int i = 0; i < 4; ++i) {
        const uint32_t *ki, *vi;
        cols(src[i], ki, vi);
        int same = -1;
        for (int j = 0; j < i && same < 0; ++j) {
            const uint32_t *kj, *vj;
            cols(src[j], kj, vj);
            if (ki == kj && vi == vj && src[i].r->stride == src[j].r->stride && src[i].r->n == src[j].r->n)
                same = j;
        }
        const uint64_t n = src[i].r->n;
        if (same >= 0) {
            if (n)
                MJ_LAUNCHM(prof, "k_copy_u64", k_copy_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s,
                           src[i].dst, src[same].dst, n);
            continue;
        }
        if ((st = tri_keys(prof, *src[i].r, src[i].key_col, src[i].dst, seed, s))) return st;
        if ((st = launch_radix_sort(prof, src[i].dst, L.tmp, n, L.rs_hist, L.rs_counts, L.rs_starts, s)))
            return st;
    }
    // lists of R per B and of T per C; groups of S per B and per C
    if ((st = launch_runs(prof, L, L.Rk, R.n, L.R, L.Rl, s))) return st;
    if ((st = launch_runs(prof, L, L.Tk, T.n, L.T, L.Tl, s))) return st;
    if ((st = launch_runs(prof, L, L.Sk, S.n, L.S, L.Sl, s))) return st;
    if ((st = launch_runs(prof, L, L.Sk2, S.n, L.S2, L.Sl2, s))) return st;
    // work queues of the two passes
    for (int q = 0; q < 2; ++q) {
        const PassBuf& P = L.P[q];
        MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, P.ctr, (uint64_t)4, 0u);
        MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(grid_for(P.n_heavy_cap, 256, 4096)), dim3(256), 0, s,
                  P.heavy_items, (uint64_t)P.n_heavy_cap, 0u);
        TriClassifyArgs C;
        C.Stg = run_index(q == 0 ? L.R : L.T);
        C.Grp = run_index(q == 0 ? L.S : L.S2);
        C.share = 1u << p.log2_share;
        C.nlight = P.ctr + 0; C.light = P.light;
        C.nheavy_groups = P.ctr + 2; C.heavy_group = P.heavy_group; C.heavy_items = P.heavy_items;
        MJ_LAUNCHM(prof, "k_tri_classify", k_tri_classify, dim3(grid_for(S.n, 256, 16384)), dim3(256), 0, s, C);
        if ((st = launch_scan_u32(prof, P.heavy_items, P.n_heavy_cap, L.partial, P.heavy_off, s))) return st;
    }
    return MJ_OK;
}

// pass 0 stages R's lists per B (groups: S by B, iterated: T's lists per C,
// taken when strictly shorter); pass 1 stages T's lists per C (groups: S by
// C, iterated: R's lists per B, taken when not longer)
TriJoinArgs tri_join_args(const TriLayout& L, const mj_plan_t& p, unsigned long long* out, int pass) {
    TriJoinArgs J;
    const PassBuf& P = L.P[pass];
    J.Stg = run_index(pass == 0 ? L.R : L.T);
    J.Grp = run_index(pass == 0 ? L.S : L.S2);
    J.Itr = run_index(pass == 0 ? L.T : L.R);
    J.Stgl = pass == 0 ? L.Rl : L.Tl;
    J.Grpl = pass == 0 ? L.Sl : L.Sl2;
    J.Itrl = pass == 0 ? L.Tl : L.Rl;
    J.strict = pass == 0 ? 1u : 0u;
    J.nlight = P.ctr + 0; J.light = P.light; J.light_next = P.ctr + 1;
    J.heavy_group = P.heavy_group; J.heavy_off = P.heavy_off; J.n_heavy_cap = P.n_heavy_cap;
    J.heavy_next = P.ctr + 3; J.share = 1u << p.log2_share; J.total = out;
    return J;
}

int cascade_triangle(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T, uint64_t* out,
                     const mj_plan_t& p, void* ws, uint64_t ws_bytes, void* stream) {
    if (p.log2_nb > PART_MAX_BITS) return MJ_ERR_INVALID_ARG;
    if (!ws) return MJ_ERR_WORKSPACE;
    CasTriLayout L = cas_tri_layout(ws, p, ws_bytes);
    if (ws_bytes < L.base_bytes || (p.join2_size && L.i_cap == 0)) return MJ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prof* prof = &ctx->prof;
    unsigned long long* total = reinterpret_cast<unsigned long long*>(out);
    MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, total, (uint64_t)1, 0ull);
    if (R->n == 0 || S->n == 0 || T->n == 0 || p.join2_size == 0) return MJ_OK;
    // join 2's side: T as sorted (m(c), m(a)) keys with its lists per C
    int st = tri_keys(prof, *T, 0, L.Tk, p.seed, s);
    if (st) return st;
    if ((st = launch_radix_sort(prof, L.Tk, L.tmp, T->n, L.rs_hist, L.rs_counts, L.rs_starts, s))) return st;
    TriLayout TL{};                    // launch_runs only uses flags / ridx / partial
    TL.flags = L.flags; TL.ridx = L.ridx; TL.partial = L.partial;
    if ((st = launch_runs(prof, TL, L.Tk, T->n, L.Trun, nullptr, s))) return st;
    // join 1: as in the linear cascade
    const uint32_t nb = 1u << p.log2_nb;
    PartLaunch P{};
    P.njobs = 2;
    P.job[0] = make_job(*R, L.R.hist, L.R.counts, L.R.starts, 1, seed_b(p), p.log2_nb, 0, 0, 0);
    P.job[0].out_pair = L.R.pairs;
    P.job[1] = make_job(*S, L.S.hist, L.S.counts, L.S.starts, 0, seed_b(p), p.log2_nb, 0, 0, 0);
    P.job[1].out_pair = L.S.pairs;
    if ((st = launch_partition(prof, "rs", P, s))) return st;
    CasIndexArgs X;
    X.R = L.R.pairs; X.rstarts = L.R.starts; X.S = L.S.pairs; X.sstarts = L.S.starts;
    X.Rgrp = L.Rgrp; X.ecnt = L.ecnt; X.elist = L.elist; X.seed = seed_w(p);
    MJ_LAUNCHM(prof, "k_cas_index", k_cas_index, dim3(nb), dim3(CAS_THREADS), 0, s, X);
    if ((st = launch_scan_u32(prof, L.ecnt, S->n, L.partial, L.eoff, s))) return st;
    MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, L.err, (uint64_t)1, 0u);
    MJ_LAUNCHM(prof, "k_check_size", k_check_size, dim3(1), dim3(64), 0, s, L.eoff + S->n,
              (unsigned long long)p.join2_size, L.err);
    const uint64_t totI = p.join2_size;
    for (uint64_t lo = 0; lo < totI; lo += L.i_cap) {
        const uint64_t hi = std::min<uint64_t>(totI, lo + L.i_cap);
        CasExpandArgs E;
        E.eoff = L.eoff; E.elist = L.elist; E.Rgrp = L.Rgrp; E.S = L.S.pairs; E.ns = S->n;
        E.lo = lo; E.hi = hi; E.I = L.I; E.swap = 0;
        MJ_LAUNCHM(prof, "k_cas_expand", k_cas_expand, dim3((uint32_t)((hi - lo + EXP_TILE - 1) / EXP_TILE)),
                  dim3(EXP_THREADS), 0, s, E);
        CasProbeTriArgs Q;
        Q.I = L.I; Q.n = hi - lo; Q.T = run_index(L.Trun); Q.Tk = L.Tk; Q.seed = p.seed; Q.total = total;
        MJ_LAUNCHM(prof, "k_cas_probe_tri", k_cas_probe_tri, dim3(grid_for(hi - lo, 256, 16384)), dim3(256), 0, s, Q);
    }
    // an intermediate of another size than the plan's: the total is all ones
    MJ_LAUNCHM(prof, "k_poison_u64", k_poison_u64, dim3(1), dim3(64), 0, s, total, (uint64_t)1, L.err);
    return MJ_OK;
}

// ------------------------------------------------------------- star join
static_assert(STAR_GROUPS == STAR_PLAN_MAX_R, "planner and kernels agree on the star limit");

struct StarLayout {
    TableLayout Rt, Tt;               // one-bucket tables: R on B, T on C
    uint32_t* occ;                    // [R slots + 1]
    unsigned long long* rid;          // [R slots + 2] ids of R's B values
    uint2* idtab;                     // [R slots] (key, id)
    unsigned long long* partial;      // per-block sums (both group-bys)
    unsigned long long* W;            // [w_len] per-B sums, by id of b
    uint64_t w_len;
    unsigned long long* scan_part;
    // binary star cascade
    uint32_t* mult;                   // [n_r + 1] multiplicity per id
    unsigned long long* roff;         // [n_r + 2]
    uint32_t* rcur;                   // [n_r + 1]
    uint32_t* ra;                     // [n_r] R's A values grouped by id
    uint32_t* icnt;                   // [n_s]
    unsigned long long* ioff;         // [n_s + 1]
    uint2* I;                         // [i_cap] (a, c) pairs
    uint64_t i_cap;
    size_t bytes;
};

StarLayout star_layout(void* ws, const mj_plan_t& p, bool cascade) {
    Bump B(ws);
    StarLayout L{};
    take_table(B, L.Rt, p.n_r, 0);
    take_table(B, L.Tt, p.n_t, 0);
    const uint64_t slots = L.Rt.pool_slots;
    L.occ = B.take<uint32_t>(slots + 1);
    L.rid = B.take<unsigned long long>(slots + 2);
    L.idtab = B.take<uint2>(std::max<uint64_t>(slots, 1));
    L.partial = B.take<unsigned long long>(uint64_t(STAR_GRID) * STAR_STRIDE);
    L.w_len = p.n_r + 1;
    L.W = B.take<unsigned long long>(L.w_len);
    const uint64_t nmax = std::max<uint64_t>({slots + 2, p.n_s + 1, p.n_r + 2});
    L.scan_part = B.take<unsigned long long>((nmax + SCAN_TILE - 1) / SCAN_TILE + 1);
    if (cascade) {
        L.mult = B.take<uint32_t>(p.n_r + 1);
        L.roff = B.take<unsigned long long>(p.n_r + 2);
        L.rcur = B.take<uint32_t>(p.n_r + 1);
        L.ra = B.take<uint32_t>(std::max<uint64_t>(p.n_r, 1));
        L.icnt = B.take<uint32_t>(std::max<uint64_t>(p.n_s, 1));
        L.ioff = B.take<unsigned long long>(p.n_s + 1);
        L.i_cap = std::max<uint64_t>(1, std::min<uint64_t>(p.join2_size, STAR_PLAN_MAX_I));
        L.I = B.take<uint2>(L.i_cap);
    }
    L.bytes = B.off + 256;
    return L;
}

StarTable star_table(const TableLayout& T, uint32_t bseed, uint32_t sseed) {
    StarTable X;
    X.dir = T.dir; X.pool = T.pool; X.bkt_seed = bseed; X.slot_seed = sseed;
    X.pool_slots = (uint32_t)T.pool_slots;
    return X;
}

uint32_t star_grid(uint64_t n) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(STAR_GRID, (n + STAR_ROWS_PER_BLOCK - 1) / STAR_ROWS_PER_BLOCK));
}

// both tables, then ids 0..k-1 of R's distinct B values
int star_prepare(Prof* prof, const mj_rel& R, const mj_rel& T, const mj_plan_t& p,
                 const StarLayout& L, hipStream_t s) {
    int st;
    if ((st = launch_tables(prof, L.Rt, R, 1, 0, seed_b(p), seed_slot(p), s))) return st;
    if ((st = launch_tables(prof, L.Tt, T, 0, 0, seed_c(p), seed_slot(p), s))) return st;
    StarOccArgs O;
    O.R = star_table(L.Rt, seed_b(p), seed_slot(p));
    O.cursor = L.Rt.pool_cursor; O.occ = L.occ;
    const uint64_t slots = L.Rt.pool_slots;
    MJ_LAUNCHM(prof, "k_star_occ", k_star_occ, dim3(grid_for(slots + 1, 256, 4096)), dim3(256), 0, s, O);
    if ((st = launch_scan_u32(prof, L.occ, slots + 1, L.scan_part, L.rid, s))) return st;
    StarIdArgs I;
    I.R = O.R; I.rid = L.rid; I.idtab = L.idtab;
    MJ_LAUNCHM(prof, "k_star_ids", k_star_ids, dim3(grid_for(slots, 256, 4096)), dim3(256), 0, s, I);
    return MJ_OK;
}

uint32_t star_grid_cu(uint64_t n, int num_cu) {       // one workgroup per CU at most
    return std::min<uint32_t>(star_grid(n), (uint32_t)std::max(num_cu, 1));
}

// group-by of (key, c) rows weighted by mult_T(c): by B (S, into W per id of
// b) or by A (I, into the counts); `out` receives the sums
int star_group(Prof* prof, const char* name, const uint32_t* col0, const uint32_t* col1,
               int64_t stride, uint64_t n, bool by_b, uint32_t ngroups_max, int num_cu,
               const mj_plan_t& p, const StarLayout& L, unsigned long long* out, uint64_t out_len,
               hipStream_t s) {
    // zeroed first: the LDS modes overwrite, the global modes add
    if (out_len)
        MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(grid_for(out_len, 256, 4096)), dim3(256), 0, s,
                  out, out_len, 0ull);
    StarGroupArgs G;
    G.col0 = col0; G.col1 = col1; G.stride = stride; G.n = n;
    G.T = star_table(L.Tt, seed_c(p), seed_slot(p));
    G.R = star_table(L.Rt, seed_b(p), seed_slot(p));
    G.idtab = L.idtab; G.rid = L.rid; G.ngroups_max = ngroups_max;
    G.partial = L.partial; G.out = out; G.err = L.Rt.err;
    const uint32_t grid = star_grid_cu(n, num_cu);
    if (by_b) MJ_LAUNCHM(prof, name, k_star_group_b, dim3(grid), dim3(STAR_THREADS), 0, s, G);
    else MJ_LAUNCHM(prof, name, k_star_group_a, dim3(grid), dim3(STAR_THREADS), 0, s, G);
    StarReduceArgs Rd;
    Rd.partial = L.partial; Rd.nblocks = grid; Rd.by_b = by_b ? 1u : 0u;
    Rd.rdir = L.Rt.dir; Rd.tdir = L.Tt.dir; Rd.rid = L.rid; Rd.pool_slots = G.R.pool_slots;
    Rd.ngroups_max = ngroups_max; Rd.out = out;
    MJ_LAUNCHM(prof, "k_star_reduce", k_star_reduce, dim3((STAR_STRIDE + 63) / 64), dim3(STAR_REDUCE_THREADS),
              0, s, Rd);
    return MJ_OK;
}

int run_star3(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T, uint32_t a_domain,
              uint64_t* count_out, const mj_plan_t& p, void* ws, uint64_t ws_bytes, hipStream_t s) {
    StarLayout L = star_layout(nullptr, p, false);
    if (!ws || ws_bytes < L.bytes) return MJ_ERR_WORKSPACE;
    if (L.Rt.pool_slots >= 0xFFFFFFF0ull || L.Tt.pool_slots >= 0xFFFFFFF0ull) return MJ_ERR_UNSUPPORTED;
    L = star_layout(ws, p, false);
    Prof* prof = &ctx->prof;
    unsigned long long* count = reinterpret_cast<unsigned long long*>(count_out);
    if (a_domain)
        MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(grid_for(a_domain, 256, 4096)), dim3(256), 0, s,
                  count, (uint64_t)a_domain, 0ull);
    if (R->n == 0 || S->n == 0 || T->n == 0 || a_domain == 0) return MJ_OK;
    int st;
    if ((st = star_prepare(prof, *R, *T, p, L, s))) return st;
    // W[id(b)] = sum of mult_T(c) over S, one pass over the fact relation
    if ((st = star_group(prof, "k_star_group_b", S->col0, S->col1, S->stride, S->n, true, 0, ctx->num_cu,
                         p, L, L.W, L.w_len, s))) return st;
    StarCountArgs C;
    C.col0 = R->col0; C.col1 = R->col1; C.stride = R->stride; C.n = R->n;
    C.R = star_table(L.Rt, seed_b(p), seed_slot(p)); C.rid = L.rid; C.W = L.W;
    C.count = count; C.a_domain = a_domain; C.err = L.Rt.err;
    MJ_LAUNCHM(prof, "k_star_count", k_star_count, dim3(grid_for(R->n, 256, 4096)), dim3(256), 0, s, C);
    // an A value out of range or a table overflow: every count all ones
    MJ_LAUNCHM(prof, "k_poison_u64", k_poison_u64, dim3(grid_for(a_domain, 256, 1024)), dim3(256), 0, s,
              count, (uint64_t)a_domain, L.Rt.err);
    return MJ_OK;
}

int run_star_cascade(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T, uint32_t a_domain,
                     uint64_t* count_out, const mj_plan_t& p, void* ws, uint64_t ws_bytes, hipStream_t s) {
    if (p.join2_size > STAR_PLAN_MAX_I) return MJ_ERR_UNSUPPORTED;
    StarLayout L = star_layout(nullptr, p, true);
    if (!ws || ws_bytes < L.bytes) return MJ_ERR_WORKSPACE;
    if (L.Rt.pool_slots >= 0xFFFFFFF0ull || L.Tt.pool_slots >= 0xFFFFFFF0ull) return MJ_ERR_UNSUPPORTED;
    L = star_layout(ws, p, true);
    Prof* prof = &ctx->prof;
    unsigned long long* count = reinterpret_cast<unsigned long long*>(count_out);
    if (R->n == 0 || S->n == 0 || T->n == 0 || a_domain == 0 || p.join2_size == 0) {
        if (a_domain)
            MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(grid_for(a_domain, 256, 4096)), dim3(256), 0, s,
                      count, (uint64_t)a_domain, 0ull);
        return MJ_OK;
    }
    int st;
    if ((st = star_prepare(prof, *R, *T, p, L, s))) return st;
    // join 1's build side: R's A values grouped by the id of B
    StarRIndexArgs X;
    X.col0 = R->col0; X.col1 = R->col1; X.stride = R->stride; X.n = R->n;
    X.R = star_table(L.Rt, seed_b(p), seed_slot(p)); X.rid = L.rid; X.roff = L.roff;
    X.rcur = L.rcur; X.ra = L.ra;
    MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(grid_for(p.n_r + 1, 256, 4096)), dim3(256), 0, s,
              L.mult, p.n_r + 1, 0u);
    MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(grid_for(p.n_r + 1, 256, 4096)), dim3(256), 0, s,
              L.rcur, p.n_r + 1, 0u);
    MJ_LAUNCHM(prof, "k_star_rmult", k_star_rmult, dim3(grid_for(uint64_t(X.R.pool_slots) + 1, 256, 4096)),
              dim3(256), 0, s, X, L.mult);
    if ((st = launch_scan_u32(prof, L.mult, p.n_r + 1, L.scan_part, L.roff, s))) return st;
    MJ_LAUNCHM(prof, "k_star_rfill", k_star_rfill, dim3(grid_for(R->n, 256, 4096)), dim3(256), 0, s, X);
    // join 1: S streamed, I = R |x| S written as (a, c) pairs
    StarExpandArgs E;
    E.col0 = S->col0; E.col1 = S->col1; E.stride = S->stride; E.n = S->n;
    E.R = X.R; E.idtab = L.idtab; E.rid = L.rid; E.roff = L.roff; E.ra = L.ra; E.icnt = L.icnt;
    E.ioff = L.ioff; E.I = L.I;
    E.i_cap = L.i_cap; E.err = L.Rt.err;
    const uint32_t g1 = star_grid_cu(S->n, ctx->num_cu);
    MJ_LAUNCHM(prof, "k_star_icount", k_star_icount, dim3(g1), dim3(STAR_THREADS), 0, s, E);
    if ((st = launch_scan_u32(prof, L.icnt, S->n, L.scan_part, L.ioff, s))) return st;
    MJ_LAUNCHM(prof, "k_star_expand", k_star_expand, dim3(g1), dim3(STAR_THREADS), 0, s, E);
    MJ_LAUNCHM(prof, "k_check_size", k_check_size, dim3(1), dim3(64), 0, s, L.ioff + S->n,
              (unsigned long long)p.join2_size, L.Rt.err);
    // join 2: I streamed past T, grouped by A
    const uint32_t* icol = reinterpret_cast<const uint32_t*>(L.I);
    if ((st = star_group(prof, "k_star_group_i", icol, icol + 1, 2, std::min<uint64_t>(p.join2_size, L.i_cap),
                         false, a_domain, ctx->num_cu, p, L, count, a_domain, s)))
        return st;
    // an intermediate of another size than the plan's, or an A value out of
    // range: every count all ones
    MJ_LAUNCHM(prof, "k_poison_u64", k_poison_u64, dim3(grid_for(a_domain, 256, 1024)), dim3(256), 0, s,
              count, (uint64_t)a_domain, L.Rt.err);
    return MJ_OK;
}

// ---------------------------------------------- FM distinct count per A
struct FmLayout {
    unsigned long long* Tk;
    unsigned long long* Sk;
    unsigned long long* tmp;
    uint32_t* rs_hist;
    uint32_t* rs_counts;
    uint32_t* rs_starts;
    uint32_t* flags;
    unsigned long long* ridx;
    unsigned long long* partial;
    RunBuf T, S;
    uint32_t* tsk;                    // [T runs][FM_WORDS]
    uint32_t* wsk;                    // [S runs][FM_WORDS]
    RelPart Ra;                       // R by range of A
    uint32_t* err;
    uint32_t a_bits, a_shift;
    bool by_range;
    size_t bytes;
};

// ranges of A of at most 2^FM_RANGE_MAX_SHIFT values, about 32K R tuples
// each, at most 2^PART_MAX_BITS of them; beyond that the sketches are ORed
// straight into the output
void fm_ranges(uint64_t n_r, uint32_t a_domain, uint32_t& bits, uint32_t& shift, bool& by_range) {
    const uint32_t L = ceil_log2(std::max<uint32_t>(a_domain, 1));
    const uint32_t want = ceil_log2((n_r + 32767) / 32768);
    bits = std::max<uint32_t>(std::min<uint32_t>(want, L), L > FM_RANGE_MAX_SHIFT ? L - FM_RANGE_MAX_SHIFT : 0);
    shift = L - bits;
    by_range = bits <= PART_MAX_BITS;
    if (!by_range) { bits = 0; shift = 0; }
}

FmLayout fm_layout(void* ws, uint64_t nr, uint64_t ns, uint64_t nt, uint32_t a_domain) {
    Bump B(ws);
    FmLayout L{};
    const uint64_t nmax = std::max<uint64_t>({nr, ns, nt, 1});
    L.Tk = B.take<unsigned long long>(std::max<uint64_t>(nt, 1));
    L.Sk = B.take<unsigned long long>(std::max<uint64_t>(ns, 1));
    L.tmp = B.take<unsigned long long>(nmax);
    const uint64_t ntiles = (nmax + RS_TILE - 1) / RS_TILE;
    L.rs_hist = B.take<uint32_t>(256 * ntiles);
    L.rs_counts = B.take<uint32_t>(256);
    L.rs_starts = B.take<uint32_t>(257);
    L.flags = B.take<uint32_t>(nmax);
    L.ridx = B.take<unsigned long long>(nmax + 1);
    L.partial = B.take<unsigned long long>((nmax + SCAN_TILE - 1) / SCAN_TILE + 1);
    take_runs(B, L.T, nt, true);
    take_runs(B, L.S, ns, true);
    L.tsk = B.take<uint32_t>(std::max<uint64_t>(nt, 1) * FM_WORDS);
    L.wsk = B.take<uint32_t>(std::max<uint64_t>(ns, 1) * FM_WORDS);
    fm_ranges(nr, a_domain, L.a_bits, L.a_shift, L.by_range);
    take_part(B, L.Ra, nr, L.a_bits);
    L.err = B.take<uint32_t>(1);
    L.bytes = B.off + 256;
    return L;
}

// ------------------------------------------ linear join, direct-indexed tables
// T by range of C, S by range of B and R by range of A in one partition
// launch group (identical partitions made once); then deg[c] over T,
// W[b] = sum of deg[s.c] over S, and count[a] = sum of W[r.b] over R, each
// one range per workgroup in LDS.
int run_dense(Prof* prof, const mj_rel& R, const mj_rel& S, const mj_rel& T, const mj_plan_t& p,
              unsigned long long* count, void* ws, hipStream_t s) {
    DenseLayout L = dense_layout(ws, p);
    // S by range of B, R by range of A, T by range of C: each on its first
    // column.  A partition identical to an earlier one (same columns,
    // stride, size and ranges: R = S = T in a self-join) is not made again;
    // its pairs and starts serve both (T then reads the keys of the pairs).
    auto same = [](const mj_rel& x, uint32_t xb, uint32_t xs, const mj_rel& y, uint32_t yb, uint32_t ys) {
        return same_rel(x, y) && xb == yb && xs == ys;
    };
    PartLaunch P{};
    P.njobs = 0;
    P.clear = L.err; P.nclear = 3;                   // the flags, cleared by the first launch
    P.job[P.njobs] = make_job(S, L.S.hist, L.S.counts, L.S.starts, 0, 0, L.b_bits, 0, 0, 0);
    P.job[P.njobs].range_on = 1; P.job[P.njobs].range_shift = L.b_shift;
    P.job[P.njobs].split = L.Ssplit;
    P.job[P.njobs++].out_pair = L.S.pairs;
    const bool r_is_s = same(R, L.a_bits, L.a_shift, S, L.b_bits, L.b_shift);
    if (!r_is_s) {
        P.job[P.njobs] = make_job(R, L.R.hist, L.R.counts, L.R.starts, 0, 0, L.a_bits, 0, 0, 0);
        P.job[P.njobs].range_on = 1; P.job[P.njobs].range_shift = L.a_shift;
        P.job[P.njobs].split = L.Rsplit;
        P.job[P.njobs++].out_pair = L.R.pairs;
    }
    const bool t_is_s = same(T, L.c_bits, L.c_shift, S, L.b_bits, L.b_shift);
    const bool t_is_r = !t_is_s && same(T, L.c_bits, L.c_shift, R, L.a_bits, L.a_shift);
    if (!t_is_s && !t_is_r) {
        P.job[P.njobs] = make_job(T, L.T.hist, L.T.counts, L.T.starts, 0, 0, L.c_bits, 0, 0, 0);
        P.job[P.njobs].range_on = 1; P.job[P.njobs].range_shift = L.c_shift;
        P.job[P.njobs].split = L.Tsplit;
        P.job[P.njobs].out_single = L.tkeys; P.job[P.njobs++].single_col = 0;
    }
    int st = launch_partition(prof, "dense", P, s);
    if (st) return st;
    const RelPart& Rp = r_is_s ? L.S : L.R;
    const RelPart* Tp = t_is_s ? &L.S : (t_is_r ? &Rp : nullptr);
    // the work items of each sum: those of the partition it reads
    const BucketItems& Rsp = r_is_s ? L.Ssplit : L.Rsplit;
    const BucketItems& Tsp = t_is_s ? L.Ssplit : (t_is_r ? Rsp : L.Tsplit);
    const uint64_t n_rp = r_is_s ? S.n : R.n;
    const uint64_t n_tp = t_is_s ? S.n : (t_is_r ? n_rp : T.n);
    RangeAccArgs<uint32_t, uint16_t, uint32_t, uint16_t> Ad{};
    Ad.pairs = Tp ? Tp->pairs : nullptr; Ad.keys = Tp ? nullptr : L.tkeys;
    Ad.starts = Tp ? Tp->starts : L.T.starts; Ad.shift = L.c_shift;
    Ad.domain = p.c_domain; Ad.table = nullptr; Ad.table_n = 0; Ad.out = L.deg; Ad.err = L.err;
    Ad.out_narrow = L.deg16; Ad.wide = L.err + 2; Ad.table_narrow = nullptr; Ad.use_wide = nullptr;
    Ad.split = Tsp; Ad.rows = L.rows; Ad.row_len = 1u << L.c_shift;
    MJ_LAUNCHM(prof, "k_range_deg", k_range_deg, dim3(split_grid(n_tp, L.c_bits)), dim3(RANGE_THREADS),
              size_t(4) << L.c_shift, s, Ad);
    RangeAccArgs<uint32_t, uint16_t, unsigned long long, uint16_t> Aw{};
    Aw.pairs = L.S.pairs; Aw.keys = nullptr; Aw.starts = L.S.starts; Aw.shift = L.b_shift;
    Aw.domain = p.b_domain; Aw.table = L.deg; Aw.table_n = p.c_domain; Aw.out = L.w; Aw.err = L.err;
    // deg's 2-byte copy unless some deg[c] needs more; W's saturating 2-byte copy
    Aw.out_narrow = L.w16; Aw.wide = nullptr; Aw.table_narrow = L.deg16; Aw.use_wide = L.err + 2;
    Aw.split = L.Ssplit; Aw.rows = L.rows; Aw.row_len = 1u << L.b_shift;
    MJ_LAUNCHM(prof, "k_range_w", k_range_w, dim3(split_grid(S.n, L.b_bits)), dim3(RANGE_THREADS),
              size_t(8) << L.b_shift, s, Aw);
    RangeAccArgs<unsigned long long, uint16_t, unsigned long long, uint32_t> Ac{};
    Ac.pairs = Rp.pairs; Ac.keys = nullptr; Ac.starts = Rp.starts; Ac.shift = L.a_shift;
    Ac.domain = p.a_domain; Ac.table = L.w; Ac.table_n = p.b_domain; Ac.out = count; Ac.err = L.err;
    // W's saturating 2-byte copy; the full W where it reads 0xFFFF
    Ac.out_narrow = nullptr; Ac.wide = nullptr; Ac.table_narrow = L.w16; Ac.use_wide = nullptr;
    Ac.split = Rsp; Ac.rows = L.rows; Ac.row_len = 1u << L.a_shift;
    MJ_LAUNCHM(prof, "k_range_count", k_range_count, dim3(split_grid(n_rp, L.a_bits)), dim3(RANGE_THREADS),
              size_t(8) << L.a_shift, s, Ac);
    // a key beyond its certified bound: every count all ones
    MJ_LAUNCHM(prof, "k_poison_u64", k_poison_u64, dim3(grid_for(p.a_domain, 256, 1024)), dim3(256), 0, s,
              count, (uint64_t)p.a_domain, L.err);
    return MJ_OK;
}

// --------------------------------------------- degree-oriented cyclic join
struct OrientLayout {
    unsigned long long *K, *K2, *tmp;  // sorted degrees: the keys (m(u), m(v)) and the sort's buffers
    uint32_t *rs_hist, *rs_counts, *rs_starts;
    RunBuf U;
    RelPart V;                         // dense ids: the first ends by range of id ...
    uint32_t* vkeys;
    uint32_t* deg;                     // ... and each vertex's degree, [vdom]
    uint32_t v_bits, v_shift;
    uint32_t* flags;
    unsigned long long *ridx, *partial;
    uint2* E;                          // kept edges (at most n)
    uint32_t* err;
    size_t bytes;
};

// Vertex ids below a small bound found by the planner: degrees from a
// direct-indexed array instead of a sort.
bool orient_dense(const mj_plan_t& p, uint32_t& bits, uint32_t& shift) {
    return (p.flags & MJ_PLAN_DENSE_KEYS) && (p.flags & MJ_PLAN_SYMMETRIC_SIMPLE) && p.b_domain &&
           key_ranges(p.n_r, p.b_domain, bits, shift);
}

// with_check: the second key array of the planner's symmetry check;
// vdom > 0: the dense form (degrees by range of id, no sort)
OrientLayout orient_layout(void* ws, uint64_t n, bool with_check, uint32_t vdom = 0) {
    Bump B(ws);
    OrientLayout L{};
    const uint64_t m = std::max<uint64_t>(n, 1);
    if (vdom && key_ranges(n, vdom, L.v_bits, L.v_shift)) {
        const uint32_t nb = 1u << L.v_bits;
        L.V.hist = B.take<uint32_t>(uint64_t(nb) * ntiles_of(n));
        L.V.counts = B.take<uint32_t>(nb);
        L.V.starts = B.take<uint32_t>(nb + 1);
        L.vkeys = B.take<uint32_t>(m);
        L.deg = B.take<uint32_t>(vdom);
    } else {
        L.K = B.take<unsigned long long>(m);
        L.K2 = with_check ? B.take<unsigned long long>(m) : nullptr;
        L.tmp = B.take<unsigned long long>(m);
        L.rs_hist = B.take<uint32_t>(256 * ((m + RS_TILE - 1) / RS_TILE));
        L.rs_counts = B.take<uint32_t>(256);
        L.rs_starts = B.take<uint32_t>(257);
        take_runs(B, L.U, n, true);
    }
    L.flags = B.take<uint32_t>(m);
    L.ridx = B.take<unsigned long long>(m + 1);
    L.partial = B.take<unsigned long long>((m + SCAN_TILE - 1) / SCAN_TILE + 1);
    L.E = B.take<uint2>(m);
    L.err = B.take<uint32_t>(1);
    L.bytes = (B.off + 511) & ~size_t(255);      // a multiple of 256: the cyclic join's layout follows
    return L;
}

// the plan of the cyclic join over the kept edges
mj_plan_t oriented_inner(const mj_plan_t& p) {
    mj_plan_t q = p;
    q.algo = MJ_ALGO_3WAY;
    q.n_r = q.n_s = q.n_t = p.n_r / 2;
    return q;
}

uint32_t oriented_vdom(const mj_plan_t& p) {
    uint32_t bits, shift;
    return orient_dense(p, bits, shift) ? p.b_domain : 0u;
}

size_t oriented_bytes(const mj_plan_t& p) {
    return orient_layout(nullptr, p.n_r, false, oriented_vdom(p)).bytes +
           tri_layout(nullptr, oriented_inner(p)).bytes;
}

// Is R = S = T one symmetric relation without duplicates or loops?  Sorts
// (m(u), m(v)) and (m(v), m(u)) fully and compares them (synchronous).
int symmetric_simple(Prof* prof, const mj_rel& E, uint32_t seed, void* ws, bool& yes, hipStream_t s) {
    OrientLayout L = orient_layout(ws, E.n, true);
    int st;
    if ((st = tri_keys(prof, E, 0, L.K, seed, s))) return st;
    if ((st = tri_keys(prof, E, 1, L.K2, seed, s))) return st;
    if ((st = launch_radix_sort(prof, L.K, L.tmp, E.n, L.rs_hist, L.rs_counts, L.rs_starts, s))) return st;
    if ((st = launch_radix_sort(prof, L.K2, L.tmp, E.n, L.rs_hist, L.rs_counts, L.rs_starts, s))) return st;
    MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, L.err, (uint64_t)1, 0u);
    MJ_LAUNCH(prof, "k_sym_check", k_sym_check, dim3(grid_for(E.n, 256, 8192)), dim3(256), 0, s, L.K, L.K2,
              E.n, L.err);
    uint32_t bad = 1;
    MJ_HIP(hipMemcpyAsync(&bad, L.err, 4, hipMemcpyDeviceToHost, s));
    MJ_HIP(hipStreamSynchronize(s));
    yes = bad == 0;
    return MJ_OK;
}

int run_oriented(Prof* prof, int num_cu, const mj_rel& Erel, const mj_plan_t& p, unsigned long long* out,
                 void* ws, hipStream_t s) {
    const uint32_t vdom = oriented_vdom(p);
    OrientLayout O = orient_layout(ws, Erel.n, false, vdom);
    const mj_plan_t q = oriented_inner(p);
    TriLayout L = tri_layout(static_cast<char*>(ws) + O.bytes, q);
    int st;
    MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, O.err, (uint64_t)1, 0u);
    OrientArgs A{};
    A.c0 = Erel.col0; A.c1 = Erel.col1; A.stride = Erel.stride; A.n = Erel.n;
    A.seed = p.seed;
    A.flags = O.flags; A.ridx = O.ridx; A.E = O.E; A.err = O.err; A.total = out;
    if (vdom) {
        // degrees: the first ends partitioned by range of id, counted per
        // range in LDS (an id at or above vdom raises err)
        PartLaunch P{};
        P.njobs = 1;
        P.job[0] = make_job(Erel, O.V.hist, O.V.counts, O.V.starts, 0, 0, O.v_bits, 0, 0, 0);
        P.job[0].range_on = 1; P.job[0].range_shift = O.v_shift;
        P.job[0].out_single = O.vkeys; P.job[0].single_col = 0;
        if ((st = launch_partition(prof, "orient", P, s))) return st;
        RangeAccArgs<uint32_t, uint16_t, uint32_t, uint16_t> Ad{};
        Ad.pairs = nullptr; Ad.keys = O.vkeys; Ad.starts = O.V.starts; Ad.shift = O.v_shift;
        Ad.domain = vdom; Ad.table = nullptr; Ad.table_n = 0; Ad.out = O.deg; Ad.err = O.err;
        Ad.out_narrow = nullptr; Ad.wide = nullptr; Ad.table_narrow = nullptr; Ad.use_wide = nullptr;
        MJ_LAUNCHM(prof, "k_range_deg", k_range_deg, dim3(1u << O.v_bits), dim3(RANGE_THREADS),
                  size_t(4) << O.v_shift, s, Ad);
        A.deg = O.deg; A.vdom = vdom;
        MJ_LAUNCHM(prof, "k_orient_flags_dense", k_orient_flags_dense,
                  dim3(grid_for((Erel.n + 3) / 4, 256, 16384)), dim3(256), 0, s, A);
    } else {
        // degrees: runs of m(u) over the relation (grouped on the high word)
        if ((st = tri_keys(prof, Erel, 0, O.K, p.seed, s))) return st;
        if ((st = launch_radix_sort(prof, O.K, O.tmp, Erel.n, O.rs_hist, O.rs_counts, O.rs_starts, s, 4)))
            return st;
        TriLayout TL{};
        TL.flags = O.flags; TL.ridx = O.ridx; TL.partial = O.partial;
        if ((st = launch_runs(prof, TL, O.K, Erel.n, O.U, nullptr, s))) return st;
        A.U = run_index(O.U);
        MJ_LAUNCHM(prof, "k_orient_flags", k_orient_flags, dim3(grid_for((Erel.n + 1) / 2, 256, 16384)),
                  dim3(256), 0, s, A);
    }
    if ((st = launch_scan_u32(prof, O.flags, Erel.n, O.partial, O.ridx, s))) return st;
    MJ_LAUNCHM(prof, "k_orient_compact", k_orient_compact, dim3(grid_for(Erel.n, 256, 16384)), dim3(256), 0, s, A);
    // R' = the kept edges reversed, S' = T' = the kept edges
    mj_rel Rp, Sp;
    Sp.col0 = reinterpret_cast<const uint32_t*>(O.E);
    Sp.col1 = Sp.col0 + 1;
    Sp.n = q.n_s;
    Sp.stride = 2;
    Rp = Sp;
    std::swap(Rp.col0, Rp.col1);
    if (q.n_s) {
        if ((st = tri_prepare(prof, num_cu, Rp, Sp, Sp, q, L, out, s))) return st;
        const uint32_t persistent = (uint32_t)num_cu * 8;
        for (int pass = 0; pass < 2; ++pass) {
            TriJoinArgs J = tri_join_args(L, q, out, pass);
            MJ_LAUNCHM(prof, "k_tri_light", k_tri_light, dim3(persistent), dim3(TRI_THREADS), 0, s, J);
            MJ_LAUNCHM(prof, "k_tri_heavy", k_tri_heavy, dim3((uint32_t)num_cu * 2), dim3(TRI_HEAVY_THREADS), 0, s,
                      J);
        }
    }
    MJ_LAUNCHM(prof, "k_orient_finish", k_orient_finish, dim3(1), dim3(64), 0, s, A, q.n_s);
    return MJ_OK;
}

// --------------------------------------------------- materialised linear join
struct EmitLayout {
    unsigned long long *Sk, *Tk, *tmp;
    uint32_t *rs_hist, *rs_counts, *rs_starts;
    uint32_t* flags;
    unsigned long long *ridx, *partial;
    RunBuf S, T;
    uint32_t *sc, *td, *tdeg, *tst, *sst, *pdeg;
    unsigned long long *P_S, *wout, *O_I, *O_R;
    ulonglong4* tiles;
    size_t bytes;
};

EmitLayout emit_layout(void* ws, uint64_t nr, uint64_t ns, uint64_t nt) {
    Bump B(ws);
    EmitLayout L{};
    const uint64_t nmax = std::max<uint64_t>({nr, ns, nt, 1});
    L.Sk = B.take<unsigned long long>(std::max<uint64_t>(ns, 1));
    L.Tk = B.take<unsigned long long>(std::max<uint64_t>(nt, 1));
    L.tmp = B.take<unsigned long long>(nmax);
    const uint64_t ntiles = (nmax + RS_TILE - 1) / RS_TILE;
    L.rs_hist = B.take<uint32_t>(256 * ntiles);
    L.rs_counts = B.take<uint32_t>(256);
    L.rs_starts = B.take<uint32_t>(257);
    L.flags = B.take<uint32_t>(nmax);
    L.ridx = B.take<unsigned long long>(nmax + 1);
    L.partial = B.take<unsigned long long>((nmax + SCAN_TILE - 1) / SCAN_TILE + 1);
    take_runs(B, L.S, ns, true);
    take_runs(B, L.T, nt, true);
    L.sc = B.take<uint32_t>(std::max<uint64_t>(ns, 1));
    L.td = B.take<uint32_t>(std::max<uint64_t>(nt, 1));
    L.tdeg = B.take<uint32_t>(std::max<uint64_t>(ns, 1));
    L.tst = B.take<uint32_t>(std::max<uint64_t>(ns, 1));
    L.P_S = B.take<unsigned long long>(ns + 1);
    L.sst = B.take<uint32_t>(std::max<uint64_t>(nr, 1));
    L.pdeg = B.take<uint32_t>(std::max<uint64_t>(nr, 1));
    L.wout = B.take<unsigned long long>(std::max<uint64_t>(nr, 1));
    L.O_I = B.take<unsigned long long>(nr + 1);
    L.O_R = B.take<unsigned long long>(nr + 1);
    L.tiles = B.take<ulonglong4>(EMIT_CHUNK_TILES);
    L.bytes = B.off + 256;
    return L;
}

}  // namespace

// =================================================================== API
extern "C" {

const char* mj_status_str(int s) {
    switch (s) {
        case MJ_OK: return "MJ_OK";
        case MJ_ERR_INVALID_ARG: return "MJ_ERR_INVALID_ARG";
        case MJ_ERR_KEY_RANGE: return "MJ_ERR_KEY_RANGE";
        case MJ_ERR_WORKSPACE: return "MJ_ERR_WORKSPACE";
        case MJ_ERR_PLAN_MISMATCH: return "MJ_ERR_PLAN_MISMATCH";
        case MJ_ERR_HIP: return "MJ_ERR_HIP";
        case MJ_ERR_OVERFLOW: return "MJ_ERR_OVERFLOW";
        case MJ_ERR_UNSUPPORTED: return "MJ_ERR_UNSUPPORTED";
        default: return "MJ_ERR_UNKNOWN";
    }
}

int mj_ctx_create(int device, mj_ctx** out) {
    if (!out) return MJ_ERR_INVALID_ARG;
    *out = nullptr;
    mj_ctx* c = new (std::nothrow) mj_ctx();
    if (!c) return MJ_ERR_HIP;
    hipError_t e;
    if (device < 0) {
        e = hipGetDevice(&c->device);
    } else {
        c->device = device;
        e = hipSetDevice(device);
    }
    if (e != hipSuccess) { delete c; return MJ_ERR_HIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
    for (const void* f : {reinterpret_cast<const void*>(&k_part_scatter), reinterpret_cast<const void*>(&k_part_scatter_multi)})
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)part_scatter_smem(PART_MAX_BITS));
    for (const void* f : {reinterpret_cast<const void*>(&k_rs_small), reinterpret_cast<const void*>(&k_rs_small_multi)})
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(RS_SMALL * sizeof(unsigned long long)));
    (void)hipGetLastError();   // an unsupported size only matters if a launch needs it
    // the scratch array's address on this device (the device is current here)
    e = hipGetSymbolAddress(&c->static_scratch, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !c->static_scratch) { delete c; return MJ_ERR_HIP; }
    *out = c;
    return MJ_OK;
}

int mj_ctx_destroy(mj_ctx* ctx) {
    if (!ctx) return MJ_ERR_INVALID_ARG;
    hipDeviceSynchronize();
    for (void* h : ctx->pinned) (void)hipHostFree(h);
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    if (ctx->stage_read) (void)hipEventDestroy(ctx->stage_read);
    delete ctx;
    return MJ_OK;
}

int mj_ctx_profile(mj_ctx* ctx, int enable) {
    if (!ctx) return MJ_ERR_INVALID_ARG;
    ctx->prof.collect();
    ctx->prof.on = enable != 0;
    if (!enable) ctx->prof.total.clear();
    return MJ_OK;
}

int mj_ctx_profile_read(mj_ctx* ctx, int max_entries, char* names, double* total_ms,
                        int64_t* launches) {
    if (!ctx || max_entries < 0) return MJ_ERR_INVALID_ARG;
    ctx->prof.collect();
    int k = 0;
    for (auto& kv : ctx->prof.total) {
        if (k >= max_entries) break;
        if (names) {
            std::strncpy(names + 32 * k, kv.first.c_str(), 31);
            names[32 * k + 31] = 0;
        }
        if (total_ms) total_ms[k] = kv.second.first;
        if (launches) launches[k] = kv.second.second;
        ++k;
    }
    ctx->prof.total.clear();
    return k;
}

uint64_t mj_join2_size_workspace(uint64_t n_r, uint64_t n_s) {
    (void)n_s;
    mj_plan_t p{};
    p.n_t = n_r;
    p.log2_nc = join2_bits(n_r);
    Bump B(nullptr);
    TableLayout L;
    take_table(B, L, n_r, p.log2_nc);
    B.take<unsigned long long>(1);
    return B.off + 256;
}

int mj_join2_size(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, uint64_t* out,
                  void* ws, uint64_t ws_bytes, void* stream) {
    if (!ctx || !out) return MJ_ERR_INVALID_ARG;
    int st = check_rel(R); if (st) return st;
    st = check_rel(S); if (st) return st;
    if (!ws && (R->n || S->n)) return MJ_ERR_INVALID_ARG;
    const uint32_t bits = join2_bits(R->n);
    Bump B(ws);
    TableLayout L;
    take_table(B, L, R->n, bits);
    unsigned long long* total = B.take<unsigned long long>(1);
    if (B.off + 256 > ws_bytes) return MJ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint32_t bseed = 0xA511E9B3u, sseed = 0x63D83595u;
    // degrees of R.b as a bucketed multiplicity table, then sum over S.b
    st = launch_tables(&ctx->prof, L, *R, 1, bits, bseed, sseed, s);
    if (st) return st;
    MJ_LAUNCHM(&ctx->prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, total, (uint64_t)1, 0ull);
    if (S->n) {
        ProbeSumArgs P;
        P.col = S->col0; P.stride = S->stride; P.n = S->n;
        P.dir = L.dir; P.pool = L.pool;
        P.bkt_seed = bseed; P.bkt_bits = bits; P.slot_seed = sseed;
        P.total = total;
        MJ_LAUNCH(&ctx->prof, "k_probe_sum", k_probe_sum, dim3(grid_for(S->n, 256, 4096)), dim3(256), 0, s, P);
    }
    unsigned long long h = 0;
    MJ_HIP(hipMemcpyAsync(&h, total, 8, hipMemcpyDeviceToHost, s));
    MJ_HIP(hipStreamSynchronize(s));
    *out = h;
    return MJ_OK;
}

// The planning workspace: a few statistics words, the learned planner's
// features and outputs, then one scratch region for the largest of the
// planning steps (the |R join S| tables, the symmetry check of a cyclic
// relation, the degree sketch).
struct PlanLayout {
    uint32_t* stats;
    float* feat;                      // [MLP_IN] features, then [MLP_OUT] outputs
    void* scratch;
    size_t scratch_bytes;
    size_t bytes;
};

static PlanLayout plan_layout(void* ws, int kind, uint64_t n_r, uint64_t n_s, uint64_t n_t) {
    Bump B(ws);
    PlanLayout L;
    L.stats = B.take<uint32_t>(64);
    L.feat = B.take<float>(MLP_IN + MLP_OUT);
    size_t need = mj_join2_size_workspace(n_r, n_s);
    if (kind == MJ_TRIANGLE && n_r >= 2) need = std::max<size_t>(need, orient_layout(nullptr, n_r, true).bytes);
    need = std::max<size_t>(need, mj_sketch_workspace(n_r, n_s, n_t));
    L.scratch = B.take<char>(need);
    L.scratch_bytes = need;
    L.bytes = B.off + 256;
    return L;
}

uint64_t mj_plan_workspace(int kind, uint64_t n_r, uint64_t n_s, uint64_t n_t) {
    return plan_layout(nullptr, kind, n_r, n_s, n_t).bytes;
}

int mj_plan(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
            uint32_t a_domain, int planner, mj_plan_t* plan, void* plan_ws, uint64_t plan_ws_bytes,
            void* stream) {
    if (!ctx || !plan) return MJ_ERR_INVALID_ARG;
    int st;
    if ((st = check_rel(R)) || (st = check_rel(S)) || (st = check_rel(T))) return st;
    if (kind != MJ_LINEAR && kind != MJ_TRIANGLE) return MJ_ERR_INVALID_ARG;
    if (planner < MJ_PLANNER_ANALYTIC || planner > MJ_PLANNER_FIXED) return MJ_ERR_INVALID_ARG;
    if (!plan_ws || plan_ws_bytes < plan_layout(nullptr, kind, R->n, S->n, T->n).bytes) return MJ_ERR_WORKSPACE;
    const PlanLayout PL = plan_layout(plan_ws, kind, R->n, S->n, T->n);
    hipStream_t s = static_cast<hipStream_t>(stream);

    mj_plan_t p = planner == MJ_PLANNER_FIXED ? *plan : mj_plan_t{};
    p.kind = kind;
    const uint32_t requests = planner == MJ_PLANNER_FIXED ? (plan->flags & MJ_PLAN_NO_DENSE) : 0u;
    p.flags = requests;                        // properties are found here, never taken on trust
    p.b_domain = p.c_domain = 0;
    p.n_r = R->n; p.n_s = S->n; p.n_t = T->n;
    p.a_domain = kind == MJ_LINEAR ? a_domain : 0;
    p.input_fingerprint = fingerprint(*R, *S, *T);

    if (kind == MJ_LINEAR) {
        if (a_domain == 0 && R->n) return MJ_ERR_KEY_RANGE;
        if (R->n) {
            uint32_t* d = PL.stats;
            MJ_LAUNCHM(&ctx->prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, d, (uint64_t)1, 0u);
            MJ_LAUNCH(&ctx->prof, "k_col_max", k_col_max, dim3(grid_for(R->n, 256, 2048)), dim3(256), 0, s,
                               R->col0, R->stride, R->n, d);
            uint32_t mx = 0;
            MJ_HIP(hipMemcpyAsync(&mx, d, 4, hipMemcpyDeviceToHost, s));
            MJ_HIP(hipStreamSynchronize(s));
            if (mx >= a_domain) return MJ_ERR_KEY_RANGE;
        }
        // B and C in small dense domains: direct-indexed tables
        if (!(requests & MJ_PLAN_NO_DENSE) && R->n && S->n && T->n) {
            uint32_t* d = PL.stats;
            MJ_LAUNCHM(&ctx->prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, d, (uint64_t)2, 0u);
            const mj_rel* src[4] = {R, S, S, T};
            const int col[4] = {1, 0, 1, 0};          // B of R and S, C of S and T
            for (int i = 0; i < 4; ++i) {
                const mj_rel& r = *src[i];
                MJ_LAUNCH(&ctx->prof, "k_col_max", k_col_max, dim3(grid_for(r.n, 256, 2048)), dim3(256), 0, s,
                          col[i] ? r.col1 : r.col0, r.stride, r.n, d + (i < 2 ? 0 : 1));
            }
            uint32_t mx[2] = {0, 0};
            MJ_HIP(hipMemcpyAsync(mx, d, 8, hipMemcpyDeviceToHost, s));
            MJ_HIP(hipStreamSynchronize(s));
            const uint64_t bdom = uint64_t(mx[0]) + 1, cdom = uint64_t(mx[1]) + 1;
            if (dense_ok(bdom, std::max(R->n, S->n)) && dense_ok(cdom, std::max(S->n, T->n))) {
                p.b_domain = (uint32_t)bdom;
                p.c_domain = (uint32_t)cdom;
                p.flags |= MJ_PLAN_DENSE_KEYS;
            }
        }
    }
    // exact size of the binary intermediate (cascade workspace, cost model)
    {
        uint64_t I = 0;
        st = mj_join2_size(ctx, R, S, &I, PL.scratch, PL.scratch_bytes, stream);
        if (st) return st;
        p.join2_size = I;
    }
    // one symmetric relation without duplicates or loops: the degree-oriented
    // cyclic join applies
    if (kind == MJ_TRIANGLE && R->n >= 2 && same_rel(*R, *S) && same_rel(*R, *T)) {
        bool yes = false;
        if ((st = symmetric_simple(&ctx->prof, *R, 0x1B873593u, PL.scratch, yes, s))) return st;
        if (yes) p.flags |= MJ_PLAN_SYMMETRIC_SIMPLE;
        // vertex ids in a small dense domain: the oriented join's degrees by
        // direct index (the relation is symmetric: its first column holds
        // every id)
        if (yes && !(requests & MJ_PLAN_NO_DENSE)) {
            uint32_t* d = PL.stats;
            MJ_LAUNCHM(&ctx->prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, d, (uint64_t)1, 0u);
            MJ_LAUNCH(&ctx->prof, "k_col_max", k_col_max, dim3(grid_for(R->n, 256, 2048)), dim3(256), 0, s,
                      R->col0, R->stride, R->n, d);
            uint32_t mx = 0;
            MJ_HIP(hipMemcpyAsync(&mx, d, 4, hipMemcpyDeviceToHost, s));
            MJ_HIP(hipStreamSynchronize(s));
            const uint64_t vdom = uint64_t(mx) + 1;
            uint32_t bits, shift;
            if (dense_ok(vdom, R->n) && key_ranges(R->n, (uint32_t)vdom, bits, shift)) {
                p.b_domain = (uint32_t)vdom;
                p.flags |= MJ_PLAN_DENSE_KEYS;
            }
        }
    }
    if (planner != MJ_PLANNER_FIXED) {
        st = analytic_plan(kind, p, ctx->num_cu, ctx->model);
        if (st) return st;
        const bool learned_choice = planner == MJ_PLANNER_LEARNED && ctx->planner;
        if (learned_choice) {
            // the network's choice replaces the analytic one; the analytic
            // estimates stay in the plan as its judge
            float* feat = PL.feat;
            float* y = feat + MLP_IN;
            if ((st = mj_sketch(ctx, kind, R, S, T, feat, PL.scratch, PL.scratch_bytes, stream))) return st;
            if ((st = mj_mlp_forward(ctx, ctx->planner, feat, 1, y, stream))) return st;
            float h[MLP_OUT];
            MJ_HIP(hipMemcpyAsync(h, y, sizeof h, hipMemcpyDeviceToHost, s));
            MJ_HIP(hipStreamSynchronize(s));
            p.pred_log2_join2 = h[0];
            p.pred_log2_out = h[1];
            // the plan of largest logit among those this join can take
            bool ok[MLP_NPLAN] = {};
            ok[MJ_ALGO_3WAY] = true;
            ok[MJ_ALGO_CASCADE] = p.join2_size <= CAS_DEFAULT_I_CAP;
            if (kind == MJ_LINEAR) {
                ok[MJ_ALGO_STAR] = p.est_ms_star > 0.0;
                ok[MJ_ALGO_STAR_CASCADE] = p.est_ms_star_cascade > 0.0;
                ok[MJ_ALGO_SLARGE] = p.est_ms_slarge > 0.0;
            } else {
                ok[MJ_ALGO_ORIENTED] = (p.flags & MJ_PLAN_SYMMETRIC_SIMPLE) != 0;
            }
            int best = MJ_ALGO_3WAY;
            for (int k = 0; k < MLP_NPLAN; ++k)
                if (ok[k] && h[MLP_PLAN0 + k] > h[MLP_PLAN0 + best]) best = k;
            // the S-largest plan needs its own bucket counts (set by the
            // analytic planner when it chose it, else derived here)
            if (best == MJ_ALGO_SLARGE && p.algo != MJ_ALGO_SLARGE) {
                uint32_t lr = 0, lt = 0;
                if (slarge_buckets(default_model(), p.n_r, p.n_s, p.n_t, lr, lt, nullptr)) {
                    p.log2_nb = lr;
                    p.log2_nc = lt;
                } else {
                    best = MJ_ALGO_3WAY;
                }
            }
            p.algo = best;
            if (kind == MJ_TRIANGLE) {            // share classes 1, 4, 16
                int bs = 0;
                for (int k = 1; k < 3; ++k) if (h[MLP_SHARE0 + k] > h[MLP_SHARE0 + bs]) bs = k;
                p.log2_share = 2 * bs;
            }
        }
        // an intermediate beyond one workspace-sized chunk is never worth
        // materialising: the three-way join reads each input a bounded
        // number of times
        if (p.algo == MJ_ALGO_CASCADE && p.join2_size > CAS_DEFAULT_I_CAP) p.algo = MJ_ALGO_3WAY;
        // counting each triangle once does less work than either form of
        // the general cyclic join, for the same total, once the relation is
        // large and skewed enough to pay for orienting it
        if (!learned_choice && (p.flags & MJ_PLAN_SYMMETRIC_SIMPLE) && orient_pays(p)) p.algo = MJ_ALGO_ORIENTED;
    } else {
        if (p.log2_nb > PART_MAX_BITS || p.log2_nc > PART_MAX_BITS || p.log2_share > 6)
            return MJ_ERR_INVALID_ARG;
        const bool ok = kind == MJ_LINEAR ? ((p.algo >= MJ_ALGO_3WAY && p.algo <= MJ_ALGO_STAR_CASCADE) ||
                                             p.algo == MJ_ALGO_SLARGE)
                                          : (p.algo == MJ_ALGO_3WAY || p.algo == MJ_ALGO_CASCADE ||
                                             p.algo == MJ_ALGO_ORIENTED);
        if (!ok) return MJ_ERR_INVALID_ARG;
        if (p.algo == MJ_ALGO_SLARGE && p.log2_nb + p.log2_nc > PART_MAX_BITS) return MJ_ERR_INVALID_ARG;
        if (p.algo == MJ_ALGO_ORIENTED && !(p.flags & MJ_PLAN_SYMMETRIC_SIMPLE)) return MJ_ERR_UNSUPPORTED;
    }
    st = plan_workspace(p);
    if (st) return st;
    *plan = p;
    return MJ_OK;
}

int mj_linear3_count(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                     uint32_t a_domain, uint64_t* count, const mj_plan_t* plan,
                     void* ws, uint64_t ws_bytes, void* stream) {
    if (!ctx || !plan || (!count && a_domain)) return MJ_ERR_INVALID_ARG;
    int st;
    if ((st = check_rel(R)) || (st = check_rel(S)) || (st = check_rel(T))) return st;
    const mj_plan_t& p = *plan;
    if (p.kind != MJ_LINEAR || p.n_r != R->n || p.n_s != S->n || p.n_t != T->n ||
        p.a_domain != a_domain || p.input_fingerprint != fingerprint(*R, *S, *T))
        return MJ_ERR_PLAN_MISMATCH;
    if (p.log2_nb > PART_MAX_BITS || p.log2_nc > PART_MAX_BITS || s_part_bits(p) > PART_MAX_BITS)
        return MJ_ERR_INVALID_ARG;
    if (p.algo == MJ_ALGO_STAR)
        return run_star3(ctx, R, S, T, a_domain, count, p, ws, ws_bytes, static_cast<hipStream_t>(stream));
    const bool slarge = p.algo == MJ_ALGO_SLARGE;
    if (slarge) {
        uint32_t ab, as;
        if (!a_ranges(p, ab, as)) return MJ_ERR_UNSUPPORTED;       // needs per-A ranges in LDS
    }
    if (!slarge && dense_plan(p)) {
        if (!ws || ws_bytes < dense_layout(nullptr, p).bytes) return MJ_ERR_WORKSPACE;
        hipStream_t sd = static_cast<hipStream_t>(stream);
        unsigned long long* cnt = reinterpret_cast<unsigned long long*>(count);
        if (R->n == 0 || S->n == 0 || T->n == 0) {
            MJ_LAUNCHM(&ctx->prof, "k_fill_u64", k_fill_u64, dim3(grid_for(a_domain, 256, 4096)), dim3(256), 0, sd,
                      cnt, (uint64_t)a_domain, 0ull);
            return MJ_OK;
        }
        return run_dense(&ctx->prof, *R, *S, *T, p, cnt, ws, sd);
    }
    LinearLayout L = linear_layout(nullptr, p);
    if (ws_bytes < L.bytes || (!ws && L.bytes)) return MJ_ERR_WORKSPACE;
    L = linear_layout(ws, p);
    hipStream_t s = static_cast<hipStream_t>(stream);

    const bool empty = R->n == 0 || S->n == 0 || T->n == 0;
    if (a_domain && (empty || !L.by_range)) {
        MJ_LAUNCHM(&ctx->prof, "k_fill_u64", k_fill_u64, dim3(grid_for(a_domain, 256, 4096)), dim3(256), 0, s,
                           reinterpret_cast<unsigned long long*>(count), (uint64_t)a_domain, 0ull);
    }
    if (empty || a_domain == 0) return MJ_OK;

    const uint32_t nb = 1u << p.log2_nb;
    // T: partition by g(C) and reduce each bucket to C -> multiplicity
    st = launch_tables(&ctx->prof, L.T, *T, 0, p.log2_nc, seed_c(p), seed_slot(p), s);
    if (st) return st;
    if (L.by_range) {
        // S by bucket of B, R by range of A (one group of launches)
        PartLaunch P{};
        P.njobs = 2;
        // S by bucket of B -- and, for the S-largest form, by bucket of C
        // within it (the digit T's tables are bucketed by)
        P.job[0] = slarge ? make_job(*S, L.S.hist, L.S.counts, L.S.starts, 0, seed_b(p), p.log2_nb,
                                     1, seed_c(p), p.log2_nc)
                          : make_job(*S, L.S.hist, L.S.counts, L.S.starts, 0, seed_b(p), p.log2_nb, 0, 0, 0);
        P.job[0].out_pair = L.S.pairs;
        if (!slarge) P.job[0].split = L.Ssplit;          // heavy buckets of B in pieces
        P.job[1] = make_job(*R, L.Ra.hist, L.Ra.counts, L.Ra.starts, 0, 0, L.a_bits, 0, 0, 0);
        P.job[1].range_on = 1;
        P.job[1].range_shift = L.a_shift;
        P.job[1].split = L.Rasplit;
        P.job[1].out_pair = L.Ra.pairs;
        if ((st = launch_partition(&ctx->prof, "rs", P, s))) return st;
        if (slarge) {
            // R's B values as tables per part of R (slots hashed as the W
            // tables are), a zero sum beside each slot; then every (R_i, T_j)
            // pair meets S_ij; then the tables become the W tables
            st = launch_tables(&ctx->prof, L.Rk, *R, 1, p.log2_nb, seed_b(p), seed_w(p), s);
            if (st) return st;
            MJ_LAUNCHM(&ctx->prof, "k_fill_u64", k_fill_u64, dim3(grid_for(L.Rk.pool_slots, 256, 4096)), dim3(256), 0, s,
                      L.wval, (uint64_t)L.Rk.pool_slots, 0ull);
            MJ_LAUNCHM(&ctx->prof, "k_fill_u64", k_fill_u64, dim3(grid_for(nb, 256, 64)), dim3(256), 0, s,
                      L.wspecial, (uint64_t)nb, 0ull);
            SlCellArgs Sc;
            Sc.S = L.S.pairs; Sc.sstarts = L.S.starts; Sc.r_bits = p.log2_nb; Sc.t_bits = p.log2_nc;
            Sc.pieces = sl_pieces(p);
            Sc.rdir = L.Rk.dir; Sc.rpool = L.Rk.pool; Sc.w_seed = seed_w(p); Sc.wval = L.wval;
            Sc.wspecial = L.wspecial; Sc.tdir = L.T.dir; Sc.tpool = L.T.pool; Sc.slot_seed = seed_slot(p);
            const uint32_t grid = (1u << (p.log2_nb + p.log2_nc)) * Sc.pieces;
            MJ_LAUNCH(&ctx->prof, "k_sl_cell", k_sl_cell, dim3(grid), dim3(SL_THREADS), 0, s, Sc);
            MJ_LAUNCH(&ctx->prof, "k_sl_wtables", k_sl_wtables, dim3(nb), dim3(256), 0, s, L.Rk.dir, L.Rk.pool,
                      L.wval, L.wspecial, L.wdir, L.wpool);
        } else {
            // W[b] per bucket of B into the pool (slots [0, W_MIN_CAP) stay empty)
            MJ_LAUNCHM(&ctx->prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s,
                      reinterpret_cast<uint32_t*>(L.wpool), (uint64_t)(4 * W_MIN_CAP), EMPTY_KEY);
            MJ_LAUNCHM(&ctx->prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, L.wcursor, (uint64_t)1,
                      (unsigned long long)W_MIN_CAP);
            WBuildArgs Wb{};
            Wb.S = L.S.pairs; Wb.sstarts = L.S.starts; Wb.ddir = L.T.dir; Wb.dpool = L.T.pool;
            Wb.c_seed = seed_c(p); Wb.c_bits = p.log2_nc; Wb.slot_seed = seed_slot(p); Wb.w_seed = seed_w(p);
            Wb.wdir = L.wdir; Wb.wpool = L.wpool; Wb.wcursor = L.wcursor; Wb.wcap = L.wslots;
            Wb.err = L.T.err;
            Wb.split = L.Ssplit; Wb.rows = L.wrows; Wb.row_special = L.wrow_special;
            MJ_LAUNCH(&ctx->prof, "k_wbuild", k_wbuild, dim3(split_grid(S->n, p.log2_nb)), dim3(CELL_THREADS), 0, s, Wb);
        }
        // per range of A: count[a] = sum of W[r.b], written once
        CountArgs Cn{};
        Cn.R = L.Ra.pairs; Cn.rstarts = L.Ra.starts; Cn.wdir = L.wdir; Cn.wpool = L.wpool;
        Cn.b_seed = seed_b(p); Cn.b_bits = p.log2_nb; Cn.w_seed = seed_w(p);
        Cn.a_shift = L.a_shift; Cn.a_domain = a_domain;
        Cn.count = reinterpret_cast<unsigned long long*>(count);
        Cn.err = L.T.err;
        Cn.split = L.Rasplit; Cn.rows = L.rows;
        MJ_LAUNCH(&ctx->prof, "k_count", k_count, dim3(split_grid(R->n, L.a_bits)), dim3(COUNT_THREADS),
                  (size_t(8) << L.a_shift), s, Cn);
        // an A value out of range or a table overflow: every count all ones
        MJ_LAUNCHM(&ctx->prof, "k_poison_u64", k_poison_u64, dim3(grid_for(a_domain, 256, 1024)), dim3(256), 0, s,
                  Cn.count, (uint64_t)a_domain, L.T.err);
        return MJ_OK;
    }
    // R and S: partition by the bucket of B (one group of launches for both)
    PartLaunch P{};
    P.njobs = 2;
    P.job[0] = make_job(*R, L.R.hist, L.R.counts, L.R.starts, 1, seed_b(p), p.log2_nb, 0, 0, 0);
    P.job[0].out_pair = L.R.pairs;
    P.job[1] = make_job(*S, L.S.hist, L.S.counts, L.S.starts, 0, seed_b(p), p.log2_nb, 0, 0, 0);
    P.job[1].out_pair = L.S.pairs;
    st = launch_partition(&ctx->prof, "rs", P, s);
    if (st) return st;
    // cells: one workgroup per b-bucket
    LinearCellArgs C;
    C.R = L.R.pairs; C.rstarts = L.R.starts; C.S = L.S.pairs; C.sstarts = L.S.starts;
    C.ddir = L.T.dir; C.dpool = L.T.pool;
    C.c_seed = seed_c(p); C.c_bits = p.log2_nc; C.slot_seed = seed_slot(p);
    C.w_seed = seed_w(p);
    C.count = reinterpret_cast<unsigned long long*>(count);
    C.a_domain = a_domain;
    C.err = L.T.err;
    MJ_LAUNCH(&ctx->prof, "k_linear_cell", k_linear_cell, dim3(nb), dim3(CELL_THREADS), 0, s, C);
    MJ_LAUNCHM(&ctx->prof, "k_poison_u64", k_poison_u64, dim3(grid_for(a_domain, 256, 1024)), dim3(256), 0, s,
              C.count, (uint64_t)a_domain, L.T.err);
    return MJ_OK;
}

uint64_t mj_linear3_count_static_max_bytes(void) { return MJ_STATIC_SCRATCH_BYTES; }

int mj_linear3_count_static(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                            uint32_t a_domain, uint64_t* count_per_a, const mj_plan_t* plan, void* stream) {
    if (!ctx || !ctx->static_scratch) return MJ_ERR_INVALID_ARG;
    // the same call with the device's scratch array as its workspace: it
    // returns MJ_ERR_WORKSPACE before any launch when the plan's path needs more
    return mj_linear3_count(ctx, R, S, T, a_domain, count_per_a, plan, ctx->static_scratch,
                            MJ_STATIC_SCRATCH_BYTES, stream);
}

int mj_triangle3_count(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                       uint64_t* total, const mj_plan_t* plan, void* ws, uint64_t ws_bytes,
                       void* stream) {
    if (!ctx || !plan || !total) return MJ_ERR_INVALID_ARG;
    int st;
    if ((st = check_rel(R)) || (st = check_rel(S)) || (st = check_rel(T))) return st;
    const mj_plan_t& p = *plan;
    if (p.kind != MJ_TRIANGLE || p.n_r != R->n || p.n_s != S->n || p.n_t != T->n ||
        p.input_fingerprint != fingerprint(*R, *S, *T))
        return MJ_ERR_PLAN_MISMATCH;
    if (p.log2_share > 16) return MJ_ERR_INVALID_ARG;
    if (p.algo == MJ_ALGO_ORIENTED) {
        if (!(p.flags & MJ_PLAN_SYMMETRIC_SIMPLE) || !same_rel(*R, *S) || !same_rel(*R, *T))
            return MJ_ERR_PLAN_MISMATCH;
        if (!ws || ws_bytes < oriented_bytes(p)) return MJ_ERR_WORKSPACE;
        hipStream_t so = static_cast<hipStream_t>(stream);
        unsigned long long* o = reinterpret_cast<unsigned long long*>(total);
        MJ_LAUNCHM(&ctx->prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, so, o, (uint64_t)1, 0ull);
        if (R->n == 0) return MJ_OK;
        return run_oriented(&ctx->prof, ctx->num_cu, *R, p, o, ws, so);
    }
    TriLayout L = tri_layout(nullptr, p);
    if (ws_bytes < L.bytes || !ws) return MJ_ERR_WORKSPACE;
    L = tri_layout(ws, p);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prof* prof = &ctx->prof;
    unsigned long long* out = reinterpret_cast<unsigned long long*>(total);
    MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, out, (uint64_t)1, 0ull);
    if (R->n == 0 || S->n == 0 || T->n == 0) return MJ_OK;
    if ((st = tri_prepare(prof, ctx->num_cu, *R, *S, *T, p, L, out, s))) return st;
    const uint32_t persistent = (uint32_t)ctx->num_cu * 8;
    for (int pass = 0; pass < 2; ++pass) {
        TriJoinArgs J = tri_join_args(L, p, out, pass);
        MJ_LAUNCHM(prof, "k_tri_light", k_tri_light, dim3(persistent), dim3(TRI_THREADS), 0, s, J);
        MJ_LAUNCHM(prof, "k_tri_heavy", k_tri_heavy, dim3((uint32_t)ctx->num_cu * 2), dim3(TRI_HEAVY_THREADS), 0, s, J);
    }
    return MJ_OK;
}

int mj_cascade2_count(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                      uint32_t a_domain, uint64_t* out, const mj_plan_t* plan,
                      void* ws, uint64_t ws_bytes, void* stream) {
    if (!ctx || !plan || !out) return MJ_ERR_INVALID_ARG;
    int st;
    if ((st = check_rel(R)) || (st = check_rel(S)) || (st = check_rel(T))) return st;
    if (kind != MJ_LINEAR && kind != MJ_TRIANGLE) return MJ_ERR_INVALID_ARG;
    const mj_plan_t& p = *plan;
    if (p.kind != kind || p.n_r != R->n || p.n_s != S->n || p.n_t != T->n ||
        (kind == MJ_LINEAR && p.a_domain != a_domain) || p.input_fingerprint != fingerprint(*R, *S, *T))
        return MJ_ERR_PLAN_MISMATCH;
    if (kind == MJ_TRIANGLE) return cascade_triangle(ctx, R, S, T, out, p, ws, ws_bytes, stream);
    if (p.log2_nb > PART_MAX_BITS || p.log2_nc > PART_MAX_BITS) return MJ_ERR_INVALID_ARG;
    if (p.algo == MJ_ALGO_STAR_CASCADE)
        return run_star_cascade(ctx, R, S, T, a_domain, out, p, ws, ws_bytes, static_cast<hipStream_t>(stream));
    if (!ws) return MJ_ERR_WORKSPACE;
    CascadeLayout L = cascade_layout(ws, p, ws_bytes);
    if (ws_bytes < L.base_bytes || (p.join2_size && L.i_cap == 0)) return MJ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prof* prof = &ctx->prof;
    unsigned long long* count = reinterpret_cast<unsigned long long*>(out);

    if (a_domain)
        MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(grid_for(a_domain, 256, 4096)), dim3(256), 0, s,
                  count, (uint64_t)a_domain, 0ull);
    if (R->n == 0 || S->n == 0 || T->n == 0 || p.join2_size == 0) return MJ_OK;

    // join 2's build side: T partitioned by C, one multiplicity table per
    // bucket -- or, for dense keys, T by range of C and deg[c] directly
    const bool dense = L.deg != nullptr;
    if (dense) {
        MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, L.dflags, (uint64_t)3, 0u);
        PartLaunch PT{};
        PT.njobs = 1;
        PT.job[0] = make_job(*T, L.Tr.hist, L.Tr.counts, L.Tr.starts, 0, 0, L.c_bits, 0, 0, 0);
        PT.job[0].range_on = 1; PT.job[0].range_shift = L.c_shift;
        PT.job[0].out_single = L.tkeys; PT.job[0].single_col = 0;
        if ((st = launch_partition(prof, "tab", PT, s))) return st;
        RangeAccArgs<uint32_t, uint16_t, uint32_t, uint16_t> Ad{};
        Ad.pairs = nullptr; Ad.keys = L.tkeys; Ad.starts = L.Tr.starts; Ad.shift = L.c_shift;
        Ad.domain = p.c_domain; Ad.table = nullptr; Ad.table_n = 0; Ad.out = L.deg; Ad.err = L.dflags;
        Ad.out_narrow = L.deg16; Ad.wide = L.dflags + 2; Ad.table_narrow = nullptr; Ad.use_wide = nullptr;
        MJ_LAUNCHM(prof, "k_range_deg", k_range_deg, dim3(1u << L.c_bits), dim3(RANGE_THREADS),
                  size_t(4) << L.c_shift, s, Ad);
    } else {
        st = launch_tables(prof, L.T, *T, 0, p.log2_nc, seed_c(p), seed_slot(p), s);
        if (st) return st;
    }
    // join 1: R and S partitioned by B.  S is the build side (its C values
    // grouped by B) and R the probe side, so the pairs of I come R tuple by R
    // tuple and the second join can sum a run of one A value before its
    // atomic.  The partitions store S as (c, b) and R as (b, a), the layout
    // the grouping kernel reads (value, key) and (key, value) in.
    const uint32_t nb = 1u << p.log2_nb;
    PartLaunch P{};
    P.njobs = 2;
    P.job[0] = make_job(*S, L.S.hist, L.S.counts, L.S.starts, 0, seed_b(p), p.log2_nb, 0, 0, 0);
    P.job[0].out_pair = L.S.pairs;
    P.job[0].swap_out = 1;
    P.job[1] = make_job(*R, L.R.hist, L.R.counts, L.R.starts, 1, seed_b(p), p.log2_nb, 0, 0, 0);
    P.job[1].out_pair = L.R.pairs;
    P.job[1].swap_out = 1;
    st = launch_partition(prof, "rs", P, s);
    if (st) return st;
    CasIndexArgs X;
    X.R = L.S.pairs; X.rstarts = L.S.starts; X.S = L.R.pairs; X.sstarts = L.R.starts;
    X.Rgrp = L.Rgrp; X.ecnt = L.ecnt; X.elist = L.elist; X.seed = seed_w(p);
    MJ_LAUNCHM(prof, "k_cas_index", k_cas_index, dim3(nb), dim3(CAS_THREADS), 0, s, X);
    if ((st = launch_scan_u32(prof, L.ecnt, R->n, L.partial, L.eoff, s))) return st;
    // the chunks below cover the plan's |I|: an intermediate of another size
    // (same relations, other contents) makes every count all ones
    uint32_t* verr = dense ? L.dflags : L.T.err;
    MJ_LAUNCHM(prof, "k_check_size", k_check_size, dim3(1), dim3(64), 0, s, L.eoff + R->n,
              (unsigned long long)p.join2_size, verr);
    // the intermediate, chunk by chunk: materialise, then join with T
    const uint64_t total = p.join2_size;
    for (uint64_t lo = 0; lo < total; lo += L.i_cap) {
        const uint64_t hi = std::min<uint64_t>(total, lo + L.i_cap);
        CasExpandArgs E;
        E.eoff = L.eoff; E.elist = L.elist; E.Rgrp = L.Rgrp; E.S = L.R.pairs; E.ns = R->n;
        E.lo = lo; E.hi = hi; E.I = L.I; E.swap = 1;          // (a, c)
        MJ_LAUNCHM(prof, "k_cas_expand", k_cas_expand, dim3((uint32_t)((hi - lo + EXP_TILE - 1) / EXP_TILE)),
                  dim3(EXP_THREADS), 0, s, E);
        CasProbeArgs Q;
        Q.I = L.I; Q.n = hi - lo; Q.ddir = dense ? nullptr : L.T.dir; Q.dpool = dense ? nullptr : L.T.pool;
        Q.c_seed = seed_c(p); Q.c_bits = p.log2_nc; Q.slot_seed = seed_slot(p);
        Q.count = count; Q.a_domain = a_domain; Q.err = dense ? L.dflags : L.T.err;
        Q.deg = L.deg; Q.deg16 = L.deg16; Q.c_domain = p.c_domain; Q.use_wide = dense ? L.dflags + 2 : nullptr;
        MJ_LAUNCHM(prof, "k_cas_probe", k_cas_probe, dim3(grid_for(hi - lo, 1024, 8192)), dim3(256), 0, s, Q);
    }
    // a key beyond its certified bound, an A value out of range, a table
    // overflow or an intermediate of another size: every count all ones
    MJ_LAUNCHM(prof, "k_poison_u64", k_poison_u64, dim3(grid_for(a_domain, 256, 1024)), dim3(256), 0, s,
              count, (uint64_t)a_domain, verr);
    return MJ_OK;
}

// ------------------------------------------------------------ learned planner
static float* mlp_master(void* p) { return static_cast<float*>(p); }
static uint16_t* mlp_wbf16(void* p) { return reinterpret_cast<uint16_t*>(static_cast<float*>(p) + 4 * MLP_P); }

uint64_t mj_mlp_param_bytes(void) { return uint64_t(4) * MLP_P * 4 + uint64_t(MLP_WB) * 2; }

uint64_t mj_mlp_workspace(uint32_t B) {
    return (uint64_t(B) * MLP_ACT + 2 * uint64_t(B) * MLP_OUT) * 4 + 512;
}

uint64_t mj_linear3_distinct_workspace(uint64_t n_r, uint64_t n_s, uint64_t n_t, uint32_t a_domain) {
    return fm_layout(nullptr, n_r, n_s, n_t, a_domain).bytes;
}

int mj_linear3_distinct(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                        uint32_t a_domain, uint32_t seed, uint32_t* sketch, double* est,
                        void* ws, uint64_t ws_bytes, void* stream) {
    if (!ctx || (!sketch && a_domain)) return MJ_ERR_INVALID_ARG;
    int st;
    if ((st = check_rel(R)) || (st = check_rel(S)) || (st = check_rel(T))) return st;
    FmLayout L = fm_layout(nullptr, R->n, S->n, T->n, a_domain);
    if (!ws || ws_bytes < L.bytes) return MJ_ERR_WORKSPACE;
    L = fm_layout(ws, R->n, S->n, T->n, a_domain);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prof* prof = &ctx->prof;
    if (a_domain == 0) return MJ_OK;
    const uint64_t words = uint64_t(a_domain) * FM_WORDS;
    if (R->n == 0 || S->n == 0 || T->n == 0) {
        MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(grid_for(words, 256, 4096)), dim3(256), 0, s,
                  sketch, words, 0u);
        if (est)
            MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(grid_for(a_domain, 256, 4096)), dim3(256), 0, s,
                      reinterpret_cast<unsigned long long*>(est), (uint64_t)a_domain, 0ull);   // 0.0
        return MJ_OK;
    }
    TriLayout TL{};                    // launch_runs only uses flags / ridx / partial
    TL.flags = L.flags; TL.ridx = L.ridx; TL.partial = L.partial;
    // T grouped by C: (mix(c), mix(d)) sorted; per run the OR of bit(mix(d))
    if ((st = tri_keys(prof, *T, 0, L.Tk, seed, s))) return st;
    // (only the grouping by the high word matters to an OR of sketches)
    if ((st = launch_radix_sort(prof, L.Tk, L.tmp, T->n, L.rs_hist, L.rs_counts, L.rs_starts, s, 4))) return st;
    if ((st = launch_runs(prof, TL, L.Tk, T->n, L.T, nullptr, s))) return st;
    FmTArgs Ft;
    Ft.T = run_index(L.T); Ft.Tk = L.Tk; Ft.tsk = L.tsk;
    MJ_LAUNCH(prof, "k_fm_tsketch", k_fm_tsketch, dim3(grid_for(T->n, FM_THREADS, 16384)), dim3(FM_THREADS),
              0, s, Ft);
    MJ_LAUNCH(prof, "k_fm_tsketch_long", k_fm_tsketch_long, dim3(grid_for(T->n, FM_THREADS, 4096)),
              dim3(FM_THREADS), 0, s, Ft);
    // S grouped by B: per run the OR of T's sketches of its C values
    if ((st = tri_keys(prof, *S, 0, L.Sk, seed, s))) return st;
    if ((st = launch_radix_sort(prof, L.Sk, L.tmp, S->n, L.rs_hist, L.rs_counts, L.rs_starts, s, 4))) return st;
    if ((st = launch_runs(prof, TL, L.Sk, S->n, L.S, nullptr, s))) return st;
    FmWArgs Fw;
    Fw.S = run_index(L.S); Fw.Sk = L.Sk; Fw.T = run_index(L.T); Fw.tsk = L.tsk; Fw.wsk = L.wsk;
    MJ_LAUNCH(prof, "k_fm_wsketch", k_fm_wsketch, dim3(grid_for(S->n, FM_THREADS, 16384)), dim3(FM_THREADS),
              0, s, Fw);
    MJ_LAUNCH(prof, "k_fm_wsketch_long", k_fm_wsketch_long, dim3(grid_for(S->n, FM_THREADS, 4096)),
              dim3(FM_THREADS), 0, s, Fw);
    // R by range of A (or as one bucket in the global mode): per a the OR of
    // the sketches of its B values
    PartLaunch P{};
    P.njobs = 1;
    P.job[0] = make_job(*R, L.Ra.hist, L.Ra.counts, L.Ra.starts, 0, 0, L.a_bits, 0, 0, 0);
    P.job[0].range_on = 1;
    P.job[0].range_shift = L.a_shift;
    P.job[0].out_pair = L.Ra.pairs;
    if ((st = launch_partition(prof, "r", P, s))) return st;
    FmAArgs Fa;
    Fa.R = L.Ra.pairs; Fa.rstarts = L.Ra.starts; Fa.n = R->n; Fa.a_shift = L.a_shift; Fa.a_domain = a_domain;
    Fa.seed = seed; Fa.S = run_index(L.S); Fa.wsk = L.wsk; Fa.sketch = sketch; Fa.est = est;
    Fa.err = L.err;
    if (L.by_range) {
        MJ_LAUNCH(prof, "k_fm_asketch", k_fm_asketch, dim3(1u << L.a_bits), dim3(FM_THREADS), 0, s, Fa);
    } else {
        MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(grid_for(words, 256, 4096)), dim3(256), 0, s,
                  sketch, words, 0u);
        MJ_LAUNCH(prof, "k_fm_asketch_global", k_fm_asketch_global, dim3(grid_for(R->n, 256, 16384)), dim3(256),
                  0, s, Fa);
        MJ_LAUNCH(prof, "k_fm_estimate", k_fm_estimate, dim3(grid_for(a_domain, 256, 4096)), dim3(256), 0, s, Fa);
    }
    return MJ_OK;
}

uint64_t mj_linear3_materialize_workspace(uint64_t n_r, uint64_t n_s, uint64_t n_t) {
    return emit_layout(nullptr, n_r, n_s, n_t).bytes;
}

int mj_linear3_materialize(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                           uint64_t first, uint64_t cap, uint32_t* out, uint64_t* total,
                           void* ws, uint64_t ws_bytes, void* stream) {
    if (!ctx || !total || (cap && !out)) return MJ_ERR_INVALID_ARG;
    int st;
    if ((st = check_rel(R)) || (st = check_rel(S)) || (st = check_rel(T))) return st;
    EmitLayout L = emit_layout(nullptr, R->n, S->n, T->n);
    if (!ws || ws_bytes < L.bytes) return MJ_ERR_WORKSPACE;
    L = emit_layout(ws, R->n, S->n, T->n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prof* prof = &ctx->prof;
    unsigned long long* tot = reinterpret_cast<unsigned long long*>(total);
    if (R->n == 0 || S->n == 0 || T->n == 0) {
        MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, tot, (uint64_t)1, 0ull);
        return MJ_OK;
    }
    // the seed only groups equal keys; the output order does not depend on it
    const uint32_t seed = 0x2545F491u;
    TriLayout TL{};                    // launch_runs only uses flags / ridx / partial
    TL.flags = L.flags; TL.ridx = L.ridx; TL.partial = L.partial;
    // T grouped by C with its raw D values, S by B with its raw C values; the
    // sort is stable, so every run keeps its relation's order
    if ((st = tri_keys(prof, *T, 0, L.Tk, seed, s, true))) return st;
    if ((st = launch_radix_sort(prof, L.Tk, L.tmp, T->n, L.rs_hist, L.rs_counts, L.rs_starts, s, 4))) return st;
    if ((st = launch_runs(prof, TL, L.Tk, T->n, L.T, L.td, s))) return st;
    if ((st = tri_keys(prof, *S, 0, L.Sk, seed, s, true))) return st;
    if ((st = launch_radix_sort(prof, L.Sk, L.tmp, S->n, L.rs_hist, L.rs_counts, L.rs_starts, s, 4))) return st;
    if ((st = launch_runs(prof, TL, L.Sk, S->n, L.S, L.sc, s))) return st;
    EmitSArgs Es;
    Es.sc = L.sc; Es.ns = S->n; Es.T = run_index(L.T); Es.seed = seed; Es.tdeg = L.tdeg; Es.tst = L.tst;
    MJ_LAUNCH(prof, "k_emit_sdeg", k_emit_sdeg, dim3(grid_for((S->n + 3) / 4, 256, 16384)), dim3(256), 0, s, Es);
    if ((st = launch_scan_u32(prof, L.tdeg, S->n, L.partial, L.P_S, s))) return st;
    EmitRArgs Er;
    Er.r1 = R->col1; Er.rstride = R->stride; Er.nr = R->n; Er.S = run_index(L.S); Er.seed = seed;
    Er.P_S = L.P_S; Er.sst = L.sst; Er.pdeg = L.pdeg; Er.wout = L.wout;
    MJ_LAUNCH(prof, "k_emit_rdeg", k_emit_rdeg, dim3(grid_for((R->n + 3) / 4, 256, 16384)), dim3(256), 0, s, Er);
    if ((st = launch_scan_u32(prof, L.pdeg, R->n, L.partial, L.O_I, s))) return st;
    if ((st = launch_scan_u64(prof, L.wout, R->n, L.partial, L.O_R, s))) return st;
    MJ_LAUNCHM(prof, "k_copy_u64", k_copy_u64, dim3(1), dim3(64), 0, s, tot, L.O_R + R->n, (uint64_t)1);
    // the window, in chunks of EMIT_CHUNK_TILES tiles
    const uint64_t chunk_max = uint64_t(EMIT_CHUNK_TILES) * EMIT_TILE;
    for (uint64_t c0 = 0; c0 < cap; c0 += chunk_max) {
        const uint64_t n = std::min<uint64_t>(cap - c0, chunk_max);
        const uint32_t ntiles = (uint32_t)((n + EMIT_TILE - 1) / EMIT_TILE);
        EmitArgs E;
        E.r0 = R->col0; E.r1 = R->col1; E.rstride = R->stride; E.nr = R->n;
        E.O_R = L.O_R; E.O_I = L.O_I; E.sst = L.sst; E.P_S = L.P_S; E.sc = L.sc; E.tst = L.tst; E.td = L.td;
        E.first = first + c0; E.cap = n;
        E.out = reinterpret_cast<uint4*>(out) + c0;
        E.tiles = L.tiles;
        MJ_LAUNCH(prof, "k_emit_tiles", k_emit_tiles, dim3((ntiles + 255) / 256), dim3(256), 0, s, E, ntiles);
        MJ_LAUNCH(prof, "k_emit", k_emit, dim3(ntiles), dim3(EMIT_THREADS), 0, s, E);
    }
    return MJ_OK;
}

int mj_mlp_sync(mj_ctx* ctx, void* params, void* stream) {
    if (!ctx || !params) return MJ_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    MJ_LAUNCH(&ctx->prof, "k_mlp_sync", k_mlp_sync, dim3((MLP_P + 255) / 256), dim3(256), 0, s,
              mlp_master(params), mlp_wbf16(params));
    return MJ_OK;
}

int mj_mlp_forward(mj_ctx* ctx, const void* params, const float* X, uint32_t B, float* Y,
                   void* stream) {
    if (!ctx || !params || (B && (!X || !Y))) return MJ_ERR_INVALID_ARG;
    if (B == 0) return MJ_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* pp = const_cast<void*>(params);
    MlpFwdArgs F{mlp_master(pp), mlp_wbf16(pp), X, Y, nullptr};
    MJ_LAUNCH(&ctx->prof, "k_mlp_fwd", k_mlp_fwd, dim3(B), dim3(MLP_H), 0, s, F);
    return MJ_OK;
}

int mj_mlp_grads(mj_ctx* ctx, void* params, const float* X, uint32_t B, const float* targets,
                 const int32_t* plan_label, const int32_t* share_label, float* loss,
                 void* ws, uint64_t ws_bytes, void* stream) {
    if (!ctx || !params || !loss || (B && (!X || !targets || !plan_label || !share_label)))
        return MJ_ERR_INVALID_ARG;
    if (B == 0) return MJ_OK;
    if (!ws || ws_bytes < mj_mlp_workspace(B)) return MJ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prof* prof = &ctx->prof;
    Bump W(ws);
    float* act = W.take<float>(uint64_t(B) * MLP_ACT);
    float* Y = W.take<float>(uint64_t(B) * MLP_OUT);
    float* dY = W.take<float>(uint64_t(B) * MLP_OUT);
    MlpFwdArgs F{mlp_master(params), mlp_wbf16(params), X, Y, act};
    MJ_LAUNCH(prof, "k_mlp_fwd", k_mlp_fwd, dim3(B), dim3(MLP_H), 0, s, F);
    MlpLossArgs Lo{Y, dY, targets, plan_label, share_label, B, loss};
    MJ_LAUNCH(prof, "k_mlp_loss", k_mlp_loss, dim3((B + 255) / 256), dim3(256), 0, s, Lo);
    MlpBwdArgs Bw{mlp_wbf16(params), X, act, dY, B, mlp_master(params) + MLP_P};
    MJ_LAUNCH(prof, "k_mlp_bwd", k_mlp_bwd, dim3((B + MLP_SPB - 1) / MLP_SPB), dim3(MLP_H), 0, s, Bw);
    return MJ_OK;
}

int mj_mlp_adamw(mj_ctx* ctx, void* params, float lr, float wd, uint32_t step, void* stream) {
    if (!ctx || !params || step == 0) return MJ_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    MlpAdamArgs A;
    A.buf = mlp_master(params); A.wbf16 = mlp_wbf16(params);
    A.lr = lr; A.wd = wd; A.beta1 = 0.9f; A.beta2 = 0.999f; A.eps = 1e-8f;
    A.bc1 = (float)(1.0 - std::pow(0.9, (double)step));
    A.bc2 = (float)(1.0 - std::pow(0.999, (double)step));
    MJ_LAUNCH(&ctx->prof, "k_mlp_adamw", k_mlp_adamw, dim3((MLP_P + 255) / 256), dim3(256), 0, s, A);
    return MJ_OK;
}

uint64_t mj_sketch_workspace(uint64_t n_r, uint64_t n_s, uint64_t n_t) {
    const uint64_t n = std::max<uint64_t>({n_r, n_s, n_t, 1});
    Bump B(nullptr);
    TableLayout L;
    take_table(B, L, n, join2_bits(n));
    B.take<uint32_t>(96);
    return B.off + 256;
}

int mj_sketch(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
              float* features, void* ws, uint64_t ws_bytes, void* stream) {
    if (!ctx || !features || (kind != MJ_LINEAR && kind != MJ_TRIANGLE)) return MJ_ERR_INVALID_ARG;
    int st;
    if ((st = check_rel(R)) || (st = check_rel(S)) || (st = check_rel(T))) return st;
    if (!ws || ws_bytes < mj_sketch_workspace(R->n, S->n, T->n)) return MJ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prof* prof = &ctx->prof;
    const uint64_t n = std::max<uint64_t>({R->n, S->n, T->n, 1});
    const uint32_t bits = join2_bits(n);
    Bump B(ws);
    TableLayout L;
    take_table(B, L, n, bits);
    uint32_t* hist = B.take<uint32_t>(96);
    MJ_LAUNCHM(prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(96), 0, s, hist, (uint64_t)96, 0u);
    const mj_rel* rels[3] = {R, S, T};
    const int cols[3] = {1, 0, 0};
    for (int h = 0; h < 3; ++h) {
        if (rels[h]->n == 0) continue;
        if ((st = launch_tables(prof, L, *rels[h], cols[h], bits, 0x6A09E667u + h, 0xBB67AE85u, s))) return st;
        MJ_LAUNCH(prof, "k_deg_hist", k_deg_hist, dim3(1u << bits), dim3(256), 0, s,
                  L.dir, L.pool, 1u << bits, hist + 32 * h);
    }
    MJ_LAUNCH(prof, "k_sketch_features", k_sketch_features, dim3(1), dim3(128), 0, s,
              hist, R->n, S->n, T->n, kind, features);
    return MJ_OK;
}

int mj_ctx_set_planner(mj_ctx* ctx, const void* params) {
    if (!ctx) return MJ_ERR_INVALID_ARG;
    ctx->planner = params;
    return MJ_OK;
}

// ------------------------------------------------------------------ batch
// A batch records every join's work (its launches, in order: a chain) and
// then issues the chains together.  Each step of the issue order is one
// kernel's launches from several joins merged into one grid (their argument
// structs and block counts in a table on the device), or one record that
// has no merged form, issued alone; the chains' order is kept.  A 3-way
// plan's cells are left out of its chain and run for all joins in one
// launch at the end.

static size_t batch_item_bytes(const mj_batch_item& it) {
    if (it.plan.algo != MJ_ALGO_3WAY) return it.plan.workspace_bytes;
    if (it.kind == MJ_LINEAR) return linear_layout(nullptr, it.plan).bytes;
    return tri_layout(nullptr, it.plan).bytes;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static int run_plan(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                    uint32_t a_domain, uint64_t* out, const mj_plan_t& p, void* ws,
                    uint64_t ws_bytes, void* stream);

struct BatchRecord {
    std::vector<LaunchChain> chains;      // one per join
    std::vector<LinearCellArgs> lin;      // the 3-way plans' cells
    std::vector<uint32_t> cell_base{0};
    std::vector<TriJoinArgs> tri;
    size_t join_bytes = 0;                // the joins' workspaces
};

// Record every join's work; `base` is where the joins' workspaces start
// (nothing is dereferenced on the host, so a stand-in serves for sizing).
static int record_batch(mj_ctx* ctx, const mj_batch_item* items, int n, char* base, hipStream_t s,
                        BatchRecord& B) {
    Prof* prof = &ctx->prof;
    B.chains.assign((size_t)n, LaunchChain());
    size_t off = 0;
    int st = MJ_OK;
    for (int i = 0; i < n && st == MJ_OK; ++i) {
        const mj_batch_item& it = items[i];
        const mj_plan_t& p = it.plan;
        void* wsi = base + off;
        const size_t bytes = batch_item_bytes(it);
        off += align256(bytes);
        prof->rec = &B.chains[(size_t)i];
        if (p.algo != MJ_ALGO_3WAY) {        // cascades, star and oriented plans run their own path
            st = run_plan(ctx, it.kind, &it.R, &it.S, &it.T, it.a_domain, it.out, p, wsi, bytes, s);
        } else if (it.kind == MJ_LINEAR) {
            st = [&]() -> int {
                LinearLayout L = linear_layout(wsi, p);
                unsigned long long* count = reinterpret_cast<unsigned long long*>(it.out);
                if (it.a_domain)
                    MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(grid_for(it.a_domain, 256, 4096)), dim3(256), 0, s,
                               count, (uint64_t)it.a_domain, 0ull);
                if (it.R.n == 0 || it.S.n == 0 || it.T.n == 0) return MJ_OK;
                int e;
                if ((e = launch_tables(prof, L.T, it.T, 0, p.log2_nc, seed_c(p), seed_slot(p), s))) return e;
                PartLaunch P{};
                P.njobs = 2;
                P.job[0] = make_job(it.R, L.R.hist, L.R.counts, L.R.starts, 1, seed_b(p), p.log2_nb, 0, 0, 0);
                P.job[0].out_pair = L.R.pairs;
                P.job[1] = make_job(it.S, L.S.hist, L.S.counts, L.S.starts, 0, seed_b(p), p.log2_nb, 0, 0, 0);
                P.job[1].out_pair = L.S.pairs;
                if ((e = launch_partition(prof, "rs", P, s))) return e;
                LinearCellArgs C;
                C.R = L.R.pairs; C.rstarts = L.R.starts; C.S = L.S.pairs; C.sstarts = L.S.starts;
                C.ddir = L.T.dir; C.dpool = L.T.pool;
                C.c_seed = seed_c(p); C.c_bits = p.log2_nc; C.slot_seed = seed_slot(p); C.w_seed = seed_w(p);
                C.count = count; C.a_domain = it.a_domain; C.err = L.T.err;
                B.lin.push_back(C);
                B.cell_base.push_back(B.cell_base.back() + (1u << p.log2_nb));
                return MJ_OK;
            }();
        } else {
            st = [&]() -> int {
                TriLayout L = tri_layout(wsi, p);
                unsigned long long* out = reinterpret_cast<unsigned long long*>(it.out);
                MJ_LAUNCHM(prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, out, (uint64_t)1, 0ull);
                if (it.R.n == 0 || it.S.n == 0 || it.T.n == 0) return MJ_OK;
                int e;
                if ((e = tri_prepare(prof, ctx->num_cu, it.R, it.S, it.T, p, L, out, s))) return e;
                B.tri.push_back(tri_join_args(L, p, out, 0));
                B.tri.push_back(tri_join_args(L, p, out, 1));
                return MJ_OK;
            }();
        }
        prof->rec = nullptr;
    }
    prof->rec = nullptr;
    B.join_bytes = off;
    return st;
}

struct BatchStep {
    std::vector<std::pair<uint32_t, uint32_t>> members;   // (chain, record)
    uint32_t grid = 0, smem = 0;
    size_t table = 0;                                     // its table in the tables' area (merged steps)
};

// The issue order.  Records with no merged form at the chains' heads go
// first (they cannot wait for company); then the merged kernel at the heads
// of the most remaining work (the chains' remaining lengths summed) runs for
// every chain it heads, so that long chains move first and chains of the
// same shape stay in step.
static size_t schedule_batch(const std::vector<LaunchChain>& ch, std::vector<BatchStep>& steps) {
    steps.clear();
    const uint32_t n = (uint32_t)ch.size();
    std::vector<size_t> head(n, 0);
    size_t left = 0, tables = 0;
    for (const LaunchChain& c : ch) left += c.recs.size();
    std::map<std::pair<const void*, uint32_t>, std::pair<size_t, std::vector<uint32_t>>> heads;
    while (left) {
        heads.clear();
        for (uint32_t i = 0; i < n; ++i) {
            // records with no merged form, and merged launches with no blocks, leave at once
            while (head[i] < ch[i].recs.size() &&
                   (!ch[i].recs[head[i]].multi || ch[i].recs[head[i]].grid == 0)) {
                const LaunchRec& r = ch[i].recs[head[i]];
                if (!r.multi) {
                    BatchStep a;
                    a.members.push_back({i, (uint32_t)head[i]});
                    steps.push_back(std::move(a));
                }
                ++head[i];
                --left;
            }
            if (head[i] == ch[i].recs.size()) continue;
            const LaunchRec& r = ch[i].recs[head[i]];
            auto& h = heads[{r.multi, r.block}];
            h.first += ch[i].recs.size() - head[i];
            h.second.push_back(i);
        }
        if (heads.empty()) break;
        auto best = heads.begin();
        for (auto g = heads.begin(); g != heads.end(); ++g)
            if (g->second.first > best->second.first) best = g;
        BatchStep m;
        for (uint32_t i : best->second.second) {
            const LaunchRec& r = ch[i].recs[head[i]];
            m.members.push_back({i, (uint32_t)head[i]});
            m.grid += r.grid;
            m.smem = std::max(m.smem, r.smem);
            ++head[i];
            --left;
        }
        if (m.members.size() > 1) {
            const size_t k = m.members.size();
            const LaunchRec& r0 = ch[m.members[0].first].recs[m.members[0].second];
            m.table = tables;
            tables += align256(k * r0.asz + (k + 1) * sizeof(uint32_t));
        }
        steps.push_back(std::move(m));
    }
    return tables;
}

// Bytes of the cell stage's tables (3-way plans) after the merged steps' ones.
static size_t cell_table_bytes(size_t nl, size_t nt) {
    return align256(nl * sizeof(LinearCellArgs)) + align256((nl + 1) * 4) + align256(nt * sizeof(TriJoinArgs));
}

uint64_t mj_batch_workspace(const mj_batch_item* items, int n) {
    if (!items || n < 0) return 0;
    // the joins' work recorded with a stand-in context and workspace, for
    // the sizes of the merged steps' tables
    mj_ctx sizing;
    BatchRecord B;
    char* stand_in = reinterpret_cast<char*>(uintptr_t(1) << 44);
    (void)record_batch(&sizing, items, n, stand_in, nullptr, B);
    std::vector<BatchStep> steps;
    const size_t tables = schedule_batch(B.chains, steps);
    const size_t nn = (size_t)n;
    return B.join_bytes + align256(tables) + cell_table_bytes(nn, 2 * nn) + 2 * align256((2 * nn + 1) * 8) +
           align256(16) + 256;
}

int mj_batch_count(mj_ctx* ctx, const mj_batch_item* items, int n, void* ws, uint64_t ws_bytes,
                   void* stream) {
    if (!ctx || (!items && n) || n < 0) return MJ_ERR_INVALID_ARG;
    if (n == 0) return MJ_OK;
    // validation first: nothing is launched unless every item is valid
    for (int i = 0; i < n; ++i) {
        const mj_batch_item& it = items[i];
        int st;
        if ((st = check_rel(&it.R)) || (st = check_rel(&it.S)) || (st = check_rel(&it.T))) return st;
        if (!it.out) return MJ_ERR_INVALID_ARG;
        const mj_plan_t& p = it.plan;
        if (p.kind != it.kind || p.n_r != it.R.n || p.n_s != it.S.n || p.n_t != it.T.n ||
            (it.kind == MJ_LINEAR && p.a_domain != it.a_domain) ||
            p.input_fingerprint != fingerprint(it.R, it.S, it.T))
            return MJ_ERR_PLAN_MISMATCH;
        if (p.log2_nb > PART_MAX_BITS || p.log2_nc > PART_MAX_BITS || p.log2_share > 16)
            return MJ_ERR_INVALID_ARG;
    }
    if (!ws || ws_bytes < mj_batch_workspace(items, n)) return MJ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Prof* prof = &ctx->prof;
    char* base = static_cast<char*>(ws);
    BatchRecord B;
    int st = record_batch(ctx, items, n, base, s, B);
    if (st) return st;
    std::vector<BatchStep> steps;
    const size_t tables = schedule_batch(B.chains, steps);
    // argument tables, staged through pinned memory: the merged steps', then
    // the cell stage's.  An eager call reuses the context's buffer once the
    // previous copy out of it has run; a captured copy is read again at every
    // replay, so its buffer is its own and lives as long as the context.
    const size_t nl = B.lin.size(), nt = B.tri.size();
    const size_t a_lin = align256(nl * sizeof(LinearCellArgs)), a_cb = align256((nl + 1) * 4);
    const size_t stage = align256(tables) + cell_table_bytes(nl, nt);
    const size_t want = std::max<size_t>(stage, 256);
    char* dev = base + B.join_bytes;
    if (uint64_t(B.join_bytes) + stage + 2 * align256((nt + 1) * 8) + align256(16) > ws_bytes)
        return MJ_ERR_WORKSPACE;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    MJ_HIP(hipStreamIsCapturing(s, &cap));
    const bool captured = cap != hipStreamCaptureStatusNone;
    char* host = nullptr;
    if (captured) {
        MJ_HIP(hipHostMalloc(reinterpret_cast<void**>(&host), want));
        ctx->pinned.push_back(host);
    } else {
        if (!ctx->stage_read) MJ_HIP(hipEventCreateWithFlags(&ctx->stage_read, hipEventDisableTiming));
        else MJ_HIP(hipEventSynchronize(ctx->stage_read));
        if (ctx->stage_bytes < want) {
            if (ctx->stage) MJ_HIP(hipHostFree(ctx->stage));
            ctx->stage = nullptr;
            ctx->stage_bytes = 0;
            MJ_HIP(hipHostMalloc(reinterpret_cast<void**>(&ctx->stage), want));
            ctx->stage_bytes = want;
        }
        host = ctx->stage;
    }
    for (const BatchStep& m : steps) {
        if (m.members.size() < 2) continue;
        const size_t k = m.members.size();
        const uint32_t asz = B.chains[m.members[0].first].recs[m.members[0].second].asz;
        char* t = host + m.table;
        uint32_t* bases = reinterpret_cast<uint32_t*>(t + k * asz);
        uint32_t at = 0;
        for (size_t q = 0; q < k; ++q) {
            const LaunchChain& c = B.chains[m.members[q].first];
            const LaunchRec& r = c.recs[m.members[q].second];
            std::memcpy(t + q * asz, c.args.data() + r.aoff, asz);
            bases[q] = at;
            at += r.grid;
        }
        bases[k] = at;
    }
    char* cells = host + align256(tables);
    if (nl) std::memcpy(cells, B.lin.data(), nl * sizeof(LinearCellArgs));
    std::memcpy(cells + a_lin, B.cell_base.data(), (nl + 1) * 4);
    if (nt) std::memcpy(cells + a_lin + a_cb, B.tri.data(), nt * sizeof(TriJoinArgs));
    MJ_HIP(hipMemcpyAsync(dev, host, stage, hipMemcpyHostToDevice, s));
    if (!captured) MJ_HIP(hipEventRecord(ctx->stage_read, s));
    // the chains' work in the issue order
    for (const BatchStep& m : steps) {
        const LaunchRec& r0 = B.chains[m.members[0].first].recs[m.members[0].second];
        hipEvent_t ea = nullptr, eb = nullptr;
        if (prof->on) { ea = prof->ev(); eb = prof->ev(); (void)hipEventRecord(ea, s); }
        if (m.members.size() == 1) {
            if ((st = r0.alone(s))) {
                std::fprintf(stderr, "libmj: batch step %s failed\n", r0.name.c_str());
                return st;
            }
        } else {
            MultiGrid M;
            M.args = dev + m.table;
            M.base = reinterpret_cast<const uint32_t*>(dev + m.table + m.members.size() * r0.asz);
            M.njobs = (uint32_t)m.members.size();
            void (*multi)(MultiGrid) = reinterpret_cast<void (*)(MultiGrid)>(const_cast<void*>(r0.multi));
            hipLaunchKernelGGL(multi, dim3(m.grid), dim3(r0.block), m.smem, s, M);
            const hipError_t le = hipGetLastError();
            if (le != hipSuccess) {
                std::fprintf(stderr, "libmj: merged launch of %s failed: %s\n", r0.name.c_str(), hipGetErrorString(le));
                return MJ_ERR_HIP;
            }
        }
        if (ea) { (void)hipEventRecord(eb, s); prof->pending.push_back({r0.name, ea, eb}); }
    }
    if (nl) {
        LinearBatchArgs C;
        C.joins = reinterpret_cast<const LinearCellArgs*>(cells - host + dev);
        C.cell_base = reinterpret_cast<const uint32_t*>(cells - host + dev + a_lin);
        C.njoins = (uint32_t)nl;
        MJ_LAUNCH(prof, "k_linear_cell_batch", k_linear_cell_batch, dim3(B.cell_base.back()),
                  dim3(CELL_THREADS), 0, s, C);
    }
    if (nt) {
        char* q = dev + stage;
        TriBatchArgs T;
        T.joins = reinterpret_cast<const TriJoinArgs*>(cells - host + dev + a_lin + a_cb);
        T.njoins = (uint32_t)nt;
        T.light_base = reinterpret_cast<unsigned long long*>(q);
        T.heavy_base = reinterpret_cast<unsigned long long*>(q + align256((nt + 1) * 8));
        T.next = reinterpret_cast<unsigned long long*>(q + 2 * align256((nt + 1) * 8));
        MJ_LAUNCH(prof, "k_tri_batch_prefix", k_tri_batch_prefix, dim3(1), dim3(64), 0, s, T);
        MJ_LAUNCH(prof, "k_tri_light_batch", k_tri_light_batch, dim3((uint32_t)ctx->num_cu * 8),
                  dim3(TRI_THREADS), 0, s, T);
        MJ_LAUNCH(prof, "k_tri_heavy_batch", k_tri_heavy_batch, dim3((uint32_t)ctx->num_cu * 2),
                  dim3(TRI_HEAVY_THREADS), 0, s, T);
    }
    return MJ_OK;
}

static int run_plan(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                    uint32_t a_domain, uint64_t* out, const mj_plan_t& p, void* ws,
                    uint64_t ws_bytes, void* stream) {
    if (p.algo == MJ_ALGO_CASCADE || p.algo == MJ_ALGO_STAR_CASCADE)
        return mj_cascade2_count(ctx, kind, R, S, T, a_domain, out, &p, ws, ws_bytes, stream);
    if (kind == MJ_LINEAR)
        return mj_linear3_count(ctx, R, S, T, a_domain, out, &p, ws, ws_bytes, stream);
    return mj_triangle3_count(ctx, R, S, T, out, &p, ws, ws_bytes, stream);
}

int mj_autotune(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                uint32_t a_domain, uint64_t* out, mj_plan_t* plan, void* ws,
                uint64_t ws_bytes, double* tuned_ms, void* stream) {
    if (!ctx || !plan || !out) return MJ_ERR_INVALID_ARG;
    if (plan->kind != kind) return MJ_ERR_PLAN_MISMATCH;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char key[128];
    std::snprintf(key, sizeof key, "%d:%u:%u:%u:%u", kind, ceil_log2(plan->n_r + 1),
                  ceil_log2(plan->n_s + 1), ceil_log2(plan->n_t + 1),
                  ceil_log2(plan->join2_size + 1));
    auto hit = ctx->tuned.find(key);
    if (hit != ctx->tuned.end()) {
        const mj_plan_t& c = hit->second;
        plan->algo = c.algo; plan->log2_nb = c.log2_nb; plan->log2_nc = c.log2_nc;
        plan->log2_share = c.log2_share; plan->seed = c.seed;
        // a hashed winner stays hashed; a dense winner applies only where this
        // plan's own data was found dense (the key is the size class alone)
        if (c.flags & MJ_PLAN_NO_DENSE)
            plan->flags = (plan->flags & ~uint32_t(MJ_PLAN_DENSE_KEYS)) | MJ_PLAN_NO_DENSE;
        int st = plan_workspace(*plan);
        if (st) return st;
        if (tuned_ms) *tuned_ms = c.est_ms_3way;
        return run_plan(ctx, kind, R, S, T, a_domain, out, *plan, ws, ws_bytes, stream);
    }
    std::vector<mj_plan_t> cand;
    mj_plan_t base = *plan;
    if (kind == MJ_LINEAR) {
        if (base.flags & MJ_PLAN_DENSE_KEYS) { mj_plan_t c = base; c.algo = MJ_ALGO_3WAY; cand.push_back(c); }
        for (uint32_t nb = 8; nb <= 10; ++nb)
            for (uint32_t nc = 8; nc <= 10; ++nc) {
                mj_plan_t c = base; c.algo = MJ_ALGO_3WAY; c.log2_nb = nb; c.log2_nc = nc;
                c.flags = (c.flags & ~uint32_t(MJ_PLAN_DENSE_KEYS)) | MJ_PLAN_NO_DENSE;
                cand.push_back(c);
            }
        for (uint32_t nb = 8; nb <= 10; ++nb) {
            mj_plan_t c = base; c.algo = MJ_ALGO_CASCADE; c.log2_nb = nb; c.log2_nc = 9;
            cand.push_back(c);
        }
        if (base.est_ms_star > 0.0) { mj_plan_t c = base; c.algo = MJ_ALGO_STAR; cand.push_back(c); }
        if (base.est_ms_slarge > 0.0) {
            mj_plan_t c = base;
            c.algo = MJ_ALGO_SLARGE;
            uint32_t lr = 0, lt = 0;
            if (slarge_buckets(default_model(), base.n_r, base.n_s, base.n_t, lr, lt, nullptr)) {
                c.log2_nb = lr;
                c.log2_nc = lt;
                cand.push_back(c);
            }
        }
        if (base.est_ms_star_cascade > 0.0) { mj_plan_t c = base; c.algo = MJ_ALGO_STAR_CASCADE; cand.push_back(c); }
    } else {
        for (uint32_t k = 0; k <= 4; k += 2) {
            mj_plan_t c = base; c.algo = MJ_ALGO_3WAY; c.log2_share = k; cand.push_back(c);
        }
        if (base.est_ms_cascade < 4.0 * base.est_ms_3way) {
            mj_plan_t c = base; c.algo = MJ_ALGO_CASCADE; cand.push_back(c);
        }
        if (base.flags & MJ_PLAN_SYMMETRIC_SIMPLE)
            for (uint32_t k = 0; k <= 4; k += 2) {
                mj_plan_t c = base; c.algo = MJ_ALGO_ORIENTED; c.log2_share = k; cand.push_back(c);
            }
    }
    hipEvent_t e0, e1;
    MJ_HIP(hipEventCreate(&e0));
    MJ_HIP(hipEventCreate(&e1));
    double best = INFINITY;
    mj_plan_t best_p = base;
    const int reps = kind == MJ_LINEAR ? 2 : 1;
    for (mj_plan_t c : cand) {
        int st = plan_workspace(c);
        if (st) return st;
        if (c.workspace_bytes > ws_bytes) continue;
        if (kind == MJ_LINEAR && (st = run_plan(ctx, kind, R, S, T, a_domain, out, c, ws, ws_bytes, stream)))
            return st;
        MJ_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r)
            if ((st = run_plan(ctx, kind, R, S, T, a_domain, out, c, ws, ws_bytes, stream))) return st;
        MJ_HIP(hipEventRecord(e1, s));
        MJ_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        MJ_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double t = ms / reps;
        if (t < best) { best = t; best_p = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!std::isfinite(best)) return MJ_ERR_WORKSPACE;
    *plan = best_p;
    mj_plan_t rec = best_p;
    rec.est_ms_3way = best;
    ctx->tuned[key] = rec;
    if (tuned_ms) *tuned_ms = best;
    // leave the winner's counts in `out`
    return run_plan(ctx, kind, R, S, T, a_domain, out, best_p, ws, ws_bytes, stream);
}

}  // extern "C"

// ============================================================== planning
namespace mj {

uint32_t join2_bits(uint64_t n) {
    // about 2048 tuples per table bucket, at most 4096 buckets
    uint32_t b = ceil_log2((n + 2047) / 2048);
    return std::min<uint32_t>(b, PART_MAX_BITS);
}

int plan_workspace(mj_plan_t& p) {
    if (p.kind == MJ_LINEAR) {
        // enough for whichever algorithm the plan picked, for the other one
        // when the caller runs both on the same plan, and for every bucket
        // count the autotuner tries (up to 2^10)
        size_t need = 0;
        for (int wide = 0; wide < 2; ++wide) {
            mj_plan_t q = p;
            if (wide) { q.log2_nb = std::max<uint32_t>(q.log2_nb, 10); q.log2_nc = std::max<uint32_t>(q.log2_nc, 10); }
            const size_t lin = linear_layout(nullptr, q).bytes;
            const CascadeLayout C = cascade_layout(nullptr, q, 0);
            need = std::max({need, lin, C.base_bytes + C.i_cap * sizeof(uint2) + 256});
        }
        if (p.flags & MJ_PLAN_DENSE_KEYS) need = std::max(need, dense_layout(nullptr, p).bytes);
        // the star plans (planned or tuned only for small R)
        if (star_plan_fits(p) || p.algo == MJ_ALGO_STAR || p.algo == MJ_ALGO_STAR_CASCADE) {
            need = std::max(need, star_layout(nullptr, p, false).bytes);
            if (p.join2_size <= STAR_PLAN_MAX_I) need = std::max(need, star_layout(nullptr, p, true).bytes);
        }
        p.workspace_bytes = need;
    } else {
        const CasTriLayout C = cas_tri_layout(nullptr, p, 0);
        p.workspace_bytes = std::max<size_t>(tri_layout(nullptr, p).bytes,
                                             C.base_bytes + C.i_cap * sizeof(uint2) + 256);
        if (p.flags & MJ_PLAN_SYMMETRIC_SIMPLE)
            p.workspace_bytes = std::max<size_t>(p.workspace_bytes, oriented_bytes(p));
    }
    return MJ_OK;
}

}  // namespace mj
