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

#include <map>
#include <string>
#include <vector>

using namespace mj;

// Optional per-kernel timing with HIP events recorded on the launch stream.
struct Prof {
    bool on = false;
    struct Rec { const char* name; hipEvent_t a, b; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> free_ev;
    std::map<std::string, std::pair<double, long>> total;   // ms, launches
    hipEvent_t ev() {
        if (!free_ev.empty()) { hipEvent_t e = free_ev.back(); free_ev.pop_back(); return e; }
        hipEvent_t e; hipEventCreate(&e); return e;
    }
    void collect() {
        for (auto& r : pending) {
            hipEventSynchronize(r.b);
            float ms = 0.f;
            hipEventElapsedTime(&ms, r.a, r.b);
            auto& t = total[r.name];
            t.first += ms; t.second += 1;
            free_ev.push_back(r.a); free_ev.push_back(r.b);
        }
        pending.clear();
    }
    ~Prof() {
        collect();
        for (auto e : free_ev) hipEventDestroy(e);
    }
};

// Launch a kernel, bracketed by timing events when profiling is on.
#define MJ_LAUNCH(prof, name, kern, grid, block, smem, st, ...)                       \
    do {                                                                           \
        hipEvent_t ea_ = nullptr, eb_ = nullptr;                                   \
        if ((prof) && (prof)->on) { ea_ = (prof)->ev(); eb_ = (prof)->ev();        \
                                    hipEventRecord(ea_, st); }                     \
        hipLaunchKernelGGL(kern, grid, block, smem, st, __VA_ARGS__);              \
        hipError_t le_ = hipGetLastError();                                        \
        if (le_ != hipSuccess) {                                                   \
            std::fprintf(stderr, "libmj: launch of %s failed: %s\n", name,        \
                         hipGetErrorString(le_));                                  \
            return MJ_ERR_HIP;                                                     \
        }                                                                          \
        if (ea_) { hipEventRecord(eb_, st); (prof)->pending.push_back({name, ea_, eb_}); } \
    } while (0)

// ------------------------------------------------------------------ context
struct mj_ctx {
    int device = 0;
    int num_cu = 256;
    // small statistics buffer owned by the context (planning only)
    void* stats = nullptr;
    size_t stats_bytes = 0;
    // grown on demand by mj_plan for degree statistics
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    Prof prof;
};

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

int ensure_scratch(mj_ctx* ctx, size_t bytes) {
    if (ctx->scratch_bytes >= bytes) return MJ_OK;
    if (ctx->scratch) {
        MJ_HIP(hipDeviceSynchronize());
        MJ_HIP(hipFree(ctx->scratch));
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    size_t want = std::max<size_t>(bytes, size_t(1) << 20);
    MJ_HIP(hipMalloc(&ctx->scratch, want));
    ctx->scratch_bytes = want;
    return MJ_OK;
}

}  // namespace

// ============================================================ validation
namespace mj {

int check_rel(const mj_rel* r) {
    if (!r) return MJ_ERR_INVALID_ARG;
    if (r->n >= (uint64_t(1) << 32)) return MJ_ERR_INVALID_ARG;
    if (r->n > 0 && (!r->col0 || !r->col1 || r->stride < 1)) return MJ_ERR_INVALID_ARG;
    return MJ_OK;
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

struct TableLayout {                 // bucketed multiplicity tables of one column
    uint32_t* counts;
    uint32_t* starts;
    uint32_t* cursor;
    uint32_t* keys;                  // the partitioned column
    DirEntry* dir;
    uint2* pool;
    unsigned long long* pool_cursor;
    uint32_t* err;
    uint64_t pool_slots;
};

uint64_t pool_slots_for(uint64_t n, uint32_t nbkt) {
    return 4 * n + uint64_t(DB_MIN_CAP) * nbkt + DB_MIN_CAP;
}

void take_table(Bump& B, TableLayout& L, uint64_t n, uint32_t bits) {
    const uint32_t nb = 1u << bits;
    L.counts = B.take<uint32_t>(nb);
    L.starts = B.take<uint32_t>(nb + 1);
    L.cursor = B.take<uint32_t>(nb);
    L.keys = B.take<uint32_t>(std::max<uint64_t>(n, 1));
    L.dir = B.take<DirEntry>(nb);
    L.pool_slots = pool_slots_for(n, nb);
    L.pool = B.take<uint2>(L.pool_slots);
    L.pool_cursor = B.take<unsigned long long>(1);
    L.err = B.take<uint32_t>(1);
}

struct LinearLayout {
    uint2* Rp;
    uint32_t* rcounts; uint32_t* rstarts; uint32_t* rcursor;
    uint2* Sp;
    uint32_t* scounts; uint32_t* sstarts; uint32_t* scursor;
    TableLayout T;
    size_t bytes;
};

LinearLayout linear_layout(void* ws, const mj_plan_t& p) {
    Bump B(ws);
    LinearLayout L;
    const uint32_t nb = 1u << p.log2_nb;
    L.Rp = B.take<uint2>(std::max<uint64_t>(p.n_r, 1));
    L.rcounts = B.take<uint32_t>(nb);
    L.rstarts = B.take<uint32_t>(nb + 1);
    L.rcursor = B.take<uint32_t>(nb);
    L.Sp = B.take<uint2>(std::max<uint64_t>(p.n_s, 1));
    L.scounts = B.take<uint32_t>(nb);
    L.sstarts = B.take<uint32_t>(nb + 1);
    L.scursor = B.take<uint32_t>(nb);
    take_table(B, L.T, p.n_t, p.log2_nc);
    L.bytes = B.off + 256;
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

// Partition T.c (or any single column) by bucket and build its tables.
int launch_tables(Prof* prof, const TableLayout& L, const mj_rel& rel, int col, uint32_t bits,
                  uint32_t bseed, uint32_t sseed, hipStream_t st) {
    const uint32_t nb = 1u << bits;
    MJ_LAUNCH(prof, "tab:k_fill_u32", k_fill_u32, dim3(grid_for(nb, 256)), dim3(256), 0, st, L.counts, (uint64_t)nb, 0u);
    MJ_LAUNCH(prof, "tab:k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(L.pool),
                       (uint64_t)(2 * DB_MIN_CAP), EMPTY_KEY);
    // pool[0..DB_MIN_CAP) keys EMPTY, counts EMPTY too: counts are never read for
    // an empty key.  cursor = DB_MIN_CAP; err = 0.
    MJ_LAUNCH(prof, "tab:k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, st, L.pool_cursor, (uint64_t)1,
                       (unsigned long long)DB_MIN_CAP);
    MJ_LAUNCH(prof, "tab:k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, st, L.err, (uint64_t)1, 0u);

    PartLaunch P{};
    P.njobs = 1;
    PartJob& J = P.job[0];
    J.col0 = rel.col0; J.col1 = rel.col1; J.stride = rel.stride; J.n = rel.n;
    J.key0_col = col; J.key1_col = 0; J.seed0 = bseed; J.bits0 = bits; J.seed1 = 0; J.bits1 = 0;
    J.counts = L.counts; J.starts = L.starts; J.cursor = L.cursor;
    J.out_pair = nullptr; J.out_single = L.keys; J.single_col = col;
    J.tile_begin = 0;
    J.ntiles = (uint32_t)((rel.n + PART_TILE - 1) / PART_TILE);
    if (J.ntiles) {
        MJ_LAUNCH(prof, "tab:k_part_hist", k_part_hist, dim3(J.ntiles), dim3(PART_THREADS), nb * 4, st, P);
    }
    MJ_LAUNCH(prof, "tab:k_part_scan", k_part_scan, dim3(1), dim3(PART_THREADS), nb * 4, st, P);
    if (J.ntiles) {
        MJ_LAUNCH(prof, "tab:k_part_scatter", k_part_scatter, dim3(J.ntiles), dim3(PART_THREADS),
                           part_scatter_smem(bits), st, P);
    }
    DBuildArgs D;
    D.keys = L.keys; D.starts = L.starts; D.nbkt = nb; D.slot_seed = sseed;
    D.dir = L.dir; D.pool = L.pool; D.pool_cursor = L.pool_cursor; D.pool_cap = L.pool_slots;
    D.err = L.err;
    MJ_LAUNCH(prof, "tab:k_dbuild", k_dbuild, dim3(nb), dim3(DB_THREADS), 0, st, D);
    return MJ_OK;
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
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_part_scatter),
                        hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)part_scatter_smem(PART_MAX_BITS));
    e = hipMalloc(&c->stats, 4096);
    if (e != hipSuccess) { delete c; return MJ_ERR_HIP; }
    c->stats_bytes = 4096;
    *out = c;
    return MJ_OK;
}

int mj_ctx_destroy(mj_ctx* ctx) {
    if (!ctx) return MJ_ERR_INVALID_ARG;
    hipDeviceSynchronize();
    if (ctx->stats) hipFree(ctx->stats);
    if (ctx->scratch) hipFree(ctx->scratch);
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
    MJ_LAUNCH(&ctx->prof, "k_fill_u64", k_fill_u64, dim3(1), dim3(64), 0, s, total, (uint64_t)1, 0ull);
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

int mj_plan(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
            uint32_t a_domain, int planner, mj_plan_t* plan, void* stream) {
    if (!ctx || !plan) return MJ_ERR_INVALID_ARG;
    int st;
    if ((st = check_rel(R)) || (st = check_rel(S)) || (st = check_rel(T))) return st;
    if (kind != MJ_LINEAR && kind != MJ_TRIANGLE) return MJ_ERR_INVALID_ARG;
    if (planner < MJ_PLANNER_ANALYTIC || planner > MJ_PLANNER_FIXED) return MJ_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);

    mj_plan_t p = planner == MJ_PLANNER_FIXED ? *plan : mj_plan_t{};
    p.kind = kind;
    p.n_r = R->n; p.n_s = S->n; p.n_t = T->n;
    p.a_domain = kind == MJ_LINEAR ? a_domain : 0;

    if (kind == MJ_LINEAR) {
        if (a_domain == 0 && R->n) return MJ_ERR_KEY_RANGE;
        if (R->n) {
            uint32_t* d = static_cast<uint32_t*>(ctx->stats);
            MJ_LAUNCH(&ctx->prof, "k_fill_u32", k_fill_u32, dim3(1), dim3(64), 0, s, d, (uint64_t)1, 0u);
            MJ_LAUNCH(&ctx->prof, "k_col_max", k_col_max, dim3(grid_for(R->n, 256, 2048)), dim3(256), 0, s,
                               R->col0, R->stride, R->n, d);
            uint32_t mx = 0;
            MJ_HIP(hipMemcpyAsync(&mx, d, 4, hipMemcpyDeviceToHost, s));
            MJ_HIP(hipStreamSynchronize(s));
            if (mx >= a_domain) return MJ_ERR_KEY_RANGE;
        }
    }
    // exact size of the binary intermediate (cascade workspace, cost model)
    {
        size_t need = mj_join2_size_workspace(R->n, S->n);
        if ((st = ensure_scratch(ctx, need))) return st;
        uint64_t I = 0;
        st = mj_join2_size(ctx, R, S, &I, ctx->scratch, ctx->scratch_bytes, stream);
        if (st) return st;
        p.join2_size = I;
    }
    if (planner != MJ_PLANNER_FIXED) {
        st = analytic_plan(kind, p, ctx->num_cu);
        if (st) return st;
    } else {
        if (p.log2_nb > PART_MAX_BITS || p.log2_nc > PART_MAX_BITS || p.log2_share > 6)
            return MJ_ERR_INVALID_ARG;
        if (kind == MJ_LINEAR && p.algo != MJ_ALGO_3WAY && p.algo != MJ_ALGO_CASCADE)
            return MJ_ERR_INVALID_ARG;
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
        p.a_domain != a_domain)
        return MJ_ERR_PLAN_MISMATCH;
    if (p.log2_nb > PART_MAX_BITS || p.log2_nc > PART_MAX_BITS) return MJ_ERR_INVALID_ARG;
    LinearLayout L = linear_layout(nullptr, p);
    if (ws_bytes < L.bytes || (!ws && L.bytes)) return MJ_ERR_WORKSPACE;
    L = linear_layout(ws, p);
    hipStream_t s = static_cast<hipStream_t>(stream);

    if (a_domain) {
        MJ_LAUNCH(&ctx->prof, "k_fill_u64", k_fill_u64, dim3(grid_for(a_domain, 256, 4096)), dim3(256), 0, s,
                           reinterpret_cast<unsigned long long*>(count), (uint64_t)a_domain, 0ull);
    }
    if (R->n == 0 || S->n == 0 || T->n == 0) return MJ_OK;

    const uint32_t nb = 1u << p.log2_nb;
    // T: partition by g(C) and reduce each bucket to C -> multiplicity
    st = launch_tables(&ctx->prof, L.T, *T, 0, p.log2_nc, seed_c(p), seed_slot(p), s);
    if (st) return st;
    // R and S: partition by the bucket of B (one launch for both)
    MJ_LAUNCH(&ctx->prof, "k_fill_u32", k_fill_u32, dim3(grid_for(nb, 256)), dim3(256), 0, s, L.rcounts, (uint64_t)nb, 0u);
    MJ_LAUNCH(&ctx->prof, "k_fill_u32", k_fill_u32, dim3(grid_for(nb, 256)), dim3(256), 0, s, L.scounts, (uint64_t)nb, 0u);
    PartLaunch P{};
    P.njobs = 2;
    PartJob& JR = P.job[0];
    JR.col0 = R->col0; JR.col1 = R->col1; JR.stride = R->stride; JR.n = R->n;
    JR.key0_col = 1; JR.seed0 = seed_b(p); JR.bits0 = p.log2_nb;
    JR.counts = L.rcounts; JR.starts = L.rstarts; JR.cursor = L.rcursor;
    JR.out_pair = L.Rp; JR.tile_begin = 0;
    JR.ntiles = (uint32_t)((R->n + PART_TILE - 1) / PART_TILE);
    PartJob& JS = P.job[1];
    JS.col0 = S->col0; JS.col1 = S->col1; JS.stride = S->stride; JS.n = S->n;
    JS.key0_col = 0; JS.seed0 = seed_b(p); JS.bits0 = p.log2_nb;
    JS.counts = L.scounts; JS.starts = L.sstarts; JS.cursor = L.scursor;
    JS.out_pair = L.Sp; JS.tile_begin = JR.ntiles;
    JS.ntiles = (uint32_t)((S->n + PART_TILE - 1) / PART_TILE);
    const uint32_t tiles = JR.ntiles + JS.ntiles;
    MJ_LAUNCH(&ctx->prof, "rs:k_part_hist", k_part_hist, dim3(tiles), dim3(PART_THREADS), nb * 4, s, P);
    MJ_LAUNCH(&ctx->prof, "rs:k_part_scan", k_part_scan, dim3(2), dim3(PART_THREADS), nb * 4, s, P);
    MJ_LAUNCH(&ctx->prof, "rs:k_part_scatter", k_part_scatter, dim3(tiles), dim3(PART_THREADS), part_scatter_smem(p.log2_nb), s, P);
    // cells: one workgroup per b-bucket
    LinearCellArgs C;
    C.R = L.Rp; C.rstarts = L.rstarts; C.S = L.Sp; C.sstarts = L.sstarts;
    C.ddir = L.T.dir; C.dpool = L.T.pool;
    C.c_seed = seed_c(p); C.c_bits = p.log2_nc; C.slot_seed = seed_slot(p);
    C.w_seed = seed_w(p);
    C.count = reinterpret_cast<unsigned long long*>(count);
    C.a_domain = a_domain;
    C.err = L.T.err;
    MJ_LAUNCH(&ctx->prof, "k_linear_cell", k_linear_cell, dim3(nb), dim3(CELL_THREADS), 0, s, C);
    return MJ_OK;
}

int mj_triangle3_count(mj_ctx*, const mj_rel*, const mj_rel*, const mj_rel*, uint64_t*,
                       const mj_plan_t*, void*, uint64_t, void*) {
    return MJ_ERR_UNSUPPORTED;
}

int mj_cascade2_count(mj_ctx*, int, const mj_rel*, const mj_rel*, const mj_rel*, uint32_t,
                      uint64_t*, const mj_plan_t*, void*, uint64_t, void*) {
    return MJ_ERR_UNSUPPORTED;
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
        size_t lin = linear_layout(nullptr, p).bytes;
        p.workspace_bytes = lin;
    } else {
        p.workspace_bytes = 256;
    }
    return MJ_OK;
}

int analytic_plan(int kind, mj_plan_t& p, int num_cu) {
    (void)num_cu;
    p.seed = 0x1B873593u;
    p.algo = MJ_ALGO_3WAY;
    if (kind == MJ_LINEAR) {
        // b-buckets: about 2048 S tuples per cell; c-buckets: about 4096 T
        // tuples per multiplicity table
        p.log2_nb = std::min<uint32_t>(PART_MAX_BITS, ceil_log2((p.n_s + 2047) / 2048));
        p.log2_nc = std::min<uint32_t>(PART_MAX_BITS, ceil_log2((p.n_t + 4095) / 4096));
    } else {
        p.log2_share = 3;
    }
    return MJ_OK;
}

}  // namespace mj
