// Replay of the benchmark's sequence of library calls on the host build
// (test infrastructure only).  Every buffer the caller passes -- relations,
// outputs, workspaces -- is its own heap allocation of exactly the size the
// call is given, filled with the byte HIPSIM_FILL (default 0xA5) so that
// nothing reads as zeros unless a kernel wrote it.  AddressSanitizer reports
// any access outside those buffers; the checks below report results that
// differ from the closed forms or between algorithms.
//
//   replay DATA_DIR [legs...]     legs: main cascade skew small fm emit star slarge batch (default: all)
//   environment: HIPSIM_STEPS (timed steps of the main leg, default 2)
#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "mj.h"

namespace {

struct Meta { uint64_t n = 0; uint32_t a_domain = 0; uint64_t closed = 0; };
std::map<std::string, Meta> g_meta;
std::string g_dir;
int g_fail = 0;

unsigned char fill_byte() {
    const char* e = std::getenv("HIPSIM_FILL");
    return e ? (unsigned char)std::strtoul(e, nullptr, 0) : 0xA5;
}

void* alloc(size_t bytes) {
    void* p = std::malloc(bytes ? bytes : 1);
    if (!p) { std::fprintf(stderr, "replay: out of memory (%zu bytes)\n", bytes); std::exit(3); }
    std::memset(p, fill_byte(), bytes);
    return p;
}

uint32_t* load(const std::string& name) {
    const Meta& m = g_meta.at(name);
    uint32_t* p = static_cast<uint32_t*>(alloc(m.n * 8));
    FILE* f = std::fopen((g_dir + "/" + name + ".bin").c_str(), "rb");
    if (!f || std::fread(p, 8, m.n, f) != m.n) { std::fprintf(stderr, "replay: cannot read %s\n", name.c_str()); std::exit(3); }
    std::fclose(f);
    return p;
}

mj_rel rel_of(const uint32_t* base, uint64_t n) {
    mj_rel r;
    r.col0 = base; r.col1 = base + 1; r.n = n; r.stride = 2;
    return r;
}

void check(int st, const char* what) {
    if (st != MJ_OK) {
        std::fprintf(stderr, "replay: %s returned %s\n", what, mj_status_str(st));
        std::exit(4);
    }
}

void expect(bool ok, const char* what) {
    std::printf("[replay]   %-60s %s\n", what, ok ? "ok" : "FAILED");
    std::fflush(stdout);
    if (!ok) ++g_fail;
}

uint64_t sum(const uint64_t* v, uint64_t n) {
    uint64_t s = 0;
    for (uint64_t i = 0; i < n; ++i) s += v[i];
    return s;
}

uint64_t fnv(const void* p, size_t bytes) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < bytes; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    return h;
}

// mj_plan with a planning workspace of its own size, allocated per call
int make_plan(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T, uint32_t a_domain,
         mj_plan_t* p) {
    const uint64_t need = mj_plan_workspace(kind, R->n, S->n, T->n);
    void* pws = alloc(need);
    const int st = mj_plan(ctx, kind, R, S, T, a_domain, MJ_PLANNER_ANALYTIC, p, pws, need, nullptr);
    std::free(pws);
    return st;
}

void leg(const char* name) {
    std::printf("[replay] leg %s\n", name);
    std::fflush(stdout);
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) { std::fprintf(stderr, "usage: replay DATA_DIR [legs]\n"); return 2; }
    g_dir = argv[1];
    {
        FILE* f = std::fopen((g_dir + "/meta.txt").c_str(), "r");
        if (!f) { std::fprintf(stderr, "replay: no meta.txt\n"); return 3; }
        char name[64];
        Meta m;
        while (std::fscanf(f, "%63s %" SCNu64 " %u %" SCNu64, name, &m.n, &m.a_domain, &m.closed) == 4) g_meta[name] = m;
        std::fclose(f);
    }
    std::vector<std::string> legs;
    for (int i = 2; i < argc; ++i) legs.push_back(argv[i]);
    auto want = [&](const char* l) {
        if (legs.empty()) return true;
        for (auto& x : legs) if (x == l) return true;
        return false;
    };
    const int steps = std::getenv("HIPSIM_STEPS") ? std::atoi(std::getenv("HIPSIM_STEPS")) : 2;

    mj_ctx* ctx = nullptr;
    check(mj_ctx_create(0, &ctx), "mj_ctx_create");

    // ------------------------------------------------ the timed workload
    const Meta& mf = g_meta.at("F");
    const uint32_t* F = load("F");
    const mj_rel RF = rel_of(F, mf.n);
    const uint32_t A = mf.a_domain;
    mj_plan_t plan;
    std::memset(&plan, 0, sizeof plan);
    check(make_plan(ctx, MJ_LINEAR, &RF, &RF, &RF, A, &plan), "mj_plan");
    std::printf("[replay] plan algo %d nb %u nc %u flags %u b_dom %u c_dom %u join2 %" PRIu64 " ws %" PRIu64 "\n",
                plan.algo, plan.log2_nb, plan.log2_nc, plan.flags, plan.b_domain, plan.c_domain, plan.join2_size,
                plan.workspace_bytes);
    void* ws = alloc(plan.workspace_bytes);
    uint64_t* out = static_cast<uint64_t*>(alloc(uint64_t(A) * 8));
    if (want("main")) {
        leg("main");
        for (int i = 0; i < 2 + 2 * steps; ++i) {
            if (i == 2) check(mj_ctx_profile(ctx, 1), "profile on");
            check(mj_linear3_count(ctx, &RF, &RF, &RF, A, out, &plan, ws, plan.workspace_bytes, nullptr),
                  "mj_linear3_count");
        }
        char names[32 * 64];
        double ms[64];
        int64_t cnt[64];
        const int k = mj_ctx_profile_read(ctx, 64, names, ms, cnt);
        check(mj_ctx_profile(ctx, 0), "profile off");
        std::printf("[replay]   %d kernels profiled\n", k);
        expect(sum(out, A) == mf.closed, "main: sum of counts equals the closed form");
    }
    if (want("cascade")) {
        leg("cascade");
        void* ws2 = alloc(plan.workspace_bytes);
        uint64_t* cnt = static_cast<uint64_t*>(alloc(uint64_t(A) * 8));
        for (int i = 0; i < 2; ++i)
            check(mj_cascade2_count(ctx, MJ_LINEAR, &RF, &RF, &RF, A, cnt, &plan, ws2, plan.workspace_bytes, nullptr),
                  "mj_cascade2_count");
        const uint64_t sc = sum(cnt, A);
        expect(sc == mf.closed, "cascade: sum equals the closed form");
        if (sc != mf.closed)
            std::printf("[replay]   cascade sum %" PRIu64 ", closed form %" PRIu64 "\n", sc, mf.closed);
        if (want("main")) {
            expect(std::memcmp(cnt, out, uint64_t(A) * 8) == 0, "cascade: equals the three-way join");
            uint64_t ndiff = 0;
            for (uint32_t a = 0; a < A; ++a) {
                if (cnt[a] == out[a]) continue;
                if (ndiff++ < 8)
                    std::printf("[replay]   a=%u cascade %" PRIu64 " three-way %" PRIu64 "\n", a, cnt[a], out[a]);
            }
            if (ndiff) std::printf("[replay]   %" PRIu64 " A values differ\n", ndiff);
        }
        std::free(ws2);
        std::free(cnt);
    }
    if (want("skew")) {
        // heavy keys: the crowded ranges run as several workgroups each,
        // with direct-indexed and with hashed tables, twice in a row
        leg("skew");
        const Meta& mk = g_meta.at("K");
        const uint32_t* K = load("K");
        const mj_rel RK = rel_of(K, mk.n);
        const uint32_t AK = mk.a_domain;
        mj_plan_t pk;
        std::memset(&pk, 0, sizeof pk);
        check(make_plan(ctx, MJ_LINEAR, &RK, &RK, &RK, AK, &pk), "mj_plan skew");
        expect((pk.flags & MJ_PLAN_DENSE_KEYS) != 0, "skew: the planner takes direct-indexed tables");
        mj_plan_t ph = pk;
        ph.algo = MJ_ALGO_3WAY;
        ph.flags = (ph.flags & ~uint32_t(MJ_PLAN_DENSE_KEYS)) | MJ_PLAN_NO_DENSE;
        {
            const uint64_t need = mj_plan_workspace(MJ_LINEAR, RK.n, RK.n, RK.n);
            void* pws = alloc(need);
            check(mj_plan(ctx, MJ_LINEAR, &RK, &RK, &RK, AK, MJ_PLANNER_FIXED, &ph, pws, need, nullptr),
                  "mj_plan skew hashed");
            std::free(pws);
        }
        uint64_t* cd = static_cast<uint64_t*>(alloc(uint64_t(AK) * 8));
        uint64_t* ch = static_cast<uint64_t*>(alloc(uint64_t(AK) * 8));
        void* wsk = alloc(std::max(pk.workspace_bytes, ph.workspace_bytes));
        for (int i = 0; i < 2; ++i) {
            check(mj_linear3_count(ctx, &RK, &RK, &RK, AK, cd, &pk, wsk, pk.workspace_bytes, nullptr), "skew dense");
            expect(sum(cd, AK) == mk.closed, "skew: direct-indexed sum equals the closed form");
            check(mj_linear3_count(ctx, &RK, &RK, &RK, AK, ch, &ph, wsk, ph.workspace_bytes, nullptr), "skew hashed");
            expect(std::memcmp(cd, ch, uint64_t(AK) * 8) == 0, "skew: hashed tables give the same counts");
        }
        std::free(wsk); std::free(cd); std::free(ch);
        std::free(const_cast<uint32_t*>(K));
        // a heavy key among many distinct keys, hashed tables in four
        // buckets of B: a piece that overflows its table (K2) and pieces
        // whose union does (K3)
        for (const char* nm : {"K2", "K3"}) {
            const Meta& m2 = g_meta.at(nm);
            const uint32_t* K2 = load(nm);
            const mj_rel R2 = rel_of(K2, m2.n);
            mj_plan_t p2;
            std::memset(&p2, 0, sizeof p2);
            check(make_plan(ctx, MJ_LINEAR, &R2, &R2, &R2, m2.a_domain, &p2), "mj_plan skew wide");
            p2.algo = MJ_ALGO_3WAY;
            p2.log2_nb = 2;
            p2.flags = (p2.flags & ~uint32_t(MJ_PLAN_DENSE_KEYS)) | MJ_PLAN_NO_DENSE;
            const uint64_t need = mj_plan_workspace(MJ_LINEAR, R2.n, R2.n, R2.n);
            void* pws = alloc(need);
            check(mj_plan(ctx, MJ_LINEAR, &R2, &R2, &R2, m2.a_domain, MJ_PLANNER_FIXED, &p2, pws, need, nullptr),
                  "mj_plan skew wide hashed");
            std::free(pws);
            void* ws2 = alloc(p2.workspace_bytes);
            uint64_t* c2 = static_cast<uint64_t*>(alloc(uint64_t(m2.a_domain) * 8));
            for (int i = 0; i < 2; ++i) {
                check(mj_linear3_count(ctx, &R2, &R2, &R2, m2.a_domain, c2, &p2, ws2, p2.workspace_bytes, nullptr),
                      "skew wide");
                expect(sum(c2, m2.a_domain) == m2.closed, "skew wide: hashed sum equals the closed form");
            }
            std::free(ws2); std::free(c2);
            std::free(const_cast<uint32_t*>(K2));
        }
    }
    if (want("small")) {
        leg("small");
        const Meta& ms = g_meta.at("Fs");
        const uint32_t* Fs = load("Fs");
        const mj_rel RS = rel_of(Fs, ms.n);
        mj_plan_t ps;
        std::memset(&ps, 0, sizeof ps);
        check(make_plan(ctx, MJ_LINEAR, &RS, &RS, &RS, ms.a_domain, &ps), "mj_plan small");
        void* wss = alloc(ps.workspace_bytes);
        uint64_t* c3 = static_cast<uint64_t*>(alloc(uint64_t(ms.a_domain) * 8));
        uint64_t* cc = static_cast<uint64_t*>(alloc(uint64_t(ms.a_domain) * 8));
        for (int i = 0; i < 3; ++i)
            check(mj_linear3_count(ctx, &RS, &RS, &RS, ms.a_domain, c3, &ps, wss, ps.workspace_bytes, nullptr), "small 3-way");
        for (int i = 0; i < 3; ++i)
            check(mj_cascade2_count(ctx, MJ_LINEAR, &RS, &RS, &RS, ms.a_domain, cc, &ps, wss, ps.workspace_bytes, nullptr),
                  "small cascade");
        expect(sum(c3, ms.a_domain) == ms.closed, "small: sum equals the closed form");
        expect(std::memcmp(c3, cc, uint64_t(ms.a_domain) * 8) == 0, "small: cascade equals the three-way join");
        std::free(wss); std::free(c3); std::free(cc);
        std::free(const_cast<uint32_t*>(Fs));
    }
    if (want("fm")) {
        leg("fm");
        const uint64_t need = mj_linear3_distinct_workspace(mf.n, mf.n, mf.n, A);
        void* wsf = alloc(need);
        uint32_t* sk = static_cast<uint32_t*>(alloc(uint64_t(A) * 64));
        double* est = static_cast<double*>(alloc(uint64_t(A) * 8));
        uint64_t h0 = 0;
        for (int i = 0; i < 2; ++i) {
            check(mj_linear3_distinct(ctx, &RF, &RF, &RF, A, 0x5EED, sk, est, wsf, need, nullptr), "mj_linear3_distinct");
            const uint64_t h = fnv(sk, uint64_t(A) * 64);
            if (i == 0) h0 = h;
            else expect(h == h0, "fm: sketches identical on a second call");
        }
        std::printf("[replay]   fm sketch hash %016" PRIx64 "\n", h0);
        std::free(wsf); std::free(sk); std::free(est);
    }
    if (want("emit")) {
        leg("emit");
        const uint64_t need = mj_linear3_materialize_workspace(mf.n, mf.n, mf.n);
        void* wse = alloc(need);
        uint64_t* total = static_cast<uint64_t*>(alloc(8));
        check(mj_linear3_materialize(ctx, &RF, &RF, &RF, 0, 0, nullptr, total, wse, need, nullptr), "emit size");
        expect(*total == mf.closed, "emit: total equals the closed form");
        // windows: the start, the middle, the end (ragged), one past the end
        const uint64_t cap = std::min<uint64_t>(*total, uint64_t(1) << 22);
        uint32_t* rows = static_cast<uint32_t*>(alloc(cap * 16));
        const uint64_t firsts[4] = {0, *total / 2, *total > cap / 2 ? *total - cap / 2 : 0, *total};
        for (uint64_t first : firsts) {
            check(mj_linear3_materialize(ctx, &RF, &RF, &RF, first, cap, rows, total, wse, need, nullptr), "emit window");
        }
        std::free(rows); std::free(total); std::free(wse);
    }
    if (want("star")) {
        leg("star");
        const Meta& mr = g_meta.at("starR");
        const uint32_t* R = load("starR");
        const uint32_t* S = load("starS");
        const uint32_t* T = load("starT");
        const mj_rel rR = rel_of(R, mr.n), rS = rel_of(S, g_meta.at("starS").n), rT = rel_of(T, g_meta.at("starT").n);
        mj_plan_t p;
        std::memset(&p, 0, sizeof p);
        check(make_plan(ctx, MJ_LINEAR, &rR, &rS, &rT, mr.a_domain, &p), "mj_plan star");
        void* wst = alloc(p.workspace_bytes);
        uint64_t* c = static_cast<uint64_t*>(alloc(uint64_t(mr.a_domain) * 8));
        const int algos[4] = {MJ_ALGO_STAR, MJ_ALGO_STAR_CASCADE, MJ_ALGO_3WAY, MJ_ALGO_CASCADE};
        for (int algo : algos) {
            mj_plan_t q = p;
            q.algo = algo;
            for (int i = 0; i < 2; ++i) {
                if (algo == MJ_ALGO_STAR || algo == MJ_ALGO_3WAY)
                    check(mj_linear3_count(ctx, &rR, &rS, &rT, mr.a_domain, c, &q, wst, p.workspace_bytes, nullptr), "star 3-way");
                else
                    check(mj_cascade2_count(ctx, MJ_LINEAR, &rR, &rS, &rT, mr.a_domain, c, &q, wst, p.workspace_bytes,
                                            nullptr), "star cascade");
            }
            char what[80];
            std::snprintf(what, sizeof what, "star algo %d: sum equals the closed form", algo);
            expect(sum(c, mr.a_domain) == mr.closed, what);
        }
        std::free(wst); std::free(c);
        std::free(const_cast<uint32_t*>(R)); std::free(const_cast<uint32_t*>(S)); std::free(const_cast<uint32_t*>(T));
    }
    if (want("slarge")) {
        leg("slarge");
        const Meta& mr = g_meta.at("slR");
        const uint32_t* R = load("slR");
        const uint32_t* S = load("slS");
        const uint32_t* T = load("slT");
        const mj_rel rR = rel_of(R, mr.n), rS = rel_of(S, g_meta.at("slS").n), rT = rel_of(T, g_meta.at("slT").n);
        mj_plan_t p;
        std::memset(&p, 0, sizeof p);
        check(make_plan(ctx, MJ_LINEAR, &rR, &rS, &rT, mr.a_domain, &p), "mj_plan S-largest");
        expect(p.algo == MJ_ALGO_SLARGE, "slarge: the planner picks the S-largest form");
        void* wst = alloc(p.workspace_bytes);
        const uint64_t na = mr.a_domain;
        uint64_t* c0 = static_cast<uint64_t*>(alloc(na * 8));
        uint64_t* c1 = static_cast<uint64_t*>(alloc(na * 8));
        for (int i = 0; i < 2; ++i)
            check(mj_linear3_count(ctx, &rR, &rS, &rT, mr.a_domain, c0, &p, wst, p.workspace_bytes, nullptr),
                  "S-largest");
        expect(sum(c0, na) == mr.closed, "slarge: sum equals the closed form");
        mj_plan_t q = p;
        q.algo = MJ_ALGO_3WAY;
        check(mj_linear3_count(ctx, &rR, &rS, &rT, mr.a_domain, c1, &q, wst, p.workspace_bytes, nullptr), "3-way");
        expect(std::memcmp(c0, c1, na * 8) == 0, "slarge: equals the partitioned three-way join");
        q.algo = MJ_ALGO_CASCADE;
        check(mj_cascade2_count(ctx, MJ_LINEAR, &rR, &rS, &rT, mr.a_domain, c1, &q, wst, p.workspace_bytes, nullptr),
              "cascade");
        expect(std::memcmp(c0, c1, na * 8) == 0, "slarge: equals the cascade");
        std::free(wst); std::free(c0); std::free(c1);
        std::free(const_cast<uint32_t*>(R)); std::free(const_cast<uint32_t*>(S)); std::free(const_cast<uint32_t*>(T));
    }
    if (want("batch")) {
        // small joins of both kinds under every plan form, as one batch:
        // each join's result equals its own call's, on two calls in a row
        leg("batch");
        const int algos_lin[3] = {MJ_ALGO_3WAY, MJ_ALGO_CASCADE, MJ_ALGO_STAR};
        const int algos_tri[3] = {MJ_ALGO_3WAY, MJ_ALGO_CASCADE, MJ_ALGO_ORIENTED};
        std::vector<const uint32_t*> data;
        std::vector<mj_batch_item> items;
        std::vector<std::vector<uint64_t>> want_out;
        for (int k = 0; g_meta.count("B" + std::to_string(k)); ++k) {
            const std::string nm = "B" + std::to_string(k);
            const Meta& m = g_meta.at(nm);
            const uint32_t* X = load(nm);
            data.push_back(X);
            const mj_rel r = rel_of(X, m.n);
            const int kind = m.a_domain ? MJ_LINEAR : MJ_TRIANGLE;
            mj_plan_t p;
            std::memset(&p, 0, sizeof p);
            check(make_plan(ctx, kind, &r, &r, &r, m.a_domain, &p), "mj_plan batch");
            p.algo = kind == MJ_LINEAR ? algos_lin[k % 3] : algos_tri[k % 3];
            if (p.algo == MJ_ALGO_STAR && (m.n > 4096)) p.algo = MJ_ALGO_3WAY;
            if (p.algo == MJ_ALGO_ORIENTED && !(p.flags & MJ_PLAN_SYMMETRIC_SIMPLE)) p.algo = MJ_ALGO_3WAY;
            if (p.algo == MJ_ALGO_STAR) { p.log2_nb = 0; p.log2_nc = 0; }
            {
                const uint64_t need = mj_plan_workspace(kind, r.n, r.n, r.n);
                void* pws = alloc(need);
                check(mj_plan(ctx, kind, &r, &r, &r, m.a_domain, MJ_PLANNER_FIXED, &p, pws, need, nullptr),
                      "mj_plan batch fixed");
                std::free(pws);
            }
            const uint64_t len = kind == MJ_LINEAR ? m.a_domain : 1;
            std::vector<uint64_t> ref(len);
            void* wsb = alloc(p.workspace_bytes);
            if (p.algo == MJ_ALGO_CASCADE || p.algo == MJ_ALGO_STAR_CASCADE)
                check(mj_cascade2_count(ctx, kind, &r, &r, &r, m.a_domain, ref.data(), &p, wsb, p.workspace_bytes,
                                        nullptr), "batch: own call");
            else if (kind == MJ_LINEAR)
                check(mj_linear3_count(ctx, &r, &r, &r, m.a_domain, ref.data(), &p, wsb, p.workspace_bytes, nullptr),
                      "batch: own call");
            else
                check(mj_triangle3_count(ctx, &r, &r, &r, ref.data(), &p, wsb, p.workspace_bytes, nullptr),
                      "batch: own call");
            std::free(wsb);
            std::printf("[replay]   join %d: kind %d algo %d n %" PRIu64 " result sum %" PRIu64 "\n", k, kind, p.algo,
                        m.n, sum(ref.data(), len));
            expect(sum(ref.data(), len) == m.closed, "batch: the join's own call gives the expected total");
            mj_batch_item it;
            std::memset(&it, 0, sizeof it);
            it.kind = kind; it.R = r; it.S = r; it.T = r; it.a_domain = m.a_domain; it.plan = p;
            it.out = static_cast<uint64_t*>(alloc(len * 8));
            items.push_back(it);
            want_out.push_back(std::move(ref));
        }
        const int nb = (int)items.size();
        if (nb == 0) std::printf("[replay]   no batch inputs (older data directory)\n");
        const uint64_t need = mj_batch_workspace(items.data(), nb);
        void* wsb = alloc(need);
        for (int call = 0; call < 2; ++call) {
            if (call == 1) check(mj_ctx_profile(ctx, 1), "profile on");
            check(mj_batch_count(ctx, items.data(), nb, wsb, need, nullptr), "mj_batch_count");
            bool same = true;
            for (int k = 0; k < nb; ++k) {
                const bool eq = std::memcmp(items[k].out, want_out[k].data(), want_out[k].size() * 8) == 0;
                if (!eq)
                    std::printf("[replay]   join %d differs: batch sum %" PRIu64 ", own call %" PRIu64 "\n", k,
                                sum(items[k].out, want_out[k].size()), sum(want_out[k].data(), want_out[k].size()));
                same = same && eq;
            }
            expect(same, call ? "batch: a second call gives the same results"
                              : "batch: every join equals its own call");
        }
        char names[64 * 64];
        double ms[64];
        int64_t cnt[64];
        const int nk = mj_ctx_profile_read(ctx, 64, names, ms, cnt);
        check(mj_ctx_profile(ctx, 0), "profile off");
        int64_t launches = 0;
        for (int q = 0; q < nk && q < 64; ++q) launches += cnt[q];
        std::printf("[replay]   batch of %d joins: %" PRId64 " launches:", nb, launches);
        for (int q = 0; q < nk && q < 64; ++q) std::printf(" %.32s x%" PRId64, names + 32 * q, cnt[q]);
        std::printf("\n");
        // one byte short of the workspace is refused
        if (nb)
            expect(mj_batch_count(ctx, items.data(), nb, wsb, need - 1, nullptr) == MJ_ERR_WORKSPACE,
                   "batch: a workspace one byte short is refused");
        std::free(wsb);
        for (auto& it : items) std::free(it.out);
        for (auto* X : data) std::free(const_cast<uint32_t*>(X));
    }
    check(mj_ctx_destroy(ctx), "mj_ctx_destroy");
    std::free(ws); std::free(out); std::free(const_cast<uint32_t*>(F));
    std::printf("[replay] %s\n", g_fail ? "FAILED" : "all checks passed");
    return g_fail ? 1 : 0;
}
