// Host-build checks of the C ABI that need a context (test infrastructure
// only): planning with a too-small planning workspace, a plan given other
// relations of the same sizes, and a too-small count workspace.
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <vector>

#include "mj.h"

static int fails = 0;
static void expect(bool ok, const char* what) {
    std::printf("[abi] %-64s %s\n", what, ok ? "ok" : "FAILED");
    if (!ok) ++fails;
}

int main() {
    mj_ctx* ctx = nullptr;
    if (mj_ctx_create(0, &ctx) != MJ_OK) { std::printf("[abi] no context\n"); return 2; }
    const uint64_t n = 5000;
    std::vector<uint32_t> F(2 * n), G(2 * n);
    for (uint64_t i = 0; i < n; ++i) {
        F[2 * i] = (uint32_t)((i * 7919u) % 600u);
        F[2 * i + 1] = (uint32_t)((i * 104729u) % 600u);
        G[2 * i] = F[2 * i];
        G[2 * i + 1] = F[2 * i + 1];
    }
    mj_rel R{F.data(), F.data() + 1, n, 2};
    mj_rel R2{G.data(), G.data() + 1, n, 2};
    const uint64_t need = mj_plan_workspace(MJ_LINEAR, n, n, n);
    std::vector<unsigned char> pws(need);
    mj_plan_t p;
    std::memset(&p, 0, sizeof p);
    expect(mj_plan(ctx, MJ_LINEAR, &R, &R, &R, 600, MJ_PLANNER_ANALYTIC, &p, pws.data(), need - 1, nullptr) ==
               MJ_ERR_WORKSPACE, "planning workspace one byte short: MJ_ERR_WORKSPACE");
    expect(mj_plan(ctx, MJ_LINEAR, &R, &R, &R, 600, MJ_PLANNER_ANALYTIC, &p, nullptr, need, nullptr) ==
               MJ_ERR_WORKSPACE, "no planning workspace: MJ_ERR_WORKSPACE");
    expect(mj_plan(ctx, MJ_LINEAR, &R, &R, &R, 600, MJ_PLANNER_ANALYTIC, &p, pws.data(), need, nullptr) == MJ_OK,
           "planning workspace of mj_plan_workspace() bytes: MJ_OK");
    std::vector<unsigned char> ws(p.workspace_bytes);
    std::vector<uint64_t> out(600);
    expect(mj_linear3_count(ctx, &R, &R, &R, 600, out.data(), &p, ws.data(), ws.size(), nullptr) == MJ_OK,
           "count on the planned relations: MJ_OK");
    uint64_t total = 0;
    for (uint64_t v : out) total += v;
    expect(total > 0, "count on the planned relations: a nonzero total");
    expect(mj_linear3_count(ctx, &R2, &R2, &R2, 600, out.data(), &p, ws.data(), ws.size(), nullptr) ==
               MJ_ERR_PLAN_MISMATCH, "same sizes, other relations: MJ_ERR_PLAN_MISMATCH");
    expect(mj_cascade2_count(ctx, MJ_LINEAR, &R2, &R, &R, 600, out.data(), &p, ws.data(), ws.size(), nullptr) ==
               MJ_ERR_PLAN_MISMATCH, "cascade, other R: MJ_ERR_PLAN_MISMATCH");
    expect(mj_linear3_count(ctx, &R, &R, &R, 600, out.data(), &p, ws.data(), 64, nullptr) == MJ_ERR_WORKSPACE,
           "count workspace too small: MJ_ERR_WORKSPACE");
    // a plan reused on the same relations after their contents changed so
    // that |R join S| grew: the cascade's chunks cover the planned |I| only,
    // so every count must come out all ones, with direct-indexed and with
    // hashed tables
    for (int hashed = 0; hashed < 2; ++hashed) {
        for (uint64_t i = 0; i < n; ++i) G[2 * i + 1] = F[2 * i + 1];
        mj_plan_t q;
        std::memset(&q, 0, sizeof q);
        if (hashed) { q.log2_nb = 3; q.log2_nc = 3; q.seed = 7; q.flags = MJ_PLAN_NO_DENSE; q.algo = MJ_ALGO_CASCADE; }
        const int planner = hashed ? MJ_PLANNER_FIXED : MJ_PLANNER_ANALYTIC;
        if (mj_plan(ctx, MJ_LINEAR, &R2, &R, &R, 600, planner, &q, pws.data(), need, nullptr) != MJ_OK) {
            expect(false, "plan for the changed-data check");
            continue;
        }
        std::vector<unsigned char> wq(q.workspace_bytes);
        std::fill(out.begin(), out.end(), 0);
        expect(mj_cascade2_count(ctx, MJ_LINEAR, &R2, &R, &R, 600, out.data(), &q, wq.data(), wq.size(), nullptr) ==
                   MJ_OK, "cascade on the planned data: MJ_OK");
        bool ones = true;
        for (uint64_t v : out) ones = ones && v == ~0ull;
        expect(!ones, "cascade on the planned data: counts");
        for (uint64_t i = 0; i < n; i += 3) G[2 * i + 1] = 5;     // B = 5 joins many more S tuples
        expect(mj_cascade2_count(ctx, MJ_LINEAR, &R2, &R, &R, 600, out.data(), &q, wq.data(), wq.size(), nullptr) ==
                   MJ_OK, "cascade after R changed in place: MJ_OK (checked on the device)");
        ones = true;
        for (uint64_t v : out) ones = ones && v == ~0ull;
        expect(ones, hashed ? "larger intermediate than planned (hashed tables): all ones"
                            : "larger intermediate than planned (direct-indexed): all ones");
    }
    // the allocation-free entry point: the same counts as the workspace call,
    // twice in a row (the second on a smaller input), and a refusal before
    // any launch when the plan's path needs more than the static array
    for (uint64_t m : {uint64_t(5000), uint64_t(1234)}) {
        mj_rel Rm{F.data(), F.data() + 1, m, 2};
        mj_plan_t q;
        std::memset(&q, 0, sizeof q);
        expect(mj_plan(ctx, MJ_LINEAR, &Rm, &Rm, &Rm, 600, MJ_PLANNER_ANALYTIC, &q, pws.data(), need, nullptr) == MJ_OK,
               "plan for the allocation-free call");
        std::vector<unsigned char> wq(q.workspace_bytes);
        std::vector<uint64_t> a(600, 7), b(600, 9);
        expect(mj_linear3_count(ctx, &Rm, &Rm, &Rm, 600, a.data(), &q, wq.data(), wq.size(), nullptr) == MJ_OK &&
                   mj_linear3_count_static(ctx, &Rm, &Rm, &Rm, 600, b.data(), &q, nullptr) == MJ_OK && a == b,
               m == 5000 ? "static scratch: equals the workspace call" : "static scratch, smaller input next: equal");
    }
    {
        const uint64_t big = uint64_t(1) << 23;
        std::vector<uint32_t> H(2 * big);
        for (uint64_t i = 0; i < 2 * big; ++i) H[i] = (uint32_t)(((i * 2654435761u) >> 8) & 0xFFFFFFu);   // sparse keys below 2^24
        mj_rel Rb{H.data(), H.data() + 1, big, 2};
        mj_plan_t q;
        std::memset(&q, 0, sizeof q);
        q.log2_nb = 10; q.log2_nc = 10; q.seed = 1; q.flags = MJ_PLAN_NO_DENSE;
        const uint64_t nb = mj_plan_workspace(MJ_LINEAR, big, big, big);
        std::vector<unsigned char> pb(nb);
        std::vector<uint64_t> o(1u << 24);
        expect(mj_plan(ctx, MJ_LINEAR, &Rb, &Rb, &Rb, 1u << 24, MJ_PLANNER_FIXED, &q, pb.data(), nb, nullptr) == MJ_OK &&
                   mj_linear3_count_static(ctx, &Rb, &Rb, &Rb, 1u << 24, o.data(), &q, nullptr) == MJ_ERR_WORKSPACE,
               "static scratch too small for the plan: MJ_ERR_WORKSPACE");
    }
    mj_ctx_destroy(ctx);
    std::printf("[abi] %s\n", fails ? "FAILED" : "all checks passed");
    return fails ? 1 : 0;
}
