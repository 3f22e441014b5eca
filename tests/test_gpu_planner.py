"""Planner and autotuner on the GPU: whatever plan is chosen, counts stay
bit-exact; the analytic choice follows the intermediate size; the cyclic
cascade equals the three-way cyclic join."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, dev, fixed_plan
from workloads import generators as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mj():
    import paper_1905_13376_amd as mj
    return mj


@pytest.fixture(scope="module")
def ctx(mj):
    c = mj.Context()
    yield c
    c.close()


def test_plan_records_exact_intermediate_and_estimates(mj, ctx):
    banner("planner estimates")
    F = G.linear_powerlaw(seed=5, n_vertices=1 << 14, m=1 << 18)
    Fd = dev(F)
    p = ctx.plan(mj.LINEAR, Fd, Fd, Fd, 1 << 14)
    assert p.join2_size == oracle.join2_size(F, F)
    assert p.est_ms_3way > 0 and p.est_ms_cascade > 0
    # a dense self-join (|I| >> |S|) is planned as a three-way join
    assert p.join2_size > 10 * F.shape[0] and p.algo == mj.ALGO_3WAY


def test_plan_cascade_estimate_follows_intermediate(mj, ctx):
    banner("planner: selective join")
    rng = np.random.default_rng(4)
    n = 200000
    R = np.stack([rng.integers(0, 1000, n), rng.integers(0, 1 << 30, n)], 1).astype(np.uint32)
    S = np.stack([rng.integers(0, 1 << 30, n), rng.integers(0, 1 << 30, n)], 1).astype(np.uint32)
    S[:100, 0] = R[:100, 1]                   # a handful of matches only
    T = rng.integers(0, 1 << 30, size=(n, 2)).astype(np.uint32)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, 1000)
    assert p.join2_size == oracle.join2_size(R, S)
    # with almost no intermediate the two estimates are close; the plan takes
    # the smaller one and both algorithms give the oracle's counts
    assert p.est_ms_cascade < 1.5 * p.est_ms_3way
    assert p.algo == (mj.ALGO_CASCADE if p.est_ms_cascade < p.est_ms_3way else mj.ALGO_3WAY)
    want = oracle.linear3_count(R, S, T, 1000)
    got = mj.as_u64(ctx.cascade2_count(mj.LINEAR, Rd, Sd, Td, 1000, plan=p))
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 1000, plan=p)), want)
    # a dense self-join of the same size: the cascade estimate is far larger
    F = G.uniform_pairs(n, 2000, seed=3)
    Fd = dev(F)
    q = ctx.plan(mj.LINEAR, Fd, Fd, Fd, 2000)
    assert q.join2_size > 50 * n and q.est_ms_cascade > 3 * q.est_ms_3way


def test_autotune_linear_is_exact_and_cached(mj, ctx):
    banner("autotune linear")
    F = G.linear_powerlaw(seed=11, n_vertices=1 << 15, m=1 << 19)
    Fd = dev(F)
    want = oracle.linear3_count(F, F, F, 1 << 15)
    plan, ms, out = ctx.autotune(mj.LINEAR, Fd, Fd, Fd, 1 << 15)
    assert ms > 0
    np.testing.assert_array_equal(mj.as_u64(out), want)
    plan2, ms2, out2 = ctx.autotune(mj.LINEAR, Fd, Fd, Fd, 1 << 15)
    assert (plan2.algo, plan2.log2_nb, plan2.log2_nc) == (plan.algo, plan.log2_nb, plan.log2_nc)
    assert ms2 == ms                           # served from the cache
    np.testing.assert_array_equal(mj.as_u64(out2), want)


def test_autotune_triangle(mj, ctx):
    banner("autotune cyclic")
    E = G.triangle_rmat(scale=12, m_undirected=16 << 12, seed=8)
    Ed = dev(E)
    plan, ms, out = ctx.autotune(mj.TRIANGLE, Ed, Ed, Ed)
    assert int(mj.as_u64(out)[0]) == oracle.triangle3_count(E, E, E)
    assert plan.log2_share <= 5 or plan.algo == mj.ALGO_CASCADE


@pytest.mark.parametrize("seed", range(4))
def test_cyclic_cascade(mj, ctx, seed):
    banner(f"cyclic cascade seed={seed}")
    rng = np.random.default_rng(90 + seed)
    dom = [5, 40, 400, 6000][seed]
    R, S, T = (rng.integers(0, dom, size=(int(rng.integers(1, 20000)), 2)).astype(np.uint32)
               for _ in range(3))
    R[:50, 0] = 0xFFFFFFFF
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    out = ctx.cascade2_count(mj.TRIANGLE, Rd, Sd, Td)
    want = oracle.triangle3_count(R, S, T)
    assert int(mj.as_u64(out)[0]) == want
    assert int(mj.as_u64(ctx.triangle3_count(Rd, Sd, Td))[0]) == want


def test_cyclic_cascade_chunked(mj, ctx):
    import torch
    banner("cyclic cascade chunked")
    E = G.gnm_symmetric(3000, 60000, seed=4)
    Ed = dev(E)
    p = ctx.plan(mj.TRIANGLE, Ed, Ed, Ed)
    need = p.workspace_bytes - 8 * min(p.join2_size, 1 << 28) + 8 * (p.join2_size // 5 + 1)
    need = max(need, 1 << 20)
    ws = torch.empty(int(need), dtype=torch.uint8, device="cuda")
    # the three-way layout may need more than the shrunken cascade slice
    out = ctx.cascade2_count(mj.TRIANGLE, Ed, Ed, Ed, plan=p, workspace=ws)
    assert int(mj.as_u64(out)[0]) == oracle.triangle3_count(E, E, E)
