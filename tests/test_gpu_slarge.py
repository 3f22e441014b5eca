"""GPU parity of the S-largest form of the linear three-way join (Sec. 4,
the paragraph after Algorithm 1: S the largest relation, R and T split
into L sub-partitions each, the L x L partitions of S streamed past the
pairs) against the oracle: bit-exact uint64 per-A counts."""
import numpy as np
import pytest

import oracle
from tests import brute
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


def run_slarge(mj, ctx, R, S, T, a_domain, log2_nb, log2_nc, seed=0x1B873593):
    import torch
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = fixed_plan(mj, ctx, mj.LINEAR, Rd, Sd, Td, a_domain, algo=mj.ALGO_SLARGE, log2_nb=log2_nb,
                   log2_nc=log2_nc, seed=seed, flags=mj.PLAN_NO_DENSE)
    out = torch.full((max(a_domain, 1),), -1, dtype=torch.int64, device="cuda")
    ctx.linear3_count(Rd, Sd, Td, a_domain, plan=p, out=out)
    return mj.as_u64(out)[:a_domain]


def test_planner_picks_slarge_for_large_dimensions(mj, ctx):
    """Dimension relations of 2^14 tuples (beyond the star plans) and a fact
    relation 64 times larger: the planner takes the S-largest form, whose
    counts equal the oracle's."""
    banner("S-largest planned")
    R, S, T = G.star_schema(n_fact=1 << 20, k_r=1 << 14, k_t=1 << 14, a_domain=1 << 12, seed=41)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, 1 << 12)
    assert p.algo == mj.ALGO_SLARGE and p.est_ms_slarge > 0
    got = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 1 << 12, plan=p))
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, 1 << 12))
    # the same plan through the cascade and the partitioned three-way join
    q = p.copy()
    q.algo = mj.ALGO_3WAY
    np.testing.assert_array_equal(mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 1 << 12, plan=q)), got)


@pytest.mark.parametrize("nb,nc", [(0, 0), (3, 5), (6, 6), (1, 11), (11, 1)])
def test_slarge_bucket_counts(mj, ctx, nb, nc):
    banner(f"S-largest log2 buckets B={nb} C={nc}")
    R, S, T = G.star_schema(n_fact=1 << 18, k_r=3000, k_t=5000, a_domain=700, seed=43 + nb)
    got = run_slarge(mj, ctx, R, S, T, 700, nb, nc)
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, 700))


@pytest.mark.parametrize("seed", range(4))
def test_slarge_random_bags_and_special_keys(mj, ctx, seed):
    """Bags with repeated keys on every join column, the keys 0xFFFFFFFF and
    0x80000000, and S tuples matching neither side."""
    banner(f"S-largest random bags seed={seed}")
    rng = np.random.default_rng(300 + seed)
    dom = [3, 50, 2000, 60000][seed]
    R = rng.integers(0, dom, size=(int(rng.integers(1, 6000)), 2)).astype(np.uint32)
    S = rng.integers(0, dom, size=(int(rng.integers(20000, 90000)), 2)).astype(np.uint32)
    T = rng.integers(0, dom, size=(int(rng.integers(1, 6000)), 2)).astype(np.uint32)
    R[:, 0] = rng.integers(0, 300, R.shape[0])
    special = np.array([0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    for X, col in ((R, 1), (S, 0), (S, 1), (T, 0)):
        m = rng.random(X.shape[0]) < 0.05
        X[m, col] = special[rng.integers(0, 2, size=m.sum())]
    got = run_slarge(mj, ctx, R, S, T, 300, 2, 3, seed=seed + 7)
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, 300))


def test_slarge_tables_beyond_the_stage_and_split_passes(mj, ctx):
    """One part of T with 20,000 distinct C values (its table is probed in
    global memory, not staged) and one part of R with 20,000 distinct B
    values (the per-B sums are split into passes)."""
    banner("S-largest: unstaged T table, split W passes")
    rng = np.random.default_rng(77)
    R = np.stack([rng.integers(0, 1000, 40000), rng.integers(0, 20000, 40000)], 1).astype(np.uint32)
    T = np.stack([rng.integers(0, 20000, 40000), rng.integers(0, 9, 40000)], 1).astype(np.uint32)
    S = np.stack([rng.integers(0, 20000, 300000), rng.integers(0, 20000, 300000)], 1).astype(np.uint32)
    got = run_slarge(mj, ctx, R, S, T, 1000, 0, 0)
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, 1000))


def test_slarge_empty_inputs_and_buckets(mj, ctx):
    banner("S-largest empty inputs")
    e = np.zeros((0, 2), dtype=np.uint32)
    R, S, T = G.star_schema(n_fact=5000, k_r=100, k_t=100, a_domain=64, seed=3)
    R, S, T = (x.view(np.uint32) for x in (R, S, T))
    for r, s, t in ((e, S, T), (R, e, T), (R, S, e)):
        assert not run_slarge(mj, ctx, r, s, t, 64, 4, 4).any()
    # many empty (i, j) cells: 2^12 cells for 5000 tuples
    np.testing.assert_array_equal(run_slarge(mj, ctx, R, S, T, 64, 6, 6), oracle.linear3_count(R, S, T, 64))


def test_slarge_full_size_sampled(mj, ctx):
    """2^26 fact tuples with dimension relations of 2^16 tuples: the planner
    takes the S-largest form; the sum equals the closed form and sampled A
    values equal the oracle's counts."""
    banner("S-largest full size 2^26 fact tuples")
    R, S, T = G.star_schema(n_fact=1 << 26, k_r=1 << 16, k_t=1 << 16, a_domain=1 << 14, seed=5002)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, 1 << 14)
    assert p.algo == mj.ALGO_SLARGE
    got = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 1 << 14, plan=p))
    assert int(got.sum(dtype=np.uint64)) == brute.linear_closed_total(R, S, T)
    rng = np.random.default_rng(5)
    sample = rng.integers(0, 1 << 14, 64).astype(np.uint32)
    al, want = oracle.linear3_count_sampled(R, S, T, sample)
    np.testing.assert_array_equal(got[al], want)
