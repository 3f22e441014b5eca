"""GPU parity of the linear three-way join on skewed inputs (heavy keys,
Sec. 1.2's skew, with overflow workgroups: a range or bucket holding too
many tuples for one workgroup runs as several) against the oracle:
bit-exact uint64 per-A counts, with direct-indexed and with hashed tables."""
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


def heavy_relation(n, dom, heavy, seed):
    """n uniform (x, y) tuples over [0, dom)^2, then the leading fractions
    of the rows given by `heavy` (key -> fraction) set to that first-column
    key, shuffled."""
    g = np.random.default_rng(seed)
    F = g.integers(0, dom, size=(n, 2)).astype(np.uint32)
    at = 0
    for key, frac in heavy:
        k = int(n * frac)
        F[at:at + k, 0] = key
        at += k
    g.shuffle(F)
    return F


def both_tables(mj, ctx, R, S, T, a_domain):
    """Per-A counts under the planner's plan and under hashed tables."""
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, a_domain)
    got = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, a_domain, plan=p)).copy()
    q = fixed_plan(mj, ctx, mj.LINEAR, Rd, Sd, Td, a_domain, algo=mj.ALGO_3WAY, log2_nb=p.log2_nb,
                   log2_nc=p.log2_nc, seed=p.seed, flags=mj.PLAN_NO_DENSE)
    hashed = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, a_domain, plan=q)).copy()
    return p, got, hashed


@pytest.mark.parametrize("n,heavy,seed", [
    (1 << 18, [(5, 0.25), (3000, 0.35)], 1),        # two crowded ranges (2 and 3 pieces)
    (1 << 18, [(0, 1.0)], 2),                       # every tuple on one key
    (1 << 18, [(4095, 0.6)], 3),                    # the last range
    (300000, [(17, 0.1), (18, 0.1), (2000, 0.05)], 4),
    (5000, [(1, 0.9)], 5),                          # below the smallest piece: no split
])
def test_heavy_keys_match_oracle(mj, ctx, n, heavy, seed):
    banner(f"skew: n={n} heavy={heavy}")
    F = heavy_relation(n, 4096, heavy, seed)
    p, got, hashed = both_tables(mj, ctx, F, F, F, 4096)
    want = oracle.linear3_count(F, F, F, 4096)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(hashed, want)


def test_heavy_keys_distinct_relations(mj, ctx):
    """R crowded on A, S on B, T on C, each in other places."""
    banner("skew: three relations crowded on their partition keys")
    R = heavy_relation(200000, 3000, [(7, 0.5)], 11)
    S = heavy_relation(250000, 3000, [(2999, 0.4), (1500, 0.2)], 12)
    T = heavy_relation(150000, 3000, [(0, 0.7)], 13)
    p, got, hashed = both_tables(mj, ctx, R, S, T, 3000)
    want = oracle.linear3_count(R, S, T, 3000)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(hashed, want)


def test_split_plan_reused(mj, ctx):
    """The same plan and workspace twice, then on another skewed input of
    the same sizes (the per-range piece counts come from the data)."""
    banner("skew: one plan, two inputs")
    F1 = heavy_relation(1 << 18, 4096, [(9, 0.5)], 21)
    F2 = heavy_relation(1 << 18, 4096, [(4000, 0.3), (100, 0.3)], 22)
    F1d, F2d = dev(F1), dev(F2)
    p = ctx.plan(mj.LINEAR, F1d, F1d, F1d, 4096)
    ws = ctx.workspace(p.workspace_bytes, F1d.device)
    want1 = oracle.linear3_count(F1, F1, F1, 4096)
    for _ in range(2):
        np.testing.assert_array_equal(
            mj.as_u64(ctx.linear3_count(F1d, F1d, F1d, 4096, plan=p, workspace=ws)), want1)
    # a fresh plan for the second input (its fingerprint differs), same workspace
    p2 = ctx.plan(mj.LINEAR, F2d, F2d, F2d, 4096)
    assert p2.workspace_bytes <= ws.numel()
    np.testing.assert_array_equal(mj.as_u64(ctx.linear3_count(F2d, F2d, F2d, 4096, plan=p2, workspace=ws)),
                                  oracle.linear3_count(F2, F2, F2, 4096))


def test_uncapped_powerlaw_full_size(mj, ctx):
    """2^24 edges over 2^20 vertices with uncapped Zipf(1.1) out-degrees
    (the largest about 1.2 million): sums equal the closed form, sampled A
    values (the heaviest among them) equal the oracle, and both table forms
    agree everywhere."""
    banner("skew: uncapped power-law 2^24 edges")
    n = 1 << 20
    F = G.powerlaw_friends(n, 1 << 24, 1234, cap=n - 1).view(np.uint32)
    p, got, hashed = both_tables(mj, ctx, F, F, F, n)
    np.testing.assert_array_equal(got, hashed)
    assert int(got.sum(dtype=np.uint64)) == brute.linear_closed_total(F, F, F)
    deg = np.bincount(F[:, 0].astype(np.int64), minlength=n)
    rng = np.random.default_rng(8)
    sample = np.unique(np.concatenate([np.argsort(deg)[-4:], rng.integers(0, n, 40)])).astype(np.uint32)
    al, want = oracle.linear3_count_sampled(F, F, F, sample)
    np.testing.assert_array_equal(got[al], want)


@pytest.mark.parametrize("m,dom,heavy", [(131072, 1 << 16, 52428), (86000, 19200, 40000), (300000, 1 << 20, 120000)])
def test_heavy_bucket_among_many_keys_hashed(mj, ctx, m, dom, heavy):
    """Hashed tables in four buckets of B with one heavy key: the heavy
    bucket runs as pieces; a piece whose table overflows sends the bucket
    back to one workgroup (keys below 2^16), pieces whose union overflows
    have the pass redone from the tuples (keys below 19200)."""
    banner(f"skew: hashed, heavy bucket among {dom} keys")
    F = heavy_relation(m, dom, [(77, heavy / m)], 31)
    Fd = dev(F)
    p = fixed_plan(mj, ctx, mj.LINEAR, Fd, Fd, Fd, dom, algo=mj.ALGO_3WAY, log2_nb=2, log2_nc=3,
                   seed=0x1B873593, flags=mj.PLAN_NO_DENSE)
    got = mj.as_u64(ctx.linear3_count(Fd, Fd, Fd, dom, plan=p))
    np.testing.assert_array_equal(got, oracle.linear3_count(F, F, F, dom))
