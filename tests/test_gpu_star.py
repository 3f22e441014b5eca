"""GPU parity of the star three-way join and the binary star cascade
(Sec. 6, linear star join) against the oracle: bit-exact uint64 per-A
counts.  Same query as the linear join; R and T are small dimension
relations, S a large fact relation."""
import numpy as np
import pytest

import oracle
from tests import brute
from tests.gpu_util import banner, dev, fixed_plan
from workloads import generators as G

pytestmark = pytest.mark.gpu

STARS = ("STAR", "STAR_CASCADE")


@pytest.fixture(scope="module")
def mj():
    import paper_1905_13376_amd as mj
    return mj


@pytest.fixture(scope="module")
def ctx(mj):
    c = mj.Context()
    yield c
    c.close()


def run_star(mj, ctx, R, S, T, a_domain, algo, **fields):
    import torch
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = fixed_plan(mj, ctx, mj.LINEAR, Rd, Sd, Td, a_domain, algo=getattr(mj, "ALGO_" + algo),
                   seed=fields.pop("seed", 0x1B873593), **fields)
    out = torch.full((max(a_domain, 1),), -1, dtype=torch.int64, device="cuda")
    if algo == "STAR":
        ctx.linear3_count(Rd, Sd, Td, a_domain, plan=p, out=out)
    else:
        ctx.cascade2_count(mj.LINEAR, Rd, Sd, Td, a_domain, plan=p, out=out)
    return mj.as_u64(out)[:a_domain]


@pytest.mark.parametrize("algo", STARS)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_star_schema_small(mj, ctx, algo, seed):
    banner(f"star schema small {algo} seed={seed}")
    R, S, T = G.star_schema(n_fact=1 << 16, k_r=512, k_t=512, a_domain=256, seed=seed)
    got = run_star(mj, ctx, R, S, T, 256, algo)
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, 256))


@pytest.mark.parametrize("algo", STARS)
@pytest.mark.parametrize("seed", range(4))
def test_star_random_bags_and_special_keys(mj, ctx, algo, seed):
    # dimensions with repeated B and C values (bags), the keys 0xFFFFFFFF and
    # 0x80000000 on every join column, and fact keys missing from both sides
    banner(f"star random bags {algo} seed={seed}")
    rng = np.random.default_rng(100 + seed)
    dom = [3, 40, 900, 5000][seed]
    nr, nt = (int(x) for x in rng.integers(1, 3000, size=2))
    ns = int(rng.integers(1, 60000))
    a_domain = int(rng.integers(1, 600))
    R = np.stack([rng.integers(0, a_domain, nr), rng.integers(0, dom, nr)], axis=1).astype(np.uint32)
    S = rng.integers(0, dom + 10, size=(ns, 2)).astype(np.uint32)
    T = rng.integers(0, dom, size=(nt, 2)).astype(np.uint32)
    special = np.array([0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    R[: min(5, nr), 1] = special[0]
    S[: min(50, ns), 0] = special[rng.integers(0, 2, min(50, ns))]
    S[: min(50, ns), 1] = special[rng.integers(0, 2, min(50, ns))]
    T[: min(5, nt), 0] = special[rng.integers(0, 2, min(5, nt))]
    got = run_star(mj, ctx, R, S, T, a_domain, algo)
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, a_domain))


@pytest.mark.parametrize("algo", STARS)
def test_star_beyond_lds_groups(mj, ctx, algo):
    # more distinct B values in R than one workgroup's LDS array holds (and,
    # for the cascade, more A values): the sums go to global memory
    banner(f"star beyond LDS groups {algo}")
    R, S, T = G.star_schema(n_fact=200000, k_r=20000, k_t=3000, a_domain=9000, seed=7)
    got = run_star(mj, ctx, R, S, T, 9000, algo)
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, 9000))


@pytest.mark.parametrize("algo", STARS)
def test_star_empty_and_tiny(mj, ctx, algo):
    banner(f"star empty and tiny {algo}")
    one = np.array([[1, 2]], dtype=np.uint32)
    empty = np.zeros((0, 2), dtype=np.uint32)
    for R, S, T in ((empty, one, one), (one, empty, one), (one, one, empty)):
        got = run_star(mj, ctx, R, S, T, 4, algo)
        assert not got.any()
    R = np.array([[3, 7]] * 2, dtype=np.uint32)
    S = np.array([[7, 9]] * 3, dtype=np.uint32)
    T = np.array([[9, 0]] * 5, dtype=np.uint32)
    got = run_star(mj, ctx, R, S, T, 4, algo)
    assert got.tolist() == [0, 0, 0, 30]


def test_star_planned_for_star_shapes(mj, ctx):
    banner("planner picks a star plan for small dimensions")
    R, S, T = G.star_schema(n_fact=1 << 20, k_r=1024, k_t=1024, a_domain=512, seed=11)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, 512)
    assert p.est_ms_star > 0.0 and p.algo == mj.ALGO_STAR
    got = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 512, plan=p))
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, 512))
    # and never for a large R
    F = G.linear_powerlaw(seed=12, n_vertices=1 << 12, m=1 << 16)
    Fd = dev(F)
    q = ctx.plan(mj.LINEAR, Fd, Fd, Fd, 1 << 12)
    assert q.est_ms_star == 0.0 and q.algo in (mj.ALGO_3WAY, mj.ALGO_CASCADE)


def test_star_full_size_sampled(mj, ctx):
    """The benchmarked star workload (2^26 fact tuples, 4096-tuple
    dimensions): the sum equals the closed form and sampled A values equal
    the oracle's counts, for both star plans."""
    banner("star full size 2^26 fact tuples")
    R, S, T = G.star_schema()
    a_domain = G.STAR["a_domain"]
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    total = brute.linear_closed_total(R, S, T)
    sample = np.arange(0, a_domain, 37, dtype=np.uint32)
    al, want = oracle.linear3_count_sampled(R, S[: 1 << 22], T, sample)
    for algo in STARS:
        p = fixed_plan(mj, ctx, mj.LINEAR, Rd, Sd, Td, a_domain, algo=getattr(mj, "ALGO_" + algo),
                       seed=0x1B873593)
        run = ctx.linear3_count if algo == "STAR" else (
            lambda *a, **k: ctx.cascade2_count(mj.LINEAR, *a, **k))
        got = mj.as_u64(run(Rd, Sd, Td, a_domain, plan=p))
        assert int(got.sum(dtype=np.uint64)) == total
        # sampled counts on the first 2^22 fact tuples
        Sd2 = dev(S[: 1 << 22])
        p2 = fixed_plan(mj, ctx, mj.LINEAR, Rd, Sd2, Td, a_domain, algo=getattr(mj, "ALGO_" + algo),
                        seed=0x1B873593)
        got2 = mj.as_u64(run(Rd, Sd2, Td, a_domain, plan=p2))
        np.testing.assert_array_equal(got2[al], want)


def test_star_in_batch(mj, ctx):
    banner("star plans inside a batch")
    import torch
    R, S, T = G.star_schema(n_fact=50000, k_r=300, k_t=300, a_domain=100, seed=21)
    F = G.linear_small()[:5000]
    Rd, Sd, Td, Fd = dev(R), dev(S), dev(T), dev(F)
    joins, plans = [], []
    for algo in (mj.ALGO_STAR, mj.ALGO_STAR_CASCADE):
        joins.append((mj.LINEAR, Rd, Sd, Td, 100))
        plans.append(fixed_plan(mj, ctx, mj.LINEAR, Rd, Sd, Td, 100, algo=algo, seed=0x1B873593))
    joins.append((mj.LINEAR, Fd, Fd, Fd, 4096))
    plans.append(ctx.plan(mj.LINEAR, Fd, Fd, Fd, 4096))
    outs = ctx.batch(joins, plans=plans).run()
    torch.cuda.synchronize()
    want = oracle.linear3_count(R, S, T, 100)
    np.testing.assert_array_equal(mj.as_u64(outs[0]), want)
    np.testing.assert_array_equal(mj.as_u64(outs[1]), want)
    np.testing.assert_array_equal(mj.as_u64(outs[2]), oracle.linear3_count(F, F, F, 4096))
