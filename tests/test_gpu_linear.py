"""GPU parity of the linear three-way join (Sec. 4) against the oracle:
bit-exact uint64 per-A counts."""
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


def run_linear(mj, ctx, R, S, T, a_domain, plan=None):
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    out = ctx.linear3_count(Rd, Sd, Td, a_domain, plan=plan)
    return mj.as_u64(out)


def test_linear_small_uniform(mj, ctx):
    banner("linear 65,536 uniform tuples over [0,4096)")
    F = G.linear_small()
    got = run_linear(mj, ctx, F, F, F, 4096)
    np.testing.assert_array_equal(got, oracle.linear3_count(F, F, F, 4096))


@pytest.mark.parametrize("nb,nc,seed", [(0, 0, 1), (1, 3, 7), (5, 2, 99), (12, 12, 3), (7, 9, 0xFFFFFFFF)])
def test_linear_bucket_sweep_invariant(mj, ctx, nb, nc, seed):
    banner(f"linear bucket sweep nb=2^{nb} nc=2^{nc} seed={seed}")
    F = G.linear_small()[:20000]
    Fd = dev(F)
    p = fixed_plan(mj, ctx, mj.LINEAR, Fd, Fd, Fd, 4096, log2_nb=nb, log2_nc=nc, seed=seed)
    got = mj.as_u64(ctx.linear3_count(Fd, Fd, Fd, 4096, plan=p))
    np.testing.assert_array_equal(got, oracle.linear3_count(F, F, F, 4096))


@pytest.mark.parametrize("seed", range(6))
def test_linear_random_bags_distinct_relations(mj, ctx, seed):
    banner(f"linear random bags seed={seed}")
    rng = np.random.default_rng(seed)
    dom = [3, 50, 1000, 70000, 5, 300][seed]
    nr, ns, nt = (int(x) for x in rng.integers(1, 30000, size=3))
    R = rng.integers(0, dom, size=(nr, 2)).astype(np.uint32)
    S = rng.integers(0, dom, size=(ns, 2)).astype(np.uint32)
    T = rng.integers(0, dom, size=(nt, 2)).astype(np.uint32)
    # high-bit and sentinel-valued join keys must behave like any other key
    special = np.array([0xFFFFFFFF, 0x80000000, 0xFFFFFFFE], dtype=np.uint32)
    for X, col in ((R, 1), (S, 0), (S, 1), (T, 0)):
        m = rng.random(X.shape[0]) < 0.05
        X[m, col] = special[rng.integers(0, 3, size=m.sum())]
    a_dom = dom
    got = run_linear(mj, ctx, R, S, T, a_dom)
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, a_dom))


def test_linear_overflowing_tables(mj, ctx):
    """One bucket with far more distinct B and C values than an LDS table
    holds: exercises the split passes of the cells and the spilled
    multiplicity tables."""
    banner("linear single-bucket overflow paths")
    rng = np.random.default_rng(5)
    n = 60000
    R = np.stack([rng.integers(0, 512, n), rng.integers(0, 40000, n)], 1).astype(np.uint32)
    S = np.stack([rng.integers(0, 40000, n), rng.integers(0, 30000, n)], 1).astype(np.uint32)
    T = np.stack([rng.integers(0, 30000, n), rng.integers(0, 9, n)], 1).astype(np.uint32)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = fixed_plan(mj, ctx, mj.LINEAR, Rd, Sd, Td, 512, log2_nb=0, log2_nc=0, seed=11)
    got = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 512, plan=p))
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, 512))


def test_linear_empty_and_tiny(mj, ctx):
    banner("linear empty / one-tuple relations")
    e = np.zeros((0, 2), dtype=np.uint32)
    one = np.array([[1, 2]], dtype=np.uint32)
    S1 = np.array([[2, 3]] * 5, dtype=np.uint32)
    T1 = np.array([[3, 0]] * 7, dtype=np.uint32)
    np.testing.assert_array_equal(run_linear(mj, ctx, one, S1, T1, 4),
                                  np.array([0, 35, 0, 0], dtype=np.uint64))
    for R, S, T in ((e, S1, T1), (one, e, T1), (one, S1, e)):
        Rd, Sd, Td = dev(R), dev(S), dev(T)
        got = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 4))
        assert not got.any()


def test_linear_column_layouts(mj, ctx):
    """Separate column tensors (stride 1) and a strided view give the same
    counts as the packed [n, 2] layout."""
    import torch
    banner("linear column layouts")
    F = G.linear_small()[:30000]
    want = oracle.linear3_count(F, F, F, 4096)
    Fd = dev(F)
    soa = torch.stack([Fd[:, 0].contiguous(), Fd[:, 1].contiguous()], 0)  # [2, n]
    R = soa.t()                                  # strides (1, n)
    got = mj.as_u64(ctx.linear3_count(R, R, R, 4096))
    np.testing.assert_array_equal(got, want)
    wide = torch.zeros((F.shape[0], 5), dtype=torch.int32, device="cuda")
    wide[:, 1] = Fd[:, 0]
    wide[:, 3] = Fd[:, 1]
    V = wide[:, 1:4:2]                           # strides (5, 2)
    got = mj.as_u64(ctx.linear3_count(V, V, V, 4096))
    np.testing.assert_array_equal(got, want)


def test_linear_powerlaw_scaled(mj, ctx):
    banner("linear power-law 2^20 edges over 2^16 vertices")
    F = G.linear_powerlaw(seed=2001, n_vertices=1 << 16, m=1 << 20)
    got = run_linear(mj, ctx, F, F, F, 1 << 16)
    np.testing.assert_array_equal(got, oracle.linear3_count(F, F, F, 1 << 16))


def test_linear_powerlaw_full_sampled(mj, ctx):
    """Full-size power-law input (2^24 edges, 2^20 vertices), in the plan
    the benchmark uses: the sum equals the closed form, and sampled A values
    equal the oracle's per-A counts."""
    banner("linear power-law full size 2^24 edges")
    F = G.linear_powerlaw()
    Fd = dev(F)
    got = mj.as_u64(ctx.linear3_count(Fd, Fd, Fd, 1 << 20))
    assert int(got.sum(dtype=np.uint64)) == brute.linear_closed_total(F, F, F)
    rng = np.random.default_rng(0)
    hubs = np.argsort(np.bincount(F[:, 0], minlength=1 << 20))[-8:]
    sample = np.concatenate([rng.integers(0, 1 << 20, 200), hubs]).astype(np.uint32)
    al, want = oracle.linear3_count_sampled(F, F, F, sample)
    np.testing.assert_array_equal(got[al], want)


def _golden(name):
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", name)))


@pytest.mark.parametrize("tables", ["dense", "hashed"])
def test_linear_powerlaw_full_golden(mj, ctx, tables):
    """Full-size power-law input (2^24 edges, 2^20 vertices): all 2^20 per-A
    counts equal the oracle's, stored by tests/golden/make_linear_golden.py
    (SHA-256 of the whole vector, plus 4096 entries that name a difference),
    with the planner's direct-indexed tables (the benchmarked plan) and with
    the hashed tables."""
    import hashlib
    banner(f"linear power-law full size 2^24 edges against the oracle's vector ({tables})")
    gold = _golden("linear_powerlaw_2e24.json")
    F = G.linear_powerlaw()
    Fd = dev(F)
    A = gold["a_domain"]
    if tables == "dense":
        p = ctx.plan(mj.LINEAR, Fd, Fd, Fd, A)
        assert p.flags & mj.PLAN_DENSE_KEYS
    else:
        p = fixed_plan(mj, ctx, mj.LINEAR, Fd, Fd, Fd, A, log2_nb=10, log2_nc=9, seed=0x2545F491,
                       flags=mj.PLAN_NO_DENSE)
    got = mj.as_u64(ctx.linear3_count(Fd, Fd, Fd, A, plan=p)).astype("<u8")
    sa = np.array(gold["sample_a"])
    np.testing.assert_array_equal(got[sa], np.array(gold["sample_count"], dtype=np.uint64))
    assert int(got.sum(dtype=np.uint64)) == gold["sum"]
    assert hashlib.sha256(got.tobytes()).hexdigest() == gold["sha256_u64_le"]


def test_join2_size(mj, ctx):
    banner("join2 size")
    F = G.linear_powerlaw(seed=3, n_vertices=1 << 14, m=1 << 18)
    Fd = dev(F)
    assert ctx.join2_size(Fd, Fd) == oracle.join2_size(F, F)
    rng = np.random.default_rng(1)
    R = rng.integers(0, 100, size=(5000, 2)).astype(np.uint32)
    S = rng.integers(0, 100, size=(7000, 2)).astype(np.uint32)
    assert ctx.join2_size(dev(R), dev(S)) == oracle.join2_size(R, S)


def test_linear_key_range_rejected(mj, ctx):
    banner("linear key range error")
    F = np.array([[7, 1], [2, 3]], dtype=np.uint32)
    Fd = dev(F)
    with pytest.raises(mj.MJError) as e:
        ctx.plan(mj.LINEAR, Fd, Fd, Fd, 5)
    assert "KEY_RANGE" in str(e.value)


def test_linear_workspace_and_plan_errors(mj, ctx):
    banner("linear workspace / plan mismatch errors")
    import torch
    F = G.linear_small()[:1000]
    Fd = dev(F)
    p = ctx.plan(mj.LINEAR, Fd, Fd, Fd, 4096)
    small = torch.empty(128, dtype=torch.uint8, device="cuda")
    with pytest.raises(mj.MJError) as e:
        ctx.linear3_count(Fd, Fd, Fd, 4096, plan=p, workspace=small)
    assert "WORKSPACE" in str(e.value)
    with pytest.raises(mj.MJError) as e:
        ctx.linear3_count(Fd[:999], Fd, Fd, 4096, plan=p)
    assert "PLAN_MISMATCH" in str(e.value)


@pytest.mark.parametrize("a_domain", [(1 << 25) + 1, 1 << 24, 1, 3])
def test_linear_a_domain_extremes(mj, ctx, a_domain):
    # a_domain above 2^(PART_MAX_BITS + ACELL_MAX_SHIFT) = 2^24 takes the
    # cells' atomic adds; at or below it, the ranges of A; every entry of the
    # output is written either way (it starts as garbage here)
    banner(f"linear a_domain={a_domain}")
    import torch
    rng = np.random.default_rng(a_domain & 0xFFFF)
    n = 20000
    R = np.stack([rng.integers(0, a_domain, size=n), rng.integers(0, 300, size=n)], axis=1).astype(np.uint32)
    R[:5, 0] = a_domain - 1
    S = rng.integers(0, 300, size=(n, 2)).astype(np.uint32)
    T = rng.integers(0, 300, size=(n, 2)).astype(np.uint32)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    out = torch.full((a_domain,), -1, dtype=torch.int64, device="cuda")
    ctx.linear3_count(Rd, Sd, Td, a_domain, out=out)
    got = mj.as_u64(out)
    a_u, want_nz = oracle.linear3_count_sampled(R, S, T, R[:, 0])
    np.testing.assert_array_equal(got[a_u], want_nz)
    untouched = np.ones(a_domain, dtype=bool)
    untouched[a_u] = False
    assert not got[untouched].any()


@pytest.mark.parametrize("seed", range(4))
def test_linear_dense_and_hashed_tables_agree(mj, ctx, seed):
    """Small B and C domains: the planner takes direct-indexed tables; a
    fixed plan asking for the hashed tables gives the same, exact counts."""
    banner(f"linear dense vs hashed tables seed={seed}")
    rng = np.random.default_rng(400 + seed)
    dom_b, dom_c, a_dom = [(3000, 5000, 700), (1, 1, 5), (70000, 100, 4096), (50000, 50000, 1 << 16)][seed]
    n = [20000, 500, 60000, 200000][seed]
    R = np.stack([rng.integers(0, a_dom, n), rng.integers(0, dom_b, n)], 1).astype(np.uint32)
    S = np.stack([rng.integers(0, dom_b, n), rng.integers(0, dom_c, n)], 1).astype(np.uint32)
    T = np.stack([rng.integers(0, dom_c, n), rng.integers(0, 1 << 31, n)], 1).astype(np.uint32)
    R[:7, 1] = dom_b - 1                         # the largest keys in use
    S[:3, 1] = dom_c - 1
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    want = oracle.linear3_count(R, S, T, a_dom)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, a_dom)
    assert p.flags & mj.PLAN_DENSE_KEYS and p.b_domain == dom_b and p.c_domain == dom_c
    np.testing.assert_array_equal(mj.as_u64(ctx.linear3_count(Rd, Sd, Td, a_dom, plan=p)), want)
    h = fixed_plan(mj, ctx, mj.LINEAR, Rd, Sd, Td, a_dom, log2_nb=7, log2_nc=5, seed=9, flags=mj.PLAN_NO_DENSE)
    assert not (h.flags & mj.PLAN_DENSE_KEYS)
    np.testing.assert_array_equal(mj.as_u64(ctx.linear3_count(Rd, Sd, Td, a_dom, plan=h)), want)


def test_linear_sparse_keys_stay_hashed(mj, ctx):
    banner("linear sparse keys: hashed tables")
    rng = np.random.default_rng(8)
    n = 30000
    R = np.stack([rng.integers(0, 1000, n), rng.integers(0, 1 << 31, n)], 1).astype(np.uint32)
    S = np.stack([R[rng.integers(0, n, n), 1], rng.integers(0, 300, n)], 1).astype(np.uint32)
    T = rng.integers(0, 300, size=(n, 2)).astype(np.uint32)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, 1000)
    assert not (p.flags & mj.PLAN_DENSE_KEYS)
    np.testing.assert_array_equal(mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 1000, plan=p)),
                                  oracle.linear3_count(R, S, T, 1000))
    Fd = dev(np.array([[0, 0xFFFFFFFF], [1, 2]], dtype=np.uint32))      # the all-ones key: domain 2^32
    assert not (ctx.plan(mj.LINEAR, Fd, Fd, Fd, 2).flags & mj.PLAN_DENSE_KEYS)


@pytest.mark.parametrize("change", ["S.b", "T.c"])
def test_linear_dense_bound_broken_after_planning(mj, ctx, change):
    banner(f"linear dense plan on changed data: {change}")
    F = G.linear_small()[:20000]
    Rd, Sd, Td = dev(F), dev(F), dev(F)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, 4096)
    assert p.flags & mj.PLAN_DENSE_KEYS
    if change == "S.b":
        Sd[5, 0] = 1 << 20
    else:
        Td[5, 0] = 1 << 20
    got = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 4096, plan=p))
    assert (got == np.uint64(2 ** 64 - 1)).all()


def test_linear_powerlaw_full_hashed_tables(mj, ctx):
    """The full-size input through the hashed tables too (the planner takes
    the direct-indexed ones): the sum equals the closed form and sampled A
    values the oracle's counts."""
    banner("linear power-law full size 2^24 edges, hashed tables")
    F = G.linear_powerlaw()
    Fd = dev(F)
    p = fixed_plan(mj, ctx, mj.LINEAR, Fd, Fd, Fd, 1 << 20, log2_nb=10, log2_nc=9, seed=0x2545F491,
                   flags=mj.PLAN_NO_DENSE)
    got = mj.as_u64(ctx.linear3_count(Fd, Fd, Fd, 1 << 20, plan=p))
    assert int(got.sum(dtype=np.uint64)) == brute.linear_closed_total(F, F, F)
    rng = np.random.default_rng(1)
    sample = rng.integers(0, 1 << 20, 200).astype(np.uint32)
    al, want = oracle.linear3_count_sampled(F, F, F, sample)
    np.testing.assert_array_equal(got[al], want)


def test_linear_dense_shared_partitions(mj, ctx):
    """Direct-indexed tables with partitions shared between relations: R = T
    as one tensor with another S (T's partition is R's), and R = S = T with
    a larger A domain (R's ranges differ; T's partition is S's)."""
    banner("linear dense tables, shared partitions")
    rng = np.random.default_rng(31)
    F = rng.integers(0, 4096, size=(50000, 2)).astype(np.uint32)
    Gs = rng.integers(0, 4096, size=(40000, 2)).astype(np.uint32)
    Fd, Gd = dev(F), dev(Gs)
    p = ctx.plan(mj.LINEAR, Fd, Gd, Fd, 4096)
    assert p.flags & mj.PLAN_DENSE_KEYS
    np.testing.assert_array_equal(mj.as_u64(ctx.linear3_count(Fd, Gd, Fd, 4096, plan=p)),
                                  oracle.linear3_count(F, Gs, F, 4096))
    q = ctx.plan(mj.LINEAR, Fd, Fd, Fd, 1 << 16)
    assert q.flags & mj.PLAN_DENSE_KEYS
    np.testing.assert_array_equal(mj.as_u64(ctx.linear3_count(Fd, Fd, Fd, 1 << 16, plan=q)),
                                  oracle.linear3_count(F, F, F, 1 << 16))


def test_linear_dense_w_at_16_bit_boundary(mj, ctx):
    """Per-B sums W[b] of 65534, 65535 and 65536 around the saturating
    2-byte copy's escape value (65535 is stored as the escape itself, so
    its reader must take the full W), and a few small ones."""
    banner("linear dense tables, W at the 2-byte copy's boundary")
    ws = [65534, 65535, 65536, 1, 700]
    S = np.concatenate([np.stack([np.full(w, b), np.zeros(w)], 1) for b, w in enumerate(ws)]).astype(np.uint32)
    T = np.array([[0, 9]], dtype=np.uint32)                       # deg[0] = 1
    R = np.stack([np.arange(10) % 7, np.arange(10) % len(ws)], 1).astype(np.uint32)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, 7)
    assert p.flags & mj.PLAN_DENSE_KEYS
    got = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 7, plan=p))
    want = oracle.linear3_count(R, S, T, 7)
    assert set(ws[:3]) <= set(int(x) for x in want)               # each boundary value is some a's count
    np.testing.assert_array_equal(got, want)


def test_linear_dense_w_beyond_32_bits(mj, ctx):
    """A per-B sum W[b] of 70000 x 70000 > 2^32: the direct-indexed path
    must read the 8-byte W, not its narrow copy."""
    banner("linear dense tables, W beyond 32 bits")
    n = 70000
    R = np.stack([np.arange(5) % 3, np.zeros(5)], 1).astype(np.uint32)
    S = np.stack([np.zeros(n), np.zeros(n)], 1).astype(np.uint32)
    T = np.stack([np.zeros(n), np.arange(n)], 1).astype(np.uint32)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = ctx.plan(mj.LINEAR, Rd, Sd, Td, 3)
    assert p.flags & mj.PLAN_DENSE_KEYS
    got = mj.as_u64(ctx.linear3_count(Rd, Sd, Td, 3, plan=p))
    want = oracle.linear3_count(R, S, T, 3)
    assert int(want.max()) > 2 ** 32
    np.testing.assert_array_equal(got, want)
