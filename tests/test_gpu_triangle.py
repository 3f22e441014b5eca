"""GPU parity of the cyclic three-way join (Sec. 5) against the oracle:
bit-exact uint64 totals; trace(A^3) = 6 x triangles on simple symmetric
graphs; invariance to the share on A."""
import math

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


def tri(mj, ctx, R, S, T, plan=None):
    out = ctx.triangle3_count(dev(R), dev(S), dev(T), plan=plan)
    return int(mj.as_u64(out)[0])


@pytest.mark.parametrize("seed", range(6))
def test_triangle_random_bags(mj, ctx, seed):
    banner(f"triangle random bags seed={seed}")
    rng = np.random.default_rng(70 + seed)
    dom = [3, 20, 200, 3000, 60000, 7][seed]
    R, S, T = (rng.integers(0, dom, size=(int(rng.integers(1, 30000)), 2)).astype(np.uint32)
               for _ in range(3))
    special = np.array([0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    for X in (R, S, T):
        for col in (0, 1):
            m = rng.random(X.shape[0]) < 0.03
            X[m, col] = special[rng.integers(0, 2, size=m.sum())]
    assert tri(mj, ctx, R, S, T) == oracle.triangle3_count(R, S, T)


@pytest.mark.parametrize("n", [8191, 8192, 8193, 16383, 16384, 16385, 131072, 131073])
def test_triangle_sort_sizes(mj, ctx, n):
    """Relations of n tuples, at the edges of the one-workgroup sort (16384
    keys; 8192 before) and of the one-launch scan (32 tiles of 4096 keys)."""
    banner(f"triangle, relations of {n} tuples")
    rng = np.random.default_rng(n)
    R, S, T = (rng.integers(0, 3000, size=(n, 2)).astype(np.uint32) for _ in range(3))
    assert tri(mj, ctx, R, S, T) == oracle.triangle3_count(R, S, T)


def test_triangle_complete_graph(mj, ctx):
    banner("triangle complete digraph K_300")
    n = 300
    K = np.array([(x, y) for x in range(n) for y in range(n) if x != y], dtype=np.uint32)
    tot = tri(mj, ctx, K, K, K)
    assert tot == n * (n - 1) * (n - 2) and tot // 6 == math.comb(n, 3)


def test_triangle_hubs_and_multiplicity(mj, ctx):
    """Heavy lists (hub keys with thousands of tuples) and duplicates: the
    slicing of R's lists over A and the wave/workgroup split."""
    banner("triangle hubs")
    rng = np.random.default_rng(5)
    n = 60000
    R = np.stack([rng.integers(0, 20000, n), rng.integers(0, 6, n)], 1).astype(np.uint32)
    S = np.stack([rng.integers(0, 6, n), rng.integers(0, 8, n)], 1).astype(np.uint32)
    T = np.stack([rng.integers(0, 8, n), rng.integers(0, 20000, n)], 1).astype(np.uint32)
    want = oracle.triangle3_count(R, S, T)
    assert tri(mj, ctx, R, S, T) == want
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    for share in (0, 3, 5):
        p = fixed_plan(mj, ctx, mj.TRIANGLE, Rd, Sd, Td, log2_share=share, seed=17 + share)
        assert int(mj.as_u64(ctx.triangle3_count(Rd, Sd, Td, plan=p))[0]) == want


def test_triangle_rmat_scale14(mj, ctx):
    banner("triangle R-MAT scale 14")
    E = G.triangle_rmat(scale=14, m_undirected=16 << 14, seed=3001)
    tot = tri(mj, ctx, E, E, E)
    assert tot == brute.triangle_sparse_selfjoin(E)
    assert tot % 6 == 0


def test_triangle_rmat_scale18_share_sweep(mj, ctx):
    banner("triangle R-MAT scale 18, shares 1/2/8/32")
    E = G.triangle_rmat(scale=18, m_undirected=16 << 18, seed=3001)
    want = oracle.triangle3_count(E, E, E)
    Ed = dev(E)
    for share in (0, 1, 3, 5):
        p = fixed_plan(mj, ctx, mj.TRIANGLE, Ed, Ed, Ed, log2_share=share, seed=0x1B873593)
        assert int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0]) == want


def test_triangle_empty_star_cycle(mj, ctx):
    banner("triangle empty / star / C3")
    e = np.zeros((0, 2), dtype=np.uint32)
    star = np.array([(0, i) for i in range(1, 50)] + [(i, 0) for i in range(1, 50)], dtype=np.uint32)
    c3 = np.array([(0, 1), (1, 0), (1, 2), (2, 1), (2, 0), (0, 2)], dtype=np.uint32)
    assert tri(mj, ctx, star, star, star) == 0
    assert tri(mj, ctx, c3, c3, c3) == 6
    assert tri(mj, ctx, e, c3, c3) == 0
    assert tri(mj, ctx, c3, c3, e) == 0


def test_triangle_relabel_invariant(mj, ctx):
    banner("triangle relabel invariance")
    E = G.gnm_symmetric(5000, 80000, seed=12)
    lab = np.random.default_rng(3).permutation(5000).astype(np.int32)
    assert tri(mj, ctx, E, E, E) == tri(mj, ctx, lab[E], lab[E], lab[E]) == \
        oracle.triangle3_count(E, E, E)


def test_triangle_rmat22_full_golden(mj, ctx):
    """Full-size R-MAT scale 22 (2^27 directed tuples) in the plan the
    benchmark uses, against the total the oracle wrote
    (tests/golden/make_triangle_golden.py)."""
    import json
    import os
    banner("triangle R-MAT scale 22 against the stored oracle total")
    path = os.path.join(os.path.dirname(__file__), "golden", "triangle_rmat22.json")
    gold = json.load(open(path))
    E = G.triangle_rmat()
    assert E.shape[0] == gold["directed_tuples"]
    Ed = dev(E)
    p = fixed_plan(mj, ctx, mj.TRIANGLE, Ed, Ed, Ed, log2_share=0, seed=0x1B873593)
    got = int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0])
    assert got == gold["total"] and got % 6 == 0
