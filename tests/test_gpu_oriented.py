"""GPU parity of the degree-oriented cyclic join (each triangle counted once
along edges oriented by degree, total = 6 x triangles) against the oracle's
cyclic join total; the planner's check of its precondition (R = S = T one
symmetric relation without duplicates or loops) and the guard when the data
changed after planning."""
import json
import math
import os

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


def complete(n):
    return np.array([(x, y) for x in range(n) for y in range(n) if x != y], dtype=np.uint32)


def sym(und):
    und = np.asarray(und, dtype=np.uint32)
    return np.concatenate([und, und[:, ::-1]]).astype(np.uint32)


CASES = {
    "rmat14": lambda: G.triangle_rmat(scale=14, m_undirected=16 << 14, seed=3001),
    "gnm": lambda: G.gnm_symmetric(5000, 80000, seed=12),
    "chung_lu": lambda: G.chung_lu_symmetric(20000, 300000, seed=5, cap=4000),
    "complete200": lambda: complete(200),
    "c3": lambda: sym([(0, 1), (1, 2), (2, 0)]),
    "star": lambda: sym([(0, i) for i in range(1, 300)]),
    "high_keys": lambda: sym([(0xFFFFFFFF, 0x80000000), (0x80000000, 7), (7, 0xFFFFFFFF), (7, 9)]),
}


def oriented_plan(mj, ctx, Ed, dense, **fields):
    """A fixed oriented plan; dense=False asks for the sorted degrees."""
    flags = {} if dense else {"flags": mj.PLAN_NO_DENSE}
    return fixed_plan(mj, ctx, mj.TRIANGLE, Ed, Ed, Ed, seed=0x1B873593, algo=mj.ALGO_ORIENTED,
                      **flags, **fields)


@pytest.mark.parametrize("dense", [True, False], ids=["dense_ids", "sorted_degrees"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_oriented_matches_oracle(mj, ctx, case, dense):
    banner(f"oriented cyclic join, {case}, dense={dense}")
    E = CASES[case]()
    Ed = dev(E)
    p = oriented_plan(mj, ctx, Ed, dense)
    assert p.flags & mj.PLAN_SYMMETRIC_SIMPLE and p.algo == mj.ALGO_ORIENTED
    # ids below 2n + 4096 are dense, unless the plan asked for the sort
    small_ids = int(E.max()) + 1 <= 2 * E.shape[0] + 4096
    assert bool(p.flags & mj.PLAN_DENSE_KEYS) == (dense and small_ids)
    if p.flags & mj.PLAN_DENSE_KEYS:
        assert p.b_domain == int(E.max()) + 1
    got = int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0])
    assert got == oracle.triangle3_count(E, E, E)
    assert got % 6 == 0


def test_oriented_dense_ids_with_gaps(mj, ctx):
    """Dense ids with most of the domain unused (degree 0): ids spread over
    [0, 2n) for a graph of n tuples."""
    banner("oriented cyclic join, dense ids with gaps")
    E = G.gnm_symmetric(3000, 20000, seed=21).astype(np.uint64)
    E = (E * 13 + 5).astype(np.uint32)                 # ids up to about 39,000 for 40,000 tuples
    Ed = dev(E)
    p = oriented_plan(mj, ctx, Ed, True)
    assert p.flags & mj.PLAN_DENSE_KEYS
    assert int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0]) == oracle.triangle3_count(E, E, E)


def test_oriented_complete_graph_closed_form(mj, ctx):
    banner("oriented cyclic join, complete graph K_300")
    n = 300
    Ed = dev(complete(n))
    p = fixed_plan(mj, ctx, mj.TRIANGLE, Ed, Ed, Ed, seed=0x1B873593, algo=mj.ALGO_ORIENTED)
    got = int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0])
    assert got == 6 * math.comb(n, 3)


def test_oriented_share_sweep_rmat18(mj, ctx):
    banner("oriented cyclic join, R-MAT scale 18, shares 1/2/8/32")
    E = G.triangle_rmat(scale=18, m_undirected=16 << 18, seed=3001)
    want = oracle.triangle3_count(E, E, E)
    Ed = dev(E)
    for share in (0, 1, 3, 5):
        p = fixed_plan(mj, ctx, mj.TRIANGLE, Ed, Ed, Ed, log2_share=share, seed=0x1B873593,
                       algo=mj.ALGO_ORIENTED)
        assert p.algo == mj.ALGO_ORIENTED
        assert int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0]) == want


def test_planner_rule(mj, ctx):
    """The planner offers the oriented join only to large skewed relations:
    an R-MAT graph of 2^16 vertices (2^21 tuples) is oriented; a G(n, m)
    graph of the same size (few wedges per edge) and a small R-MAT graph
    are not."""
    banner("oriented join: the planner's rule")
    for E, want in ((G.triangle_rmat(scale=16, m_undirected=16 << 16, seed=3001), True),
                    (G.gnm_symmetric(1 << 16, 1 << 20, seed=4), False),
                    (G.triangle_rmat(scale=9, m_undirected=16 << 9, seed=3001), False)):
        Ed = dev(E)
        p = ctx.plan(mj.TRIANGLE, Ed, Ed, Ed)
        assert p.flags & mj.PLAN_SYMMETRIC_SIMPLE
        assert (p.algo == mj.ALGO_ORIENTED) == want, (E.shape, p.join2_size)
        assert int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0]) == oracle.triangle3_count(E, E, E)


def not_eligible_cases():
    rng = np.random.default_rng(4)
    base = G.gnm_symmetric(2000, 20000, seed=7).astype(np.uint32)
    directed = np.unique(rng.integers(0, 3000, size=(30000, 2)).astype(np.uint32), axis=0)
    directed = directed[directed[:, 0] != directed[:, 1]]
    dup = np.concatenate([base, base[:1], base[:1, ::-1]])          # symmetric, one pair twice
    loop = np.concatenate([base, [[5, 5]]]).astype(np.uint32)       # symmetric, one loop
    return {"directed": directed, "duplicate": dup, "loop": loop}


@pytest.mark.parametrize("case", ["directed", "duplicate", "loop"])
def test_not_eligible_keeps_general_join(mj, ctx, case):
    banner(f"oriented join not offered: {case}")
    E = not_eligible_cases()[case]
    Ed = dev(E)
    p = ctx.plan(mj.TRIANGLE, Ed, Ed, Ed)
    assert not (p.flags & mj.PLAN_SYMMETRIC_SIMPLE) and p.algo != mj.ALGO_ORIENTED
    assert int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0]) == oracle.triangle3_count(E, E, E)
    with pytest.raises(mj.MJError) as e:
        fixed_plan(mj, ctx, mj.TRIANGLE, Ed, Ed, Ed, algo=mj.ALGO_ORIENTED)
    assert "UNSUPPORTED" in str(e.value)


def test_unaliased_copies_not_checked(mj, ctx):
    banner("oriented join needs R, S, T to be one relation")
    E = G.gnm_symmetric(2000, 20000, seed=8)
    R, S, T = dev(E), dev(E), dev(E)
    p = ctx.plan(mj.TRIANGLE, R, S, T)
    assert not (p.flags & mj.PLAN_SYMMETRIC_SIMPLE) and p.algo != mj.ALGO_ORIENTED
    assert int(mj.as_u64(ctx.triangle3_count(R, S, T, plan=p))[0]) == oracle.triangle3_count(E, E, E)


@pytest.mark.parametrize("dense", [True, False], ids=["dense_ids", "sorted_degrees"])
@pytest.mark.parametrize("change", ["loop", "unknown_end", "id_above_domain"])
def test_data_changed_after_planning(mj, ctx, change, dense):
    banner(f"oriented plan on changed data: {change}, dense={dense}")
    E = G.gnm_symmetric(2000, 20000, seed=9)
    Ed = dev(E)
    p = oriented_plan(mj, ctx, Ed, dense)
    assert p.algo == mj.ALGO_ORIENTED and bool(p.flags & mj.PLAN_DENSE_KEYS) == dense
    if change == "loop":
        Ed[0, 1] = Ed[0, 0]
    elif change == "unknown_end":
        Ed[0, 1] = 1_000_000_000                  # a vertex with no edges of its own
    else:
        # both directions of one edge move to a new id above the planned
        # domain: still symmetric and simple, but outside the dense array
        u, v = E[0]
        j = int(np.nonzero((E[:, 0] == v) & (E[:, 1] == u))[0][0])
        Ed[0, 1] = 5000
        Ed[j, 0] = 5000
    got = int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0])
    if change == "id_above_domain" and not dense:
        # the sorted degrees are not bound to a domain: the new edge is valid
        Eh = Ed.cpu().numpy().view(np.uint32)
        assert got == oracle.triangle3_count(Eh, Eh, Eh)
    else:
        assert got == 2 ** 64 - 1


def test_oriented_rmat22_full_golden(mj, ctx):
    """Full-size R-MAT scale 22 (2^27 directed tuples): the planner finds the
    relation symmetric and simple and picks the oriented join; its total
    equals the stored oracle total."""
    banner("oriented cyclic join, R-MAT scale 22 against the stored oracle total")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "triangle_rmat22.json")))
    E = G.triangle_rmat()
    Ed = dev(E)
    p = ctx.plan(mj.TRIANGLE, Ed, Ed, Ed)
    assert p.algo == mj.ALGO_ORIENTED and p.flags & mj.PLAN_DENSE_KEYS
    got = int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=p))[0])
    assert got == gold["total"]
    # the same plan with the degrees from the sort
    q = oriented_plan(mj, ctx, Ed, False)
    assert not (q.flags & mj.PLAN_DENSE_KEYS)
    assert int(mj.as_u64(ctx.triangle3_count(Ed, Ed, Ed, plan=q))[0]) == gold["total"]
