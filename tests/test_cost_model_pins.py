"""Pins for the analytic cost formulas: the paper's worked examples and
closed-form optima checked against brute-force minimisation."""
import math

import numpy as np
import pytest

from oracle import cost_model as cm


def test_example3_linear_threshold():
    # Example 3: F = 6e11 tuples, the binary join of F with itself ~1.8e14;
    # the 3-way join reads fewer tuples iff M > 1.003e9.
    F, I = 6e11, 1.8e14
    M = cm.linear_threshold(F, F, F, I)
    assert M == pytest.approx(1.0033e9, rel=2e-4)
    assert f"{M:.3e}" == "1.003e+09"
    assert cm.linear_tuples_read(F, F, F, M * 1.001) < cm.cascade_tuples_moved(I)
    assert cm.linear_tuples_read(F, F, F, M * 0.999) > cm.cascade_tuples_moved(I)


def test_example3_footnote_half_the_nodes():
    # Example 3's footnote: the break-even M is close to half the number of
    # nodes, whatever the mean degree; for ~300 million users ~150 million.
    for n in (3e8, 2e9):
        for f in (50.0, 300.0, 1000.0):
            F = n * f
            I = F * F / n
            M = cm.linear_threshold(F, F, F, I)
            assert M == pytest.approx(n / 2, rel=1.0 / (f - 1) + 1e-12)
    M_tw = cm.linear_threshold(9e10, 9e10, 9e10, 9e10 ** 2 / 3e8)
    assert 1.45e8 < M_tw < 1.55e8


def test_example4_cyclic_threshold_both_readings():
    F, budget = 6e11, 1.8e14
    printed = cm.cyclic_example_threshold_printed(F, budget)
    assert printed == pytest.approx(6.71e6, rel=1e-3)        # "seven million"
    derived = cm.cyclic_threshold(F, F, F, budget)
    assert derived == pytest.approx(2.6845e7, rel=1e-4)
    assert cm.cyclic_min_tuples_read(F, F, F, derived * 1.0001) < budget
    assert cm.cyclic_min_tuples_read(F, F, F, derived * 0.9999) > budget


@pytest.mark.parametrize("R,S,T,M", [(1e6, 2e6, 3e6, 1e4), (5e8, 5e8, 5e8, 2e6),
                                     (1e7, 1e9, 1e8, 1e5)])
def test_cyclic_optimum_vs_bruteforce(R, S, T, M):
    H_star = cm.cyclic_optimal_H(R, S, T, M)
    Hs = np.exp(np.linspace(math.log(H_star) - 5, math.log(H_star) + 5, 200001))
    costs = R + Hs * S + R * T / (M * Hs)
    assert Hs[np.argmin(costs)] == pytest.approx(H_star, rel=1e-3)
    assert cm.cyclic_tuples_read(R, S, T, M, H_star) == pytest.approx(
        cm.cyclic_min_tuples_read(R, S, T, M), rel=1e-12)
    assert costs.min() >= cm.cyclic_min_tuples_read(R, S, T, M) * (1 - 1e-12)


def test_cyclic_smallest_relation_first():
    # Sec. 5.2: only the |R| term is not symmetric, so R should be smallest
    a, b, c, M = 1e6, 3e6, 9e6, 1e4
    costs = {p: cm.cyclic_min_tuples_read(*p, M) for p in [(a, b, c), (b, a, c), (c, b, a)]}
    assert min(costs, key=costs.get)[0] == a


def test_linear_symmetric_in_R_T_except_first_term():
    assert cm.linear_tuples_read(1e6, 2e6, 3e6, 1e4) - 1e6 == \
        cm.linear_tuples_read(3e6, 2e6, 1e6, 1e4) - 3e6


def test_branch_probability_simulation():
    # App. A: with g3 buckets on C, of the |S||T|/g3 same-bucket pairs a
    # fraction g3/d have equal keys.
    rng = np.random.default_rng(0)
    d, g3 = 64, 8
    s = rng.integers(0, d, 4000)
    t = rng.integers(0, d, 4000)
    bucket = lambda k: k % g3
    same = bucket(s)[:, None] == bucket(t)[None, :]
    equal = s[:, None] == t[None, :]
    frac = equal.sum() / same.sum()
    assert frac == pytest.approx(cm.branch_hit_probability(g3, d), rel=0.03)
    assert cm.comparisons_3way_ST(4000, 4000, 2, 16, g3) == pytest.approx(4000 * 4000 / g3)
    assert same.sum() == pytest.approx(4000 * 4000 / g3, rel=0.03)


def test_uniform_join_size_estimate():
    rng = np.random.default_rng(2)
    d = 1000
    R = rng.integers(0, d, 20000)
    S = rng.integers(0, d, 30000)
    I = (np.bincount(R, minlength=d) * np.bincount(S, minlength=d)).sum()
    assert I == pytest.approx(cm.join2_size_uniform(20000, 30000, d), rel=0.02)


def test_star_footnote_terms():
    R, S, T, d, h, g = 1e4, 1e7, 1e4, 1e3, 64, 64
    I = cm.join2_size_uniform(R, S, d)
    assert cm.star_cascade_comparisons(R, S, T, d, h, g) == pytest.approx(
        R * S / h + cm.cascade_join2_comparisons(I, T, g))


def _simulated_hash_join(probe_keys, build_keys, nbuckets, bucket_of):
    """A literal bucketed hash join, counted: every tuple is loaded once into
    its bucket, every pair of one bucket is compared, equal keys match.
    Returns (tuples loaded, comparisons, matches)."""
    pb, bb = bucket_of[probe_keys], bucket_of[build_keys]
    loaded = comparisons = matches = 0
    for q in range(nbuckets):
        p, b = probe_keys[pb == q], build_keys[bb == q]
        loaded += p.size + b.size
        comparisons += p.size * b.size
        matches += int((p[:, None] == b[None, :]).sum())
    return loaded, comparisons, matches


def test_cascade_second_join_counts_simulated():
    # Sec. 6.3: the second join loads |R join S| + |T| tuples; with g buckets
    # on C it makes |I||T|/g comparisons, of which |I||T|/d match (App. A's
    # hit probability g/d).  Counted on a materialised I under uniform keys.
    import oracle
    rng = np.random.default_rng(5)
    d, g = 320, 16
    R = rng.integers(0, d, size=(3000, 2)).astype(np.uint32)
    S = rng.integers(0, d, size=(3000, 2)).astype(np.uint32)
    T = rng.integers(0, d, size=(4000, 2)).astype(np.uint32)
    # I = R join S on B, as (a, c) pairs
    by_b = {}
    for b, c in S:
        by_b.setdefault(int(b), []).append(int(c))
    I_c = np.array([c for a, b in R for c in by_b.get(int(b), [])], dtype=np.int64)
    bucket_of = np.arange(d) % g                     # a radix digit of C: balanced buckets
    loaded, comparisons, matches = _simulated_hash_join(I_c, T[:, 0].astype(np.int64), g, bucket_of)
    assert loaded == cm.cascade_join2_loaded(I_c.size, T.shape[0])
    assert comparisons == pytest.approx(cm.cascade_join2_comparisons(I_c.size, T.shape[0], g), rel=0.05)
    assert matches == pytest.approx(cm.cascade_join2_matches(I_c.size, T.shape[0], d), rel=0.05)
    # the matches are the three-way join's result tuples
    assert matches == int(oracle.linear3_count(R, S, T, d).sum())


def test_star_cascade_comparisons_simulated():
    # Sec. 6.5's footnote: the binary cascade of the star join compares
    # |R||S|/h pairs in its first join (h buckets on B) and |R||S||T|/(dg)
    # in its second (g buckets on C, |I| = |R||S|/d), counted here.
    rng = np.random.default_rng(8)
    d, h, g = 384, 32, 32
    R = rng.integers(0, d, size=(2000, 2)).astype(np.int64)      # (a, b)
    S = rng.integers(0, d, size=(40000, 2)).astype(np.int64)     # (b, c)
    T = rng.integers(0, d, size=(2000, 2)).astype(np.int64)      # (c, d)
    hb = np.arange(d) % h                            # radix digits: balanced buckets
    hc = (np.arange(d) // 3) % g
    _, cmp1, m1 = _simulated_hash_join(S[:, 0], R[:, 1], h, hb)
    # I = R join S as the C value of each match
    deg_r = np.bincount(R[:, 1], minlength=d)
    I_c = np.repeat(S[:, 1], deg_r[S[:, 0]])
    assert I_c.size == m1
    _, cmp2, _ = _simulated_hash_join(I_c, T[:, 0], g, hc)
    want = cm.star_cascade_comparisons(R.shape[0], S.shape[0], T.shape[0], d, h, g)
    assert cmp1 + cmp2 == pytest.approx(want, rel=0.05)
    # each term on its own
    assert cmp1 == pytest.approx(R.shape[0] * S.shape[0] / h, rel=0.05)
    assert cmp2 == pytest.approx(R.shape[0] * S.shape[0] * T.shape[0] / (d * g), rel=0.08)
