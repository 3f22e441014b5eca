"""Pins for the CPU oracle: it is checked against literal triple loops,
closed forms, special cases with known answers, expectations under uniform
keys and invariances -- never against itself."""
import itertools
import math

import numpy as np
import pytest

import oracle
from tests import brute
from workloads import generators as G


def rand_bag(rng, n, dom, dtype=np.uint32):
    return rng.integers(0, dom, size=(n, 2)).astype(dtype)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(12))
def test_linear_vs_triple_loop(seed):
    rng = np.random.default_rng(seed)
    dom = [1, 2, 3, 5, 8][seed % 5]
    R, S, T = (rand_bag(rng, rng.integers(0, 48), dom) for _ in range(3))
    got = oracle.linear3_count(R, S, T, dom)
    np.testing.assert_array_equal(got, brute.linear_bruteforce(R, S, T, dom))


@pytest.mark.parametrize("seed", range(12))
def test_triangle_vs_triple_loop(seed):
    rng = np.random.default_rng(100 + seed)
    dom = [1, 2, 3, 5, 8][seed % 5]
    R, S, T = (rand_bag(rng, rng.integers(0, 48), dom) for _ in range(3))
    assert oracle.triangle3_count(R, S, T) == brute.triangle_bruteforce(R, S, T)


@pytest.mark.parametrize("seed", range(8))
def test_join2_vs_double_loop(seed):
    rng = np.random.default_rng(200 + seed)
    dom = [1, 3, 8, 16][seed % 4]
    R, S = rand_bag(rng, 60, dom), rand_bag(rng, 50, dom)
    assert oracle.join2_size(R, S) == brute.join2_bruteforce(R, S)


def test_high_bit_keys_are_plain_patterns():
    # keys with the sign bit set and the all-ones pattern are ordinary keys
    vals = np.array([0xFFFFFFFF, 0x80000000, 0x7FFFFFFF, 0], dtype=np.uint32)
    rng = np.random.default_rng(7)
    mk = lambda n: vals[rng.integers(0, 4, size=(n, 2))]
    R, S, T = mk(30), mk(30), mk(30)
    assert oracle.triangle3_count(R, S, T) == brute.triangle_bruteforce(R, S, T)
    R2 = R.copy()
    R2[:, 0] = rng.integers(0, 4, size=30)
    np.testing.assert_array_equal(oracle.linear3_count(R2, S, T, 4),
                                  brute.linear_bruteforce(R2, S, T, 4))


# ---------------------------------------------------------------- closed forms
def test_linear_small_closed_forms():
    F = G.linear_small()
    cnt = oracle.linear3_count(F, F, F, 4096)
    np.testing.assert_array_equal(cnt, brute.linear_closed_per_a(F, F, F, 4096))
    assert int(cnt.sum(dtype=np.uint64)) == brute.linear_closed_total(F, F, F)


def test_linear_powerlaw_scaled_closed_forms():
    F = G.linear_powerlaw(seed=2001, n_vertices=1 << 14, m=1 << 18)
    a_dom = 1 << 14
    cnt = oracle.linear3_count(F, F, F, a_dom)
    np.testing.assert_array_equal(cnt, brute.linear_closed_per_a(F, F, F, a_dom))
    assert int(cnt.sum(dtype=np.uint64)) == brute.linear_closed_total(F, F, F)


def test_linear_distinct_relations_closed_form():
    rng = np.random.default_rng(11)
    R = rand_bag(rng, 5000, 300)
    S = rand_bag(rng, 7000, 300)
    T = rand_bag(rng, 6000, 300)
    cnt = oracle.linear3_count(R, S, T, 300)
    np.testing.assert_array_equal(cnt, brute.linear_closed_per_a(R, S, T, 300))


def test_join2_closed_form():
    F = G.linear_powerlaw(seed=5, n_vertices=1 << 12, m=1 << 16)
    assert oracle.join2_size(F, F) == brute.join2_closed(F, F)


@pytest.mark.parametrize("seed", range(3))
def test_triangle_trace_dense(seed):
    rng = np.random.default_rng(300 + seed)
    n = [40, 200, 1000][seed]
    R, S, T = (rand_bag(rng, 4 * n, n) for _ in range(3))
    assert oracle.triangle3_count(R, S, T) == brute.triangle_trace(R, S, T)


def test_triangle_rmat_scale14_sparse_trace():
    E = G.triangle_rmat(scale=14, m_undirected=16 << 14, seed=3001)
    tot = oracle.triangle3_count(E, E, E)
    assert tot == brute.triangle_sparse_selfjoin(E)
    assert tot % 6 == 0


# ---------------------------------------------------------------- special cases
@pytest.mark.parametrize("n", [2, 3, 7, 20])
def test_complete_digraph(n):
    K = np.array([(x, y) for x in range(n) for y in range(n) if x != y], dtype=np.uint32)
    np.testing.assert_array_equal(oracle.linear3_count(K, K, K, n),
                                  np.full(n, (n - 1) ** 3, dtype=np.uint64))
    tot = oracle.triangle3_count(K, K, K)
    assert tot == n * (n - 1) * (n - 2)               # ordered triples
    assert tot // 6 == math.comb(n, 3)


def test_star_and_cycle():
    star = np.array([(0, i) for i in range(1, 50)] + [(i, 0) for i in range(1, 50)], dtype=np.uint32)
    assert oracle.triangle3_count(star, star, star) == 0
    c3 = np.array([(0, 1), (1, 0), (1, 2), (2, 1), (2, 0), (0, 2)], dtype=np.uint32)
    assert oracle.triangle3_count(c3, c3, c3) == 6


def test_replicated_tuples_multiply():
    k, l, m = 3, 5, 7
    R = np.array([(1, 2)] * k, dtype=np.uint32)
    S = np.array([(2, 3)] * l, dtype=np.uint32)
    T = np.array([(3, 4)] * m, dtype=np.uint32)
    out = oracle.linear3_count(R, S, T, 4)
    np.testing.assert_array_equal(out, np.array([0, k * l * m, 0, 0], dtype=np.uint64))
    T2 = np.array([(3, 1)] * m, dtype=np.uint32)
    assert oracle.triangle3_count(R, S, T2) == k * l * m


def test_empty_and_disjoint():
    e = np.zeros((0, 2), dtype=np.uint32)
    F = G.linear_small()[:1000]
    assert not oracle.linear3_count(e, F, F, 4096).any()
    assert not oracle.linear3_count(F, e, F, 4096).any()
    assert not oracle.linear3_count(F, F, e, 4096).any()
    assert oracle.triangle3_count(e, F, F) == 0
    assert oracle.triangle3_count(F, F, e) == 0
    G2 = F + np.uint32(5000)                          # disjoint key range
    assert not oracle.linear3_count(F, G2, F, 4096).any()
    assert oracle.triangle3_count(F, G2, F) == 0


def test_key_range_error():
    F = np.array([(5, 1)], dtype=np.uint32)
    with pytest.raises(oracle.OracleError):
        oracle.linear3_count(F, F, F, 5)


# ------------------------------------------------- expectations, uniform keys
def test_uniform_expectations():
    """Uniform keys over d values: E|I| = |R||S|/d (Sec. 6.3) and
    E[total] = |F|^3/d^2; the drawn instance is within a few sigma."""
    F = G.linear_small()
    n, d = F.shape[0], 4096
    I = oracle.join2_size(F, F)
    assert abs(I - n * n / d) < 5 * math.sqrt(n * n / d) * 2
    tot = int(oracle.linear3_count(F, F, F, d).sum(dtype=np.uint64))
    expect = n ** 3 / d ** 2
    assert abs(tot - expect) / expect < 0.02


# ---------------------------------------------------------------- invariants
def test_invariant_to_order_and_relabel():
    rng = np.random.default_rng(21)
    E = G.gnm_symmetric(300, 3000, seed=9)
    tot = oracle.triangle3_count(E, E, E)
    perm = rng.permutation(E.shape[0])
    assert oracle.triangle3_count(E[perm], E[rng.permutation(E.shape[0])], E) == tot
    lab = rng.permutation(300).astype(np.int32)
    E2 = lab[E]
    assert oracle.triangle3_count(E2, E2, E2) == tot
    cnt = oracle.linear3_count(E, E, E, 300)
    cnt2 = oracle.linear3_count(E2, E2, E2, 300)
    np.testing.assert_array_equal(cnt2[lab], cnt)


def test_sampled_linear_matches_full():
    F = G.linear_powerlaw(seed=7, n_vertices=1 << 12, m=1 << 16)
    full = oracle.linear3_count(F, F, F, 1 << 12)
    al, part = oracle.linear3_count_sampled(F, F, F, np.array([5, 77, 3, 4000, 77], np.uint32))
    np.testing.assert_array_equal(part, full[al])


def test_masked_triangle_is_additive():
    E = G.gnm_symmetric(500, 6000, seed=3)
    rng = np.random.default_rng(1)
    m = rng.integers(0, 2, size=E.shape[0]).astype(np.uint8)
    tot = oracle.triangle3_count(E, E, E)
    assert oracle.triangle3_count(E, E, E, smask=m) + \
        oracle.triangle3_count(E, E, E, smask=1 - m) == tot
