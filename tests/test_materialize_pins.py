"""Pins of the oracle's materialised linear join (the join of Sec. 4 with
its result written out instead of aggregated): the sequence of result
tuples (a, b, c, d) in nested-loop order over R, S and T as given.

Against: literal triple loops on tiny bags (which fix the order too), an
independent relational join (pandas merge) as a multiset, the per-A counts
and the closed-form total already pinned for the count, and the agreement
of windows and single positions with the whole sequence."""
import numpy as np
import pytest

import oracle
from tests import brute


def triple_loops(R, S, T):
    out = []
    for a, b in R.tolist():
        for b2, c in S.tolist():
            if b2 != b:
                continue
            for c2, d in T.tolist():
                if c2 == c:
                    out.append((a, b, c, d))
    return np.array(out, dtype=np.uint32).reshape(-1, 4)


def rand_rel(rng, n, dom):
    return rng.integers(0, dom, size=(n, 2)).astype(np.uint32)


@pytest.mark.parametrize("seed", range(8))
def test_sequence_equals_triple_loops(seed):
    rng = np.random.default_rng(seed)
    dom = [2, 3, 4, 6, 8, 3, 5, 2][seed]
    R, S, T = (rand_rel(rng, int(rng.integers(0, 30)), dom) for _ in range(3))
    if seed == 5:                                     # the all-ones key is an ordinary key
        R[:, 1] = np.where(R[:, 1] == 0, 0xFFFFFFFF, R[:, 1])
        S[:, 0] = np.where(S[:, 0] == 0, 0xFFFFFFFF, S[:, 0])
    got, total = oracle.linear3_materialize(R, S, T)
    want = triple_loops(R, S, T)
    assert total == want.shape[0]
    np.testing.assert_array_equal(got, want)


def test_multiset_equals_relational_join():
    import pandas as pd
    rng = np.random.default_rng(11)
    R, S, T = rand_rel(rng, 3000, 60), rand_rel(rng, 2500, 60), rand_rel(rng, 2000, 60)
    got, total = oracle.linear3_materialize(R, S, T)
    j = (pd.DataFrame(R.astype(np.int64), columns=["a", "b"])
         .merge(pd.DataFrame(S.astype(np.int64), columns=["b", "c"]), on="b")
         .merge(pd.DataFrame(T.astype(np.int64), columns=["c", "d"]), on="c"))
    want = j[["a", "b", "c", "d"]].to_numpy()
    assert total == want.shape[0]
    key = lambda x: np.lexsort(x.T[::-1])
    np.testing.assert_array_equal(got[key(got)].astype(np.int64), want[key(want)])


def test_counts_and_closed_form_total():
    rng = np.random.default_rng(3)
    R, S, T = rand_rel(rng, 4000, 200), rand_rel(rng, 4000, 200), rand_rel(rng, 4000, 200)
    got, total = oracle.linear3_materialize(R, S, T)
    assert total == brute.linear_closed_total(R, S, T)
    per_a = np.bincount(got[:, 0], minlength=200).astype(np.uint64)
    np.testing.assert_array_equal(per_a, oracle.linear3_count(R, S, T, 200))
    # every element is a join result: (a, b) in R, (b, c) in S, (c, d) in T
    enc = lambda x, y: (x.astype(np.uint64) << np.uint64(32)) | y.astype(np.uint64)
    assert np.isin(enc(got[:, 0], got[:, 1]), enc(R[:, 0], R[:, 1])).all()
    assert np.isin(enc(got[:, 1], got[:, 2]), enc(S[:, 0], S[:, 1])).all()
    assert np.isin(enc(got[:, 2], got[:, 3]), enc(T[:, 0], T[:, 1])).all()
    # nested-loop order: the blocks of the R tuples come in R's order, each
    # as long as that tuple's count of (s, t) combinations
    deg_t = np.bincount(T[:, 0], minlength=200)
    w_b = np.bincount(S[:, 0], weights=deg_t[S[:, 1]], minlength=200).astype(np.int64)
    ridx = np.repeat(np.arange(R.shape[0]), w_b[R[:, 1]])
    np.testing.assert_array_equal(got[:, :2], R[ridx])


def test_replicated_tuples():
    R = np.array([[1, 2]] * 3, dtype=np.uint32)
    S = np.array([[2, 3]] * 4, dtype=np.uint32)
    T = np.array([[3, 7]] * 5, dtype=np.uint32)
    got, total = oracle.linear3_materialize(R, S, T)
    assert total == 60
    assert (got == np.array([1, 2, 3, 7], dtype=np.uint32)).all()


def test_empty_and_disjoint():
    e = np.zeros((0, 2), dtype=np.uint32)
    F = np.array([[0, 1], [1, 2]], dtype=np.uint32)
    for R, S, T in ((e, F, F), (F, e, F), (F, F, e), (F, F + 10, F)):
        got, total = oracle.linear3_materialize(R, S, T)
        assert total == 0 and got.shape == (0, 4)


def test_windows_and_positions_agree_with_the_sequence():
    rng = np.random.default_rng(7)
    R, S, T = rand_rel(rng, 500, 20), rand_rel(rng, 400, 20), rand_rel(rng, 300, 20)
    full, total = oracle.linear3_materialize(R, S, T)
    assert total > 10000
    for w in (17, 1000, total):
        parts = [oracle.linear3_materialize(R, S, T, lo, w)[0] for lo in range(0, total, w)]
        np.testing.assert_array_equal(np.concatenate(parts), full)
    for lo in list(range(50)) + [total - 1]:                 # single elements
        np.testing.assert_array_equal(oracle.linear3_materialize(R, S, T, lo, 1)[0], full[lo:lo + 1])
    past, t2 = oracle.linear3_materialize(R, S, T, total + 5, 10)
    assert past.shape == (0, 4) and t2 == total
    pos = np.concatenate([np.arange(total), [total, total + 100]])
    at, t3 = oracle.linear3_materialize_at(R, S, T, pos[::-1])
    assert t3 == total
    np.testing.assert_array_equal(at[2:][::-1], full)
    assert (at[:2] == 0xFFFFFFFF).all()
