"""Pins of the oracle's Flajolet-Martin distinct count of D per A (the
footnotes to Example 1 and to Sec. 4's step list): the exact sets against
brute force, the sketch's union property, the placement of bits, and the
estimator's accuracy against its published bound (standard error about
0.78 / sqrt(m) with m = 16 bitmaps)."""
import itertools

import numpy as np
import pytest

import oracle


def brute_sets(R, S, T):
    out = {}
    for (a, b), (b2, c), (c2, d) in itertools.product(R.tolist(), S.tolist(), T.tolist()):
        if b == b2 and c == c2:
            out.setdefault(a, set()).add(d)
    return out


@pytest.mark.parametrize("seed", range(6))
def test_exact_sets_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    dom = [2, 3, 5, 8, 3, 4][seed]
    R, S, T = (rng.integers(0, dom, size=(int(rng.integers(1, 25)), 2)).astype(np.uint32) for _ in range(3))
    if seed == 4:                                     # the sentinel-like key everywhere
        R[0, 1] = S[0, 0] = 0xFFFFFFFF
        S[0, 1] = T[0, 0] = 0xFFFFFFFF
    want = brute_sets(R, S, T)
    al, sk, est, exact = oracle.linear3_distinct(R, S, T, np.arange(dom), seed=99)
    for i, a in enumerate(al.tolist()):
        ds = want.get(a, set())
        assert exact[i] == len(ds)
        ref, ref_est = oracle.fm_sketch(np.array(sorted(ds), dtype=np.uint32), 99)
        np.testing.assert_array_equal(sk[i], ref)
        assert est[i] == ref_est
        if not ds:
            assert est[i] == 0.0 and not sk[i].any()


def test_union_property_and_duplicates():
    rng = np.random.default_rng(5)
    A = rng.integers(0, 1 << 31, 5000)
    B = rng.integers(0, 1 << 31, 7000)
    sa, _ = oracle.fm_sketch(A, 3)
    sb, _ = oracle.fm_sketch(B, 3)
    su, _ = oracle.fm_sketch(np.concatenate([A, B]), 3)
    np.testing.assert_array_equal(su, sa | sb)
    sd, _ = oracle.fm_sketch(np.concatenate([A, A, A[:100]]), 3)
    np.testing.assert_array_equal(sd, sa)


def test_bit_placement():
    # 2^20 distinct values: every bitmap sees about 2^16 of them, so its low
    # bits are all set (bit r is hit with probability 2^-(r+1)) and bits
    # 24..27 stay clear (bit 28 is the rare h >> 4 == 0 case)
    sk, _ = oracle.fm_sketch(np.arange(1 << 20), 11)
    assert all((int(x) & 0x3FF) == 0x3FF for x in sk)
    assert all(int(x) & 0x0F000000 == 0 for x in sk)
    # the saturating case: a value whose hash is below 16 sets bit 28
    h = oracle.fm_sketch(np.array([0], dtype=np.uint32), 0)[0]      # hash(0 ^ 0) = 0
    assert int(h[0]) == 1 << 28 and not h[1:].any()
    # a single value sets exactly one bit
    one, est1 = oracle.fm_sketch(np.array([12345], dtype=np.uint32), 11)
    assert sum(bin(int(x)).count("1") for x in one) == 1
    assert 0.0 < est1 < 100.0
    empty, est0 = oracle.fm_sketch(np.zeros(0, dtype=np.uint32), 11)
    assert not empty.any() and est0 == 0.0


@pytest.mark.parametrize("n", [20000, 200000])
def test_estimator_accuracy(n):
    ratios = []
    for seed in range(60):
        vals = np.random.default_rng(seed).choice(1 << 31, size=n, replace=False)
        _, est = oracle.fm_sketch(vals, seed + 1)
        ratios.append(est / n)
    r = np.array(ratios)
    assert abs(r.mean() - 1.0) < 0.08           # asymptotically unbiased
    assert 0.12 < r.std() < 0.30                # 0.78 / sqrt(16) = 0.195


def test_hash_against_murmur3_vectors():
    # MurmurHash3_x86_32 of the empty input with seed s is the finaliser
    # applied to s; the published test vectors give 0x514E28B7 for s = 1 and
    # 0x81F16F39 for s = 0xFFFFFFFF.  The value 0 with those seeds hashes to
    # them: bitmap h & 15 (7, then 9), bit = trailing zeros of h >> 4 (0 for both)
    sk, est = oracle.fm_sketch(np.array([0], dtype=np.uint32), 1)
    assert int(sk[7]) == 1 and sk.sum() == 1
    sk, _ = oracle.fm_sketch(np.array([0], dtype=np.uint32), 0xFFFFFFFF)
    assert int(sk[9]) == 1 and sk.sum() == 1
    # one bitmap with lowest zero bit 1, the others 0: 2^(1/16) * 16 / 0.77351
    assert est == pytest.approx(16 / 0.77351 * 2 ** (1 / 16), rel=1e-14)
