"""GPU parity of the Flajolet-Martin distinct count of D per A (the
footnotes to Example 1 and to Sec. 4's step list) against the oracle: the
sketches bit for bit, the estimates exactly (both sides take the same
sequence of double operations from the same bits)."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, dev
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


def run_fm(ctx, R, S, T, a_domain, seed):
    sk, est = ctx.linear3_distinct(dev(R), dev(S), dev(T), a_domain, seed=seed)
    return sk.cpu().numpy().view(np.uint32), est.cpu().numpy()


def check(ctx, R, S, T, a_domain, seed, alist=None):
    sk, est = run_fm(ctx, R, S, T, a_domain, seed)
    al = np.arange(a_domain, dtype=np.uint32) if alist is None else np.asarray(alist, dtype=np.uint32)
    a_u, want_sk, want_est, _ = oracle.linear3_distinct(R, S, T, al, seed)
    np.testing.assert_array_equal(sk[a_u], want_sk)
    np.testing.assert_array_equal(est[a_u], want_est)
    return sk, est


def test_fm_linear_small_all_a(mj, ctx):
    banner("FM distinct count, linear small (65,536 tuples), every A")
    F = G.linear_small()
    check(ctx, F, F, F, 4096, seed=0x1234)


@pytest.mark.parametrize("seed", range(5))
def test_fm_random_bags_and_special_keys(mj, ctx, seed):
    banner(f"FM random bags seed={seed}")
    rng = np.random.default_rng(300 + seed)
    dom = [3, 40, 900, 70000, 6][seed]
    a_domain = int(rng.integers(1, 3000))
    nr, ns, nt = (int(x) for x in rng.integers(1, 20000, size=3))
    R = np.stack([rng.integers(0, a_domain, nr), rng.integers(0, dom, nr)], axis=1).astype(np.uint32)
    S = rng.integers(0, dom, size=(ns, 2)).astype(np.uint32)
    T = rng.integers(0, dom, size=(nt, 2)).astype(np.uint32)
    sp = np.array([0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    R[: min(5, nr), 1] = sp[0]
    S[: min(20, ns), 0] = sp[rng.integers(0, 2, min(20, ns))]
    S[: min(20, ns), 1] = sp[rng.integers(0, 2, min(20, ns))]
    T[: min(20, nt), 0] = sp[rng.integers(0, 2, min(20, nt))]
    T[: min(20, nt), 1] = sp[rng.integers(0, 2, min(20, nt))]
    check(ctx, R, S, T, a_domain, seed=seed * 7919)


@pytest.mark.parametrize("a_domain", [1, (1 << 22) + 5, (1 << 23) + 1])
def test_fm_a_domain_extremes(mj, ctx, a_domain):
    # ranges of A in LDS up to 2^22 values (2^12 ranges of 2^10), the output
    # ORed in place beyond that; every entry written either way
    banner(f"FM a_domain={a_domain}")
    rng = np.random.default_rng(a_domain & 0xFFFF)
    n = 30000
    R = np.stack([rng.integers(0, a_domain, n), rng.integers(0, 500, n)], axis=1).astype(np.uint32)
    R[:3, 0] = a_domain - 1
    S = rng.integers(0, 500, size=(n, 2)).astype(np.uint32)
    T = rng.integers(0, 1 << 20, size=(n, 2)).astype(np.uint32)
    T[:, 0] %= 500
    sk, est = check(ctx, R, S, T, a_domain, seed=5, alist=np.unique(R[:, 0]))
    untouched = np.ones(a_domain, dtype=bool)
    untouched[R[:, 0]] = False
    assert not sk[untouched].any() and not est[untouched].any()


def test_fm_empty_inputs(mj, ctx):
    banner("FM empty inputs")
    one = np.array([[1, 2]], dtype=np.uint32)
    empty = np.zeros((0, 2), dtype=np.uint32)
    for R, S, T in ((empty, one, one), (one, empty, one), (one, one, empty)):
        sk, est = run_fm(ctx, R, S, T, 8, seed=1)
        assert not sk.any() and not est.any()


def test_fm_powerlaw_full_sampled(mj, ctx):
    """The benchmarked friends graph (2^24 edges, 2^20 vertices): sketches
    and estimates of sampled people (and the 8 with most friends) against
    the oracle, and the estimates within the sketch's error of the exact
    counts."""
    banner("FM power-law full size, sampled A values")
    F = G.linear_powerlaw()
    sk, est = run_fm(ctx, F, F, F, 1 << 20, seed=0x5EED)
    rng = np.random.default_rng(1)
    hubs = np.argsort(np.bincount(F[:, 0], minlength=1 << 20))[-8:]
    sample = np.concatenate([rng.integers(0, 1 << 20, 150), hubs]).astype(np.uint32)
    a_u, want_sk, want_est, exact = oracle.linear3_distinct(F, F, F, sample, 0x5EED)
    np.testing.assert_array_equal(sk[a_u], want_sk)
    np.testing.assert_array_equal(est[a_u], want_est)
    big = exact >= 1000                    # the sketch's error is about 0.78 / sqrt(16)
    rel = est[a_u][big] / exact[big]
    assert big.sum() >= 20 and abs(np.median(rel) - 1.0) < 0.15
