"""Input generators: determinism per seed and the distribution properties
the workloads promise."""
import hashlib

import numpy as np

from workloads import generators as G


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_deterministic_per_seed():
    assert digest(G.linear_small()) == digest(G.linear_small())
    a = G.linear_powerlaw(seed=9, n_vertices=1 << 12, m=1 << 16)
    b = G.linear_powerlaw(seed=9, n_vertices=1 << 12, m=1 << 16)
    c = G.linear_powerlaw(seed=10, n_vertices=1 << 12, m=1 << 16)
    assert digest(a) == digest(b) != digest(c)
    assert digest(G.triangle_rmat(scale=10, seed=1)) == digest(G.triangle_rmat(scale=10, seed=1))


def test_linear_small_shape():
    F = G.linear_small()
    assert F.shape == (65536, 2) and F.dtype == np.uint32
    assert F.min() == 0 and F.max() == 4095


def test_powerlaw_degrees():
    n, m = 1 << 16, 1 << 20
    F = G.linear_powerlaw(seed=2001, n_vertices=n, m=m)
    assert F.shape == (m, 2) and F.dtype == np.int32
    out = np.bincount(F[:, 0], minlength=n)
    assert out.max() == 4096 and out.sum() == m
    deg = np.sort(G.zipf_degrees(n, m, 1.1, 4096))[::-1]
    np.testing.assert_array_equal(np.sort(out)[::-1], deg)
    # preferential attachment: destinations much more skewed than uniform
    inn = np.bincount(F[:, 1], minlength=n)
    assert inn.max() > 50 * (m / n)


def test_rmat_symmetric_simple():
    scale, m = 12, 16 << 12
    E = G.triangle_rmat(scale=scale, m_undirected=m, seed=5)
    assert E.shape == (2 * m, 2)
    assert (E[:, 0] != E[:, 1]).all()
    k = (E[:, 0].astype(np.int64) << 32) | E[:, 1].astype(np.int64)
    assert np.unique(k).size == 2 * m                      # no duplicates
    kr = (E[:, 1].astype(np.int64) << 32) | E[:, 0].astype(np.int64)
    assert np.array_equal(np.sort(k), np.sort(kr))          # symmetric
    assert E.max() < (1 << scale)


def test_batch_mix():
    inst = G.batch_instances(count=8, lo_exp=3, hi_exp=3.5)
    assert [x["kind"] for x in inst] == ["linear"] * 4 + ["triangle"] * 4
    for x in inst:
        assert 10 ** 3 - 1 <= x["m"] <= 10 ** 3.5 + 1
        assert x["n"] == max(64, x["m"] // 16)
