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


def test_star_schema_shape_and_keys():
    R, S, T = G.star_schema(n_fact=1 << 16, k_r=512, k_t=256, a_domain=100, seed=9)
    R2, S2, T2 = G.star_schema(n_fact=1 << 16, k_r=512, k_t=256, a_domain=100, seed=9)
    assert all(np.array_equal(x, y) for x, y in ((R, R2), (S, S2), (T, T2)))
    assert R.shape == (512, 2) and S.shape == (1 << 16, 2) and T.shape == (256, 2)
    assert np.unique(R[:, 1]).size == 512                       # R's B values are keys
    assert R[:, 0].min() >= 0 and R[:, 0].max() < 100
    assert T[:, 0].min() >= 0 and T[:, 0].max() < 256 and S[:, 1].max() < 256
    hit = np.isin(S[:, 0], R[:, 1]).mean()
    assert abs(hit - 15 / 16) < 0.01                              # fact keys found in R
