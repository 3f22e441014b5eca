"""Seeded synthetic join inputs.

This module only draws inputs; it holds none of the join arithmetic and is
shared by the oracle tests, the GPU tests and the benchmark.  Every function
is deterministic for a given seed (numpy's PCG64 via ``default_rng``).

Relations are returned as ``[n, 2]`` arrays (column 0, column 1), uint32 for
the uniform small workload and int32 for the graph workloads.  Keys are
compared by their 32-bit pattern everywhere, so the dtype only matters for
how a value prints.

Workloads (the paper's experiments use synthetic relations of N records and
d distinct values, Sec. 6; its motivating queries are friends-of-friends and
triangles over a social graph, Examples 1 and 2):

* ``uniform_pairs``      -- both columns i.i.d. uniform, duplicates kept.
* ``powerlaw_friends``   -- out-degrees rank-Zipf(s) capped, destinations by
                            a copy-model preferential attachment.
* ``rmat_symmetric``     -- R-MAT edges, canonicalised, loops and duplicates
                            removed, exactly ``m`` undirected edges, seeded
                            relabel, symmetrised into ``2m`` directed tuples.
* ``gnm_symmetric`` / ``chung_lu_symmetric`` -- small triangle inputs.
* ``batch_instances``    -- the mixed batch of many small joins.
"""
from __future__ import annotations

import numpy as np

U64 = np.uint64
_MASK64 = (1 << 64) - 1


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(int(seed))


# ----------------------------------------------------------------------------
# Uniform pairs
# ----------------------------------------------------------------------------
def uniform_pairs(n: int, domain: int, seed: int, dtype=np.uint32) -> np.ndarray:
    """``n`` tuples, both columns uniform in ``[0, domain)``, duplicates kept."""
    g = _rng(seed)
    out = g.integers(0, domain, size=(n, 2), dtype=np.int64)
    return np.ascontiguousarray(out.astype(dtype))


# ----------------------------------------------------------------------------
# Power-law "friends" graph
# ----------------------------------------------------------------------------
def zipf_degrees(n: int, m: int, s: float, cap: int) -> np.ndarray:
    """Integer out-degrees k_r = min(cap, lam * r^-s) for ranks r = 1..n with
    sum exactly m.  ``lam`` is found by bisection on the real-valued sum, the
    result is integerised by largest remainder."""
    r = np.arange(1, n + 1, dtype=np.float64)
    base = r ** (-s)
    if cap * n < m:
        raise ValueError("cap * n < m: no degree sequence exists")

    def total(lam):
        return np.minimum(cap, lam * base).sum()

    lo, hi = 0.0, 1.0
    while total(hi) < m:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < m:
            lo = mid
        else:
            hi = mid
    k = np.minimum(cap, hi * base)
    fl = np.floor(k)
    rem = int(m - fl.sum())
    frac = k - fl
    # ranks with the largest fractional parts get one more (stable order)
    order = np.argsort(-frac, kind="stable")
    add = np.zeros(n, dtype=np.int64)
    if rem > 0:
        cand = order[fl[order] < cap]
        add[cand[:rem]] = 1
    deg = fl.astype(np.int64) + add
    assert int(deg.sum()) == m, (int(deg.sum()), m)
    assert int(deg.max()) <= cap
    return deg


def powerlaw_friends(n: int, m: int, seed: int, s: float = 1.1,
                     cap: int = 4096, dtype=np.int32) -> np.ndarray:
    """Directed edges (src, dst) over ``n`` vertices.

    Out-degrees follow a capped rank-Zipf law; ranks are mapped to vertex
    ids by a seeded permutation and the sources are shuffled.  Destinations
    follow a copy model of preferential attachment: edge 0 picks a uniform
    vertex; edge e picks a uniform vertex with probability 1/2, else copies
    the destination of a uniformly chosen earlier edge.  Loops and duplicate
    edges are kept."""
    g = _rng(seed)
    cap = min(cap, n)
    deg = zipf_degrees(n, m, s, cap)
    ids = g.permutation(n)
    src = np.repeat(ids, deg)
    g.shuffle(src)
    # copy model, resolved by pointer doubling (parent[e] < e or == e)
    own = g.random(m) < 0.5
    own[0] = True
    uni = g.integers(0, n, size=m, dtype=np.int64)
    e = np.arange(m, dtype=np.int64)
    prev = (g.random(m) * np.maximum(e, 1)).astype(np.int64)
    prev = np.minimum(prev, np.maximum(e - 1, 0))
    parent = np.where(own, e, prev)
    while True:
        nxt = parent[parent]
        if np.array_equal(nxt, parent):
            break
        parent = nxt
    dst = uni[parent]
    out = np.empty((m, 2), dtype=dtype)
    out[:, 0] = src
    out[:, 1] = dst
    return out


# ----------------------------------------------------------------------------
# R-MAT symmetric simple graph
# ----------------------------------------------------------------------------
def _splitmix64(x: np.ndarray) -> np.ndarray:
    x = (x + U64(0x9E3779B97F4A7C15)) & U64(_MASK64)
    z = x
    z = (z ^ (z >> U64(30))) * U64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> U64(27))) * U64(0x94D049BB133111EB)
    return z ^ (z >> U64(31))


def _rmat_draw(g, count, scale, a, b, c):
    """One R-MAT quadrant choice per level: a -> (0,0), b -> (0,1),
    c -> (1,0), d -> (1,1), from a uniform 32-bit draw per level."""
    ta = np.uint32(int(a * 2**32))
    tb = np.uint32(int((a + b) * 2**32))
    tc = np.uint32(int((a + b + c) * 2**32))
    u = np.zeros(count, dtype=np.uint32)
    v = np.zeros(count, dtype=np.uint32)
    ge_a = np.empty(count, dtype=bool)
    ge_b = np.empty(count, dtype=bool)
    ge_c = np.empty(count, dtype=bool)
    for _ in range(scale):
        r = g.integers(0, 2**32, size=count, dtype=np.uint32)
        np.greater_equal(r, ta, out=ge_a)
        np.greater_equal(r, tb, out=ge_b)
        np.greater_equal(r, tc, out=ge_c)
        u <<= np.uint32(1)
        v <<= np.uint32(1)
        u |= ge_b                                  # quadrants c, d
        np.logical_xor(ge_a, ge_b, out=ge_a)       # quadrant b
        np.logical_xor(ge_a, ge_c, out=ge_a)       # ... or quadrant d
        v |= ge_a
    return u, v


def rmat_undirected(scale: int, m: int, seed: int, a=0.57, b=0.19, c=0.19,
                    oversample: float = 1.06) -> np.ndarray:
    """Exactly ``m`` distinct undirected non-loop edges (u < v) drawn by
    R-MAT, before relabelling.  More samples are drawn until ``m`` distinct
    edges exist; if more remain, the ``m`` with the smallest seeded 64-bit
    hash of (u, v) are kept."""
    g = _rng(seed)
    keys = np.empty(0, dtype=np.uint64)
    draw = int(m * oversample) + 1024
    while True:
        u, v = _rmat_draw(g, draw, scale, a, b, c)
        lo = np.minimum(u, v).astype(np.uint64)
        hi = np.maximum(u, v).astype(np.uint64)
        ok = lo != hi
        k = (lo[ok] << U64(32)) | hi[ok]
        keys = np.unique(np.concatenate([keys, k]))
        if keys.size >= m:
            break
        draw = int((m - keys.size) * 1.2) + 1024
    if keys.size > m:
        h = _splitmix64(keys ^ U64(int(seed) & _MASK64))
        sel = np.argpartition(h, m - 1)[:m]
        keys = np.sort(keys[sel])
    out = np.empty((m, 2), dtype=np.uint32)
    out[:, 0] = (keys >> U64(32)).astype(np.uint32)
    out[:, 1] = (keys & U64(0xFFFFFFFF)).astype(np.uint32)
    return out


def symmetrize(und: np.ndarray, n: int, seed: int, dtype=np.int32) -> np.ndarray:
    """Relabel vertices by a seeded permutation of [0, n), emit both
    directions of every undirected edge, shuffle the directed tuples."""
    g = _rng(seed ^ 0x5EED)
    perm = g.permutation(n).astype(np.int64)
    x = perm[und[:, 0].astype(np.int64)]
    y = perm[und[:, 1].astype(np.int64)]
    d = np.empty((2 * und.shape[0], 2), dtype=dtype)
    d[0::2, 0] = x
    d[0::2, 1] = y
    d[1::2, 0] = y
    d[1::2, 1] = x
    return d[g.permutation(d.shape[0])]


def rmat_symmetric(scale: int, m: int, seed: int, dtype=np.int32) -> np.ndarray:
    und = rmat_undirected(scale, m, seed)
    return symmetrize(und, 1 << scale, seed, dtype)


# ----------------------------------------------------------------------------
# Small triangle inputs for the batch
# ----------------------------------------------------------------------------
def gnm_symmetric(n: int, m: int, seed: int, dtype=np.int32) -> np.ndarray:
    """Uniform graph: m samples of distinct endpoints, canonicalised and
    de-duplicated (so at most m undirected edges), symmetrised."""
    g = _rng(seed)
    u = g.integers(0, n, size=m, dtype=np.int64)
    v = g.integers(0, n, size=m, dtype=np.int64)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    ok = lo != hi
    k = np.unique((lo[ok] << 32) | hi[ok])
    und = np.stack([k >> 32, k & 0xFFFFFFFF], axis=1)
    return symmetrize(und, n, seed, dtype)


def chung_lu_symmetric(n: int, m: int, seed: int, s: float = 1.1,
                       cap: int = 4096, dtype=np.int32) -> np.ndarray:
    """Chung-Lu style graph: both endpoints drawn with probability
    proportional to capped Zipf weights, canonicalised, de-duplicated,
    symmetrised."""
    g = _rng(seed)
    cap = min(cap, n - 1)
    w = np.minimum(float(cap), np.arange(1, n + 1, dtype=np.float64) ** (-s) * n)
    p = w / w.sum()
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    u = np.searchsorted(cdf, g.random(m), side="right")
    v = np.searchsorted(cdf, g.random(m), side="right")
    ids = g.permutation(n)
    u, v = ids[np.minimum(u, n - 1)], ids[np.minimum(v, n - 1)]
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    ok = lo != hi
    k = np.unique((lo[ok].astype(np.int64) << 32) | hi[ok].astype(np.int64))
    und = np.stack([k >> 32, k & 0xFFFFFFFF], axis=1)
    return symmetrize(und, n, seed, dtype)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------
LINEAR_SMALL = dict(n=65536, domain=4096, seed=1001, a_domain=4096)
LINEAR_POWERLAW = dict(n_vertices=1 << 20, m=1 << 24, seed=2001, a_domain=1 << 20)
TRIANGLE_RMAT = dict(scale=22, m_undirected=1 << 26, seed=3001)
STAR = dict(n_fact=1 << 26, k_r=4096, k_t=4096, a_domain=1024, seed=5001)


def linear_small(seed: int = LINEAR_SMALL["seed"]) -> np.ndarray:
    """65,536 uint32 tuples, both columns uniform in [0, 4096)."""
    return uniform_pairs(LINEAR_SMALL["n"], LINEAR_SMALL["domain"], seed)


def linear_powerlaw(seed: int = LINEAR_POWERLAW["seed"], n_vertices: int = None,
                    m: int = None) -> np.ndarray:
    """2^24 directed int32 edges over 2^20 vertices (scaled-down variants via
    ``n_vertices``/``m`` keep the mean degree of 16)."""
    nv = n_vertices or LINEAR_POWERLAW["n_vertices"]
    mm = m or LINEAR_POWERLAW["m"]
    return powerlaw_friends(nv, mm, seed)


def triangle_rmat(scale: int = TRIANGLE_RMAT["scale"], m_undirected: int = None,
                  seed: int = TRIANGLE_RMAT["seed"]) -> np.ndarray:
    """Symmetric simple R-MAT graph as 2*m directed int32 tuples."""
    mu = m_undirected or (16 << scale)
    return rmat_symmetric(scale, mu, seed)


def star_schema(n_fact: int = STAR["n_fact"], k_r: int = STAR["k_r"], k_t: int = STAR["k_t"],
                a_domain: int = STAR["a_domain"], seed: int = STAR["seed"]):
    """A fact relation S(B, C) of ``n_fact`` tuples with two dimension
    relations R(A, B) and T(C, D) (the star join's shape, N >> K).

    R: ``k_r`` tuples whose B values are distinct keys drawn from [0, 2^31)
    and whose A values are uniform in [0, a_domain).  T: ``k_t`` tuples with
    C uniform in [0, k_t) (a bag: some C values repeat, some are missing)
    and D uniform in [0, 2^31).  S: each B is one of R's keys (uniformly)
    with probability 15/16, else a uniform key in [0, 2^31) (almost surely
    absent from R); each C is uniform in [0, k_t).  Returns int32 arrays
    (R, S, T) of shape [n, 2]."""
    g = _rng(seed)
    keys = np.unique(g.integers(0, 1 << 31, size=2 * k_r + 64, dtype=np.int64))
    keys = keys[g.permutation(keys.size)][:k_r]
    R = np.empty((k_r, 2), dtype=np.int32)
    R[:, 0] = g.integers(0, a_domain, size=k_r)
    R[:, 1] = keys
    T = np.empty((k_t, 2), dtype=np.int32)
    T[:, 0] = g.integers(0, k_t, size=k_t)
    T[:, 1] = g.integers(0, 1 << 31, size=k_t)
    S = np.empty((n_fact, 2), dtype=np.int32)
    hit = g.random(n_fact) < 15.0 / 16.0
    S[:, 0] = np.where(hit, keys[g.integers(0, k_r, size=n_fact)], g.integers(0, 1 << 31, size=n_fact))
    S[:, 1] = g.integers(0, k_t, size=n_fact)
    return R, S, T


def batch_instances(count: int = 512, base_seed: int = 4000,
                    lo_exp: float = 3.0, hi_exp: float = 6.0):
    """The mixed batch: the first half linear, the second half triangle.

    Edge counts are log-uniform in [10^lo_exp, 10^hi_exp]; vertex counts keep
    the mean degree at 16 (at least 64 vertices); even instances have
    uniform degrees, odd ones Zipf(1.1) degrees capped at min(4096, n-1).
    Yields dicts with ``kind`` ('linear' | 'triangle'), ``F`` (the relation
    used for R, S and T), ``n`` and ``seed``."""
    return [batch_instance(k, count, base_seed, lo_exp, hi_exp) for k in range(count)]


def batch_instance(k: int, count: int = 512, base_seed: int = 4000,
                   lo_exp: float = 3.0, hi_exp: float = 6.0):
    """Instance k of batch_instances (generated alone)."""
    seed = base_seed + k
    g = _rng(seed)
    m = int(round(10 ** g.uniform(lo_exp, hi_exp)))
    n = max(64, m // 16)
    kind = "linear" if k < count // 2 else "triangle"
    if kind == "linear":
        if k % 2 == 0:
            F = uniform_pairs(m, n, seed, dtype=np.int32)
        else:
            F = powerlaw_friends(n, m, seed, cap=min(4096, n - 1))
    else:
        if k % 2 == 0:
            F = gnm_symmetric(n, m, seed)
        else:
            F = chung_lu_symmetric(n, m, seed, cap=min(4096, n - 1))
    return dict(kind=kind, F=F, n=n, seed=seed, m=m)
