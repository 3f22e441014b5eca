"""Independent checkers used to pin the oracle: literal triple loops for tiny
inputs and closed forms written with numpy / scipy.  Nothing here is shared
with the oracle's C code or with the HIP library."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def as_u32(x):
    return np.ascontiguousarray(np.asarray(x)).view(np.uint32).reshape(-1, 2)


def linear_bruteforce(R, S, T, a_domain):
    """Literal triple loop over (r, s, t)."""
    R, S, T = as_u32(R), as_u32(S), as_u32(T)
    out = [0] * a_domain
    for (a, b) in R.tolist():
        for (b2, c) in S.tolist():
            if b2 != b:
                continue
            for (c2, _d) in T.tolist():
                if c2 == c:
                    out[a] += 1
    return np.array(out, dtype=np.uint64)


def triangle_bruteforce(R, S, T):
    R, S, T = as_u32(R), as_u32(S), as_u32(T)
    tot = 0
    for (a, b) in R.tolist():
        for (b2, c) in S.tolist():
            if b2 != b:
                continue
            for (c2, a2) in T.tolist():
                if c2 == c and a2 == a:
                    tot += 1
    return tot


def join2_bruteforce(R, S):
    R, S = as_u32(R), as_u32(S)
    return sum(1 for (_a, b) in R.tolist() for (b2, _c) in S.tolist() if b2 == b)


def _dense_ids(*cols):
    allv = np.concatenate([np.asarray(c, dtype=np.uint32) for c in cols])
    keys, inv = np.unique(allv, return_inverse=True)
    out, o = [], 0
    for c in cols:
        out.append(inv[o:o + len(c)])
        o += len(c)
    return keys, out


def linear_closed_total(R, S, T):
    """Sum over (b, c) in S of deg_R(b) * deg_T(c), with degrees from
    np.unique counts (exact while the total stays below 2^63)."""
    R, S, T = as_u32(R), as_u32(S), as_u32(T)

    def deg_of(keys, cnts, q):
        i = np.searchsorted(keys, q)
        i = np.minimum(i, max(len(keys) - 1, 0))
        hit = (keys[i] == q) if len(keys) else np.zeros(len(q), bool)
        return np.where(hit, cnts[i] if len(keys) else 0, 0).astype(np.int64)

    rb, rcnt = np.unique(R[:, 1], return_counts=True)
    tc, tcnt = np.unique(T[:, 0], return_counts=True)
    dR = deg_of(rb, rcnt, S[:, 0])
    dT = deg_of(tc, tcnt, S[:, 1])
    return int((dR * dT).sum())


def linear_closed_per_a(R, S, T, a_domain):
    """count = M_R (M_S deg_T): two sparse matrix-vector products, exact in
    int64 (callers keep totals below 2^63)."""
    R, S, T = as_u32(R), as_u32(S), as_u32(T)
    keys, (rb, sb, sc, tc) = _dense_ids(R[:, 1], S[:, 0], S[:, 1], T[:, 0])
    n = keys.size
    one = lambda k: np.ones(k, dtype=np.int64)
    MR = sp.csr_matrix((one(len(rb)), (R[:, 0].astype(np.int64), rb)), shape=(a_domain, n))
    MS = sp.csr_matrix((one(len(sb)), (sb, sc)), shape=(n, n))
    degT = np.bincount(tc, minlength=n).astype(np.int64)
    return (MR @ (MS @ degT)).astype(np.uint64)


def join2_closed(R, S):
    R, S = as_u32(R), as_u32(S)
    rb, rc = np.unique(R[:, 1], return_counts=True)
    sb, sc = np.unique(S[:, 0], return_counts=True)
    common, ir, is_ = np.intersect1d(rb, sb, return_indices=True)
    return int((rc[ir].astype(object) * sc[is_].astype(object)).sum()) if common.size else 0


def triangle_trace(R, S, T):
    """trace(M_R M_S M_T) with dense int64 matrices (small vertex sets)."""
    R, S, T = as_u32(R), as_u32(S), as_u32(T)
    keys, (ra, rb, sb, sc, tc, ta) = _dense_ids(R[:, 0], R[:, 1], S[:, 0], S[:, 1],
                                                 T[:, 0], T[:, 1])
    n = keys.size
    MR = np.zeros((n, n), dtype=np.int64)
    MS = np.zeros((n, n), dtype=np.int64)
    MT = np.zeros((n, n), dtype=np.int64)
    np.add.at(MR, (ra, rb), 1)
    np.add.at(MS, (sb, sc), 1)
    np.add.at(MT, (tc, ta), 1)
    return int(np.trace(MR @ MS @ MT))


def triangle_sparse_selfjoin(E):
    """For R = S = T = E: sum((A @ A) .* A^T) = trace(A^3), scipy sparse."""
    E = as_u32(E)
    keys, (x, y) = _dense_ids(E[:, 0], E[:, 1])
    n = keys.size
    A = sp.csr_matrix((np.ones(len(x), dtype=np.int64), (x, y)), shape=(n, n))
    A.sum_duplicates()
    return int((A @ A).multiply(A.T).sum())
