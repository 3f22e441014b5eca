"""CPU oracle for the multiway joins -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  The product library never calls it, and the
two share no code: the oracle's C file (``oracle.c``) is compiled here with
gcc, on its own.

Contents
  * the join counts (plain nested-loop joins in C, Sec. 3 / Sec. 5):
      ``linear3_count``, ``triangle3_count``, ``join2_size``,
      ``triangle3_count_masked``, ``linear3_count_sampled``
  * the Flajolet-Martin distinct count of D per A: ``linear3_distinct``,
    ``fm_sketch``
  * the linear join's result written out, in nested-loop order:
    ``linear3_materialize``, ``linear3_materialize_at``
  * ``cost_model``: the paper's analytic cost formulas (Sec. 4.2, 5.2, 6.3,
    6.5 footnote, App. A), in float64
  * ``mlp_ref``: a float64 reference of the learned planner's network
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, OVERFLOW, KEY_RANGE, NOMEM = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (in place)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def bind(lib):
    """Declare the C signatures on a loaded oracle library."""
    u32p = ctypes.c_void_p
    i64, u64 = ctypes.c_int64, ctypes.c_uint64
    lib.orc_linear3_count.argtypes = [u32p, u32p, i64, u64, u32p, u32p, i64, u64,
                                      u32p, i64, u64, ctypes.c_uint32, u32p]
    lib.orc_join2_size.argtypes = [u32p, u32p, i64, u64, u32p, i64, u64, u32p]
    lib.orc_triangle3_count.argtypes = [u32p, u32p, i64, u64, u32p, u32p, i64, u64,
                                        u32p, u32p, i64, u64, u32p, u32p]
    lib.orc_triangle3_count_masked.argtypes = [u32p, u32p, i64, u64, u32p, u32p, i64, u64,
                                               u32p, u32p, u32p, i64, u64, u32p, u32p]
    lib.orc_linear3_count_sampled.argtypes = [u32p, u32p, i64, u64, u32p, u32p, i64, u64,
                                              u32p, i64, u64, u32p, u64, u32p]
    lib.orc_linear3_distinct.argtypes = [u32p, u32p, i64, u64, u32p, u32p, i64, u64,
                                         u32p, u32p, i64, u64, u32p, u64, ctypes.c_uint32,
                                         u32p, u32p, u32p]
    lib.orc_fm_sketch.argtypes = [u32p, u64, ctypes.c_uint32, u32p, u32p]
    lib.orc_linear3_materialize.argtypes = [u32p, u32p, i64, u64, u32p, u32p, i64, u64,
                                            u32p, u32p, i64, u64, u64, u64, u32p, u32p]
    lib.orc_linear3_materialize_at.argtypes = [u32p, u32p, i64, u64, u32p, u32p, i64, u64,
                                               u32p, u32p, i64, u64, u32p, u64, u32p, u32p]
    for f in ("orc_linear3_count", "orc_join2_size", "orc_triangle3_count",
              "orc_triangle3_count_masked", "orc_linear3_count_sampled",
              "orc_linear3_distinct", "orc_fm_sketch", "orc_linear3_materialize",
              "orc_linear3_materialize_at"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = bind(ctypes.CDLL(_LIB))
    return _lib


def _rel(x):
    """[n, 2] array of 32-bit values -> (uint32 contiguous array, col0, col1, stride, n)."""
    a = np.ascontiguousarray(np.asarray(x)).view(np.uint32).reshape(-1, 2)
    a = np.ascontiguousarray(a)
    p = a.ctypes.data
    return a, ctypes.c_void_p(p), ctypes.c_void_p(p + 4), 2, a.shape[0]


class OracleError(RuntimeError):
    pass


def _check(st, what):
    if st == KEY_RANGE:
        raise OracleError(f"{what}: an A value is outside [0, a_domain)")
    if st == NOMEM:
        raise MemoryError(what)
    if st == OVERFLOW:
        raise OverflowError(f"{what}: a count does not fit 64 bits")


def linear3_count(R, S, T, a_domain: int) -> np.ndarray:
    """uint64[a_domain]: out[a] = #{(r,s,t): r.a=a, r.b=s.b, s.c=t.c}."""
    lib = _load()
    ra, r0, r1, rs, nr = _rel(R)
    sa, s0, s1, ss, ns = _rel(S)
    ta, t0, _t1, ts, nt = _rel(T)
    out = np.zeros(max(int(a_domain), 1), dtype=np.uint64)
    st = lib.orc_linear3_count(r0, r1, rs, nr, s0, s1, ss, ns, t0, ts, nt,
                               ctypes.c_uint32(a_domain), out.ctypes.data)
    _check(st, "linear3_count")
    return out[:a_domain]


def linear3_count_sampled(R, S, T, alist) -> np.ndarray:
    """Counts for the A values in ``alist`` only (returned in sorted order of
    the unique values: ``np.unique(alist)``)."""
    lib = _load()
    ra, r0, r1, rs, nr = _rel(R)
    sa, s0, s1, ss, ns = _rel(S)
    ta, t0, _t1, ts, nt = _rel(T)
    al = np.unique(np.asarray(alist).view(np.uint32) if np.asarray(alist).dtype.itemsize == 4
                   else np.asarray(alist, dtype=np.uint32))
    al = np.ascontiguousarray(al.astype(np.uint32))
    out = np.zeros(max(al.size, 1), dtype=np.uint64)
    st = lib.orc_linear3_count_sampled(r0, r1, rs, nr, s0, s1, ss, ns, t0, ts, nt,
                                       al.ctypes.data, al.size, out.ctypes.data)
    _check(st, "linear3_count_sampled")
    return al, out[:al.size]


def linear3_distinct(R, S, T, alist, seed: int):
    """For each A value in ``np.unique(alist)``: the Flajolet-Martin sketch
    (uint32[16]) of the set of D values it reaches through R |x| S |x| T,
    the sketch's estimate (float64) and the exact size of the set.
    Returns (a_values, sketches [na, 16], estimates [na], exact [na])."""
    lib = _load()
    ra, r0, r1, rs, nr = _rel(R)
    sa, s0, s1, ss, ns = _rel(S)
    ta, t0, t1, ts, nt = _rel(T)
    al = np.ascontiguousarray(np.unique(np.asarray(alist).astype(np.int64) & 0xFFFFFFFF).astype(np.uint32))
    sk = np.zeros((max(al.size, 1), 16), dtype=np.uint32)
    est = np.zeros(max(al.size, 1), dtype=np.float64)
    exact = np.zeros(max(al.size, 1), dtype=np.uint64)
    st = lib.orc_linear3_distinct(r0, r1, rs, nr, s0, s1, ss, ns, t0, t1, ts, nt,
                                  al.ctypes.data, al.size, ctypes.c_uint32(seed & 0xFFFFFFFF),
                                  sk.ctypes.data, est.ctypes.data, exact.ctypes.data)
    _check(st, "linear3_distinct")
    return al, sk[:al.size], est[:al.size], exact[:al.size]


def fm_sketch(values, seed: int):
    """The Flajolet-Martin sketch (uint32[16]) and estimate of a set of
    32-bit values (duplicates are harmless: the sketch is a union)."""
    lib = _load()
    v = np.ascontiguousarray(np.asarray(values).astype(np.int64) & 0xFFFFFFFF).astype(np.uint32)
    sk = np.zeros(16, dtype=np.uint32)
    est = np.zeros(1, dtype=np.float64)
    st = lib.orc_fm_sketch(v.ctypes.data, v.size, ctypes.c_uint32(seed & 0xFFFFFFFF),
                           sk.ctypes.data, est.ctypes.data)
    _check(st, "fm_sketch")
    return sk, float(est[0])


def join2_size(R, S) -> int:
    """|R(AB) join S(BC)| on B."""
    lib = _load()
    ra, r0, r1, rs, nr = _rel(R)
    sa, s0, s1, ss, ns = _rel(S)
    out = np.zeros(1, dtype=np.uint64)
    st = lib.orc_join2_size(r0, r1, rs, nr, s0, ss, ns, out.ctypes.data)
    _check(st, "join2_size")
    return int(out[0])


def triangle3_count(R, S, T, smask=None) -> int:
    """#{(r,s,t): r.b=s.b, s.c=t.c, t.a=r.a} (optionally over the S tuples
    whose mask byte is non-zero)."""
    lib = _load()
    ra, r0, r1, rs, nr = _rel(R)
    sa, s0, s1, ss, ns = _rel(S)
    ta, t0, t1, ts, nt = _rel(T)
    lo = np.zeros(1, dtype=np.uint64)
    hi = np.zeros(1, dtype=np.uint64)
    if smask is None:
        st = lib.orc_triangle3_count(r0, r1, rs, nr, s0, s1, ss, ns, t0, t1, ts, nt,
                                     lo.ctypes.data, hi.ctypes.data)
    else:
        m = np.ascontiguousarray(np.asarray(smask, dtype=np.uint8))
        assert m.size == ns
        st = lib.orc_triangle3_count_masked(r0, r1, rs, nr, s0, s1, ss, ns, m.ctypes.data,
                                            t0, t1, ts, nt, lo.ctypes.data, hi.ctypes.data)
    if st == NOMEM:
        raise MemoryError("triangle3_count")
    return int(lo[0]) + (int(hi[0]) << 64)


def linear3_materialize(R, S, T, lo: int = 0, cap: int | None = None):
    """The result tuples (a, b, c, d) of R |x| S |x| T in nested-loop order
    (r in R's order, then the matching s in S's order, then the matching t
    in T's order): elements [lo, lo + cap) as uint32 [k, 4], and the total
    length of the sequence."""
    lib = _load()
    ra, r0, r1, rs, nr = _rel(R)
    sa, s0, s1, ss, ns = _rel(S)
    ta, t0, t1, ts, nt = _rel(T)
    total = np.zeros(1, dtype=np.uint64)
    if cap is None:
        st = lib.orc_linear3_materialize(r0, r1, rs, nr, s0, s1, ss, ns, t0, t1, ts, nt,
                                         0, 0, None, total.ctypes.data)
        _check(st, "linear3_materialize")
        cap = max(int(total[0]) - lo, 0)
    out = np.zeros((max(cap, 1), 4), dtype=np.uint32)
    st = lib.orc_linear3_materialize(r0, r1, rs, nr, s0, s1, ss, ns, t0, t1, ts, nt,
                                     lo, cap, out.ctypes.data, total.ctypes.data)
    _check(st, "linear3_materialize")
    n = max(0, min(cap, int(total[0]) - lo))
    return out[:n], int(total[0])


def linear3_materialize_at(R, S, T, positions):
    """The elements of the same sequence at the given positions (uint32
    [k, 4]; all-ones rows past its end), and its total length."""
    lib = _load()
    ra, r0, r1, rs, nr = _rel(R)
    sa, s0, s1, ss, ns = _rel(S)
    ta, t0, t1, ts, nt = _rel(T)
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.uint64))
    out = np.zeros((max(pos.size, 1), 4), dtype=np.uint32)
    total = np.zeros(1, dtype=np.uint64)
    st = lib.orc_linear3_materialize_at(r0, r1, rs, nr, s0, s1, ss, ns, t0, t1, ts, nt,
                                        pos.ctypes.data, pos.size, out.ctypes.data, total.ctypes.data)
    _check(st, "linear3_materialize_at")
    return out[:pos.size], int(total[0])
