"""Inputs for the host-build replay (tests/hostsim/replay.cpp): the seeded
workloads written as raw little-endian uint32 [n, 2] files, with their
closed-form totals in meta.json.

    python tests/hostsim/make_inputs.py OUT_DIR [--full | --tiny]

The batch leg's eighty small joins are the same at every size.  Without
--full the power-law graph is scaled down (2^20 edges over 2^16
vertices, --tiny: 2^16 over 2^12) and the star schema's fact relation to
2^22 tuples (--tiny: 2^18).
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import generators as G  # noqa: E402


def closed_total(R, S, T):
    """Sum over S of deg_R(s.b) * deg_T(s.c): the linear join's total."""
    keys_r, cnt_r = np.unique(R[:, 1], return_counts=True)
    keys_t, cnt_t = np.unique(T[:, 0], return_counts=True)
    ir = np.searchsorted(keys_r, S[:, 0])
    it = np.searchsorted(keys_t, S[:, 1])
    ir_ok = (ir < keys_r.size) & (keys_r[np.minimum(ir, keys_r.size - 1)] == S[:, 0])
    it_ok = (it < keys_t.size) & (keys_t[np.minimum(it, keys_t.size - 1)] == S[:, 1])
    dr = np.where(ir_ok, cnt_r[np.minimum(ir, keys_r.size - 1)], 0).astype(np.uint64)
    dt = np.where(it_ok, cnt_t[np.minimum(it, keys_t.size - 1)], 0).astype(np.uint64)
    return int((dr * dt).sum(dtype=np.uint64))


def main():
    out = sys.argv[1]
    full = "--full" in sys.argv
    tiny = "--tiny" in sys.argv
    os.makedirs(out, exist_ok=True)
    meta = {}

    def put(name, arr, a_domain=None, R=None, S=None, T=None):
        arr = np.ascontiguousarray(np.asarray(arr).view(np.uint32).reshape(-1, 2))
        arr.tofile(os.path.join(out, name + ".bin"))
        meta[name] = {"n": int(arr.shape[0])}
        if a_domain is not None:
            meta[name]["a_domain"] = int(a_domain)

    if full:
        F = G.linear_powerlaw()
        a_dom = 1 << 20
    elif tiny:
        F = G.linear_powerlaw(seed=2001, n_vertices=1 << 12, m=1 << 16)
        a_dom = 1 << 12
    else:
        F = G.linear_powerlaw(seed=2001, n_vertices=1 << 16, m=1 << 20)
        a_dom = 1 << 16
    F = F.view(np.uint32)
    put("F", F, a_dom)
    meta["F"]["closed_total"] = closed_total(F, F, F)
    Fs = G.linear_small().view(np.uint32)
    put("Fs", Fs, 4096)
    meta["Fs"]["closed_total"] = closed_total(Fs, Fs, Fs)
    R, S, T = G.star_schema() if full else G.star_schema(n_fact=1 << (18 if tiny else 22))
    R, S, T = (x.view(np.uint32) for x in (R, S, T))
    put("starR", R, G.STAR["a_domain"])
    put("starS", S)
    put("starT", T)
    meta["starR"]["closed_total"] = closed_total(R, S, T)
    # the S-largest shape: dimension relations too large for the star plans
    k = 1 << (13 if tiny else 16)
    R, S, T = G.star_schema(n_fact=1 << (18 if tiny else (26 if full else 22)), k_r=k, k_t=k,
                            a_domain=1 << 14, seed=5002)
    R, S, T = (x.view(np.uint32) for x in (R, S, T))
    put("slR", R, 1 << 14)
    put("slS", S)
    put("slT", T)
    meta["slR"]["closed_total"] = closed_total(R, S, T)
    # skew: heavy first-column keys crowding two of the ranges (each range
    # then runs as several workgroups)
    g = np.random.default_rng(77)
    n = 1 << (18 if tiny else 21)
    K = g.integers(0, 4096, size=(n, 2)).astype(np.uint32)
    K[: n // 4, 0] = 5
    K[n // 4: (4 * n) // 5, 0] = 3000
    g.shuffle(K)
    put("K", K, 4096)
    meta["K"]["closed_total"] = closed_total(K, K, K)
    # a heavy key among many distinct ones, for hashed tables in four
    # buckets: with keys below 2^16 a piece of the heavy bucket overflows
    # its table (the bucket is read whole); below 19200 the pieces fit but
    # their union does not (the pass is redone from the tuples)
    for name, m, dom, heavy in (("K2", 131072, 1 << 16, 52428), ("K3", 86000, 19200, 40000)):
        K2 = g.integers(0, dom, size=(m, 2)).astype(np.uint32)
        K2[:heavy, 0] = 77
        g.shuffle(K2)
        put(name, K2, dom)
        meta[name]["closed_total"] = closed_total(K2, K2, K2)
    # a batch: small joins of both kinds (the mixed batch's generator);
    # a_domain 0 marks a cyclic join
    # twelve joins of 10^2.7..10^4 edges, then 68 of 10^2.2..10^2.9 (merged
    # launches of more than 64 joins)
    batch = [("B", k, G.batch_instance(k, count=12, lo_exp=2.7, hi_exp=4.0)) for k in range(12)]
    batch += [("B", 12 + k, G.batch_instance(k, count=68, base_seed=4600, lo_exp=2.2, hi_exp=2.9)) for k in range(68)]
    for _, k, x in batch:
        F = x["F"].view(np.uint32)
        put(f"B{k}", F, x["n"] if x["kind"] == "linear" else 0)
        # the linear join's total in closed form; the cyclic join's count from the oracle
        meta[f"B{k}"]["closed_total"] = closed_total(F, F, F) if x["kind"] == "linear" else \
            oracle.triangle3_count(F, F, F)
    with open(os.path.join(out, "meta.json"), "w") as f:
        json.dump(meta, f, indent=1)
    with open(os.path.join(out, "meta.txt"), "w") as f:          # name n a_domain closed_total
        for k, v in meta.items():
            f.write(f"{k} {v['n']} {v.get('a_domain', 0)} {v.get('closed_total', 0)}\n")
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
