"""Write the expected per-A counts of the power-law linear workload (2^24
edges over 2^20 vertices, seed 2001, R = S = T = F, a_domain = 2^20) using
only the CPU oracle.

The count of A value a sums over R tuples with r.a = a, so the oracle runs
on disjoint slices of R (tuple index mod P) in P processes and the slice
vectors are added.  Stored: the SHA-256 of the uint64[2^20] vector
(little-endian), its sum, the number of nonzero entries and 4096 sampled
entries (fixed seed), so that a test can compare all 2^20 entries by the
hash and name a differing one by the samples.

    python tests/golden/make_linear_golden.py [--procs 8]
"""
import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def _slice(args):
    k, procs = args
    import oracle
    from workloads import generators as G
    F = G.linear_powerlaw().view(np.uint32)
    R = np.ascontiguousarray(F[k::procs])
    t0 = time.time()
    c = oracle.linear3_count(R, F, F, 1 << 20)
    return k, c, time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    import oracle
    oracle.build()
    t0 = time.time()
    with ProcessPoolExecutor(args.procs) as ex:
        parts = list(ex.map(_slice, [(k, args.procs) for k in range(args.procs)]))
    count = np.zeros(1 << 20, dtype=np.uint64)
    for _, c, _ in parts:
        count += c.astype(np.uint64)
    rng = np.random.default_rng(20)
    sample = np.sort(rng.choice(1 << 20, size=4096, replace=False))
    out = {"workload": "power-law friends graph, 2^24 int32 edges over 2^20 vertices, Zipf(1.1) "
                       "out-degrees capped at 4096, preferential-attachment destinations, seed 2001; "
                       "R = S = T = F, a_domain = 2^20",
           "a_domain": 1 << 20,
           "sha256_u64_le": hashlib.sha256(count.astype("<u8").tobytes()).hexdigest(),
           "sum": int(count.sum(dtype=np.uint64)), "nonzero": int((count != 0).sum()),
           "sample_a": sample.tolist(), "sample_count": count[sample].astype(np.uint64).tolist(),
           "oracle_cpu_seconds": round(sum(p[2] for p in parts), 1),
           "wall_seconds": round(time.time() - t0, 1),
           "command": f"python tests/golden/make_linear_golden.py --procs {args.procs}"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "linear_powerlaw_2e24.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(json.dumps({k: v for k, v in out.items() if not k.startswith("sample")}))


if __name__ == "__main__":
    main()
