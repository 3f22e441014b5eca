"""Write the expected result of every join of the 512-join batch workload
(seeds 4000 + k; joins 0-255 linear with a_domain = n_k, 256-511 cyclic;
R = S = T = the instance's relation) using only the CPU oracle, one join per
task in P processes.

Stored per join: its kind, sizes, the SHA-256 of the uint64 per-A vector
(little-endian; linear) or the total (cyclic), the sum, and the oracle's
CPU seconds.

    python tests/golden/make_batch_golden.py [--procs 8]
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


def _join(k):
    import oracle
    from workloads import generators as G
    x = G.batch_instance(k)
    F = np.ascontiguousarray(x["F"]).view(np.uint32)
    t0 = time.time()
    if x["kind"] == "linear":
        c = oracle.linear3_count(F, F, F, x["n"]).astype("<u8")
        rec = {"kind": "linear", "a_domain": int(x["n"]), "sha256_u64_le": hashlib.sha256(c.tobytes()).hexdigest(),
               "sum": int(c.sum(dtype=np.uint64))}
    else:
        tot = int(oracle.triangle3_count(F, F, F))
        rec = {"kind": "triangle", "total": tot, "sum": tot}
    rec.update({"k": k, "seed": int(x["seed"]), "tuples": int(F.shape[0]),
                "oracle_cpu_seconds": round(time.time() - t0, 3)})
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    import oracle
    oracle.build()
    t0 = time.time()
    # the largest joins first, so that the pool ends together (the edge
    # count is the first draw of each instance's generator)
    sizes = [int(round(10 ** np.random.default_rng(np.random.SeedSequence(4000 + k)).uniform(3.0, 6.0)))
             for k in range(512)]
    order = sorted(range(512), key=lambda k: -sizes[k])
    with ProcessPoolExecutor(args.procs) as ex:
        recs = sorted(ex.map(_join, order), key=lambda r: r["k"])
    out = {"workload": "512 joins: k < 256 linear, k >= 256 cyclic; m_k log-uniform in [10^3, 10^6] "
                       "edges, n_k = max(64, m_k / 16); uniform (k even) or Zipf(1.1) degrees (k odd); "
                       "seeds 4000 + k; R = S = T",
           "joins": recs,
           "oracle_cpu_seconds": round(sum(r["oracle_cpu_seconds"] for r in recs), 1),
           "wall_seconds": round(time.time() - t0, 1),
           "command": f"python tests/golden/make_batch_golden.py --procs {args.procs}"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch512.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(json.dumps({k: v for k, v in out.items() if k != "joins"}))


if __name__ == "__main__":
    main()
