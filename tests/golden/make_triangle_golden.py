"""Write the expected cyclic-join total for the R-MAT scale-22 workload
(2^26 undirected edges, seed 3001, R = S = T) using only the CPU oracle.

The total is a sum over S tuples, so the oracle runs on disjoint slices of S
(tuple index mod P) in P processes and the slice totals are added.

    python tests/golden/make_triangle_golden.py [--procs 8] [--scale 22]
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def _slice(args):
    scale, seed, k, procs = args
    import oracle
    from workloads import generators as G
    E = G.triangle_rmat(scale=scale, m_undirected=16 << scale, seed=seed)
    mask = (np.arange(E.shape[0]) % procs == k).astype(np.uint8)
    t0 = time.time()
    tot = oracle.triangle3_count(E, E, E, smask=mask)
    return k, tot, time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--seed", type=int, default=3001)
    args = ap.parse_args()
    import oracle
    oracle.build()
    t0 = time.time()
    with ProcessPoolExecutor(args.procs) as ex:
        parts = list(ex.map(_slice, [(args.scale, args.seed, k, args.procs) for k in range(args.procs)]))
    total = sum(p[1] for p in parts)
    assert total % 6 == 0
    out = {"workload": f"R-MAT scale {args.scale}, {16 << args.scale} undirected edges, "
                       f"a=.57 b=c=.19 d=.05, seed {args.seed}, R = S = T (symmetric)",
           "scale": args.scale, "seed": args.seed, "directed_tuples": 2 * (16 << args.scale),
           "total": total, "triangles": total // 6,
           "slices": {str(k): int(t) for k, t, _ in parts},
           "oracle_cpu_seconds": round(sum(p[2] for p in parts), 1),
           "wall_seconds": round(time.time() - t0, 1),
           "command": f"python tests/golden/make_triangle_golden.py --procs {args.procs} "
                      f"--scale {args.scale} --seed {args.seed}"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        f"triangle_rmat{args.scale}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
