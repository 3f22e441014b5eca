"""Benchmark: the linear three-way join on the power-law friends graph.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--paths]
    python bench.py --only LEG      (one of the other paths alone)

Workload: F = 2^24 directed int32 edges over 2^20 vertices, out-degrees
Zipf(1.1) capped at 4096, destinations by preferential attachment (seed
2001); R = S = T = F; per-A uint64 path counts over a_domain = 2^20.
A step is one mj_linear3_count call: with the planner's direct-indexed
tables, one range partition of F and three per-range sums (multiplicities
of C, W per B, counts per A).  Inputs are resident in HBM before timing
starts; planning happens once, outside the timed region.  One JSON line
goes to stdout.  The other paths (cascade, small, fm, emit, star,
triangle, batch, planner) run with --only LEG, or all of them with
--paths, each in a child process of its own.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(name, n_r, n_s, n_t, distinct_t, distinct_b, a_domain, b_domain=0, c_domain=0,
                 shared_partition=False):
    """Algorithmic HBM bytes of one launch of the named kernel.  With
    ``shared_partition`` (R = S = T one relation, whose partitions by range of
    its first column are one and the same) the partition launches move one
    relation, not three."""
    part_hist = 4 * n_s if shared_partition else 4 * (n_r + n_s + n_t)
    part_scatter = 16 * n_s if shared_partition else 16 * (n_r + n_s) + 8 * n_t
    table = {
        # direct-indexed tables: T.c, S and R partitioned by range in one launch group
        "dense:k_part_hist": part_hist,                 # read the key columns
        "dense:k_part_scatter": part_scatter,           # read + write the pairs (T: its C column)
        # T's pairs (the shared partition), deg[] and its 2-byte copy written once
        "k_range_deg": 8 * n_t + 6 * c_domain,
        # S pairs, one 2-byte deg[c] read per tuple, W[] and its 2-byte copy written once
        "k_range_w": 10 * n_s + 10 * b_domain,
        # R pairs, one 2-byte W[b] read per tuple (the full W only where the copy
        # saturates: 0.03 % of the reads here, not counted), the counts written once
        "k_range_count": 10 * n_r + 8 * a_domain,
        "rs:k_part_hist": 4 * (n_r + n_s),              # read the bucketed columns
        "rs:k_part_scatter": 16 * (n_r + n_s),          # read + write 8-byte tuples
        "tab:k_part_hist": 4 * n_t,                     # read the C column
        "tab:k_part_scatter": 8 * n_t,                  # read + write the C column
        "tab:k_dbuild": 4 * n_t + 16 * distinct_t,      # read C, write the table
        # S, one 8-byte multiplicity slot per s, the W table (16-byte slots, load 1/2)
        "k_wbuild": 16 * n_s + 32 * distinct_b,
        # R, one 16-byte W slot per r, the counts written once
        "k_count": 24 * n_r + 8 * a_domain,
        "k_linear_cell": 16 * n_s + 16 * n_r,           # S, R, one table slot per s, one count per r
    }
    return table.get(name)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel's sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec["traffic_bytes"] if h.hexdigest() == rec["sha256"] else None


def cpu_baseline(F, a_domain):
    """The oracle (single-threaded C) on a bounded sample: R = every 16th
    tuple of F, S = T = F."""
    import numpy as np
    import oracle
    Rs = np.ascontiguousarray(F[::16])
    t0 = time.perf_counter()
    oracle.linear3_count(Rs, F, F, a_domain)
    dt = time.perf_counter() - t0
    n_in = Rs.shape[0] + 2 * F.shape[0]
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n_in / dt, "unit": "input tuples/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_nproc": os.cpu_count(),
            "sample": f"R = every 16th tuple of F ({Rs.shape[0]} tuples), S = T = F "
                      f"({F.shape[0]} tuples); {dt:.2f} s single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (to scale HBM byte counters)")
    ap.add_argument("--no-extra", action="store_true",
                    help="time only the main workload (no child legs)")
    ap.add_argument("--paths", action="store_true",
                    help="after the main workload, run every other path (not only the default "
                         "legs), each in a child process of its own (bench.py --only LEG)")
    ap.add_argument("--only", choices=LEGS, default=None,
                    help="run one of the other paths alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1905_13376_amd as mj
    from workloads import generators as G

    if args.only in OWN_WORKLOAD_LEGS:
        # a leg on a workload of its own: the power-law graph is not needed
        ctx = mj.Context()
        print(json.dumps({args.only: extra_paths(mj, ctx, None, None, 1 << 20, None, None, only=args.only)}),
              flush=True)
        return
    log("generating the power-law friends graph (2^24 edges, 2^20 vertices)")
    F = G.linear_powerlaw()
    a_domain = 1 << 20
    n = F.shape[0]
    Fd = torch.from_numpy(F).to("cuda")
    torch.cuda.synchronize()

    # a plain device copy of known size (1 GiB read + 1 GiB written): the
    # measured bandwidth beside the 8 TB/s peak, and the calibration of the
    # byte counters (--calib-copy only adds the run to a profile)
    src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * (1 << 30) * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
    ctx = mj.Context()
    t0 = time.perf_counter()
    plan = ctx.plan(mj.LINEAR, Fd, Fd, Fd, a_domain)
    plan_ms = (time.perf_counter() - t0) * 1e3
    log(f"plan {plan.as_dict()} ({plan_ms:.1f} ms)")
    if args.only:
        print(json.dumps({args.only: extra_paths(mj, ctx, F, Fd, a_domain, plan, None, only=args.only)}),
              flush=True)
        return
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    out = torch.empty(a_domain, dtype=torch.int64, device="cuda")

    def step():
        ctx.linear3_count(Fd, Fd, Fd, a_domain, plan=plan, out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # correctness of the benchmarked configuration (outside the timed region)
    got = mj.as_u64(out)
    indeg = np.bincount(F[:, 1], minlength=a_domain).astype(np.int64)
    outdeg = np.bincount(F[:, 0], minlength=a_domain).astype(np.int64)
    closed = int((indeg[F[:, 0]] * outdeg[F[:, 1]]).sum())
    exact = int(got.sum(dtype=np.uint64)) == closed
    log(f"sum of counts {int(got.sum(dtype=np.uint64))} vs closed form {closed}: {exact}")

    stream = torch.cuda.current_stream()

    def timed_steps():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    # the timed region: K steps with nothing else on the stream
    ms = timed_steps()
    # the same K steps again with the library's HIP events around every
    # kernel, on the stream the kernels run on: per-kernel launch times
    ctx.profile(True)
    ctx.profile_read()
    ms_profiled = timed_steps()
    prof = ctx.profile_read()
    ctx.profile(False)
    log(f"{ms:.4f} ms per step ({ms_profiled:.4f} ms with per-kernel events)")
    kern = {k: (v[0] / max(v[1], 1), v[1] // args.steps) for k, v in prof.items()}
    for k, (avg, per) in sorted(kern.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        log(f"  {k:24s} {avg * 1e3:9.1f} us x {per}")

    distinct_t = int(np.unique(F[:, 0]).size)       # T.c and S.b are both F's first column
    dom = max(kern, key=lambda k: kern[k][0] * kern[k][1])
    avg_ms = kern[dom][0]
    nbytes = kernel_bytes(dom, n, n, n, distinct_t, distinct_t, a_domain, plan.b_domain, plan.c_domain,
                          shared_partition=True)
    roof = None
    if nbytes:
        ach = nbytes / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom),
                "algorithmic_bytes": nbytes, "avg_launch_us": round(avg_ms * 1e3, 2),
                "measured_copy_gbs": round(copy_gbs, 1)}
    # every kernel of the step on its own algorithmic bytes
    per_kernel = {}
    for k, (avg, per) in kern.items():
        kb = kernel_bytes(k, n, n, n, distinct_t, distinct_t, a_domain, plan.b_domain, plan.c_domain,
                          shared_partition=True)
        if kb:
            per_kernel[k] = {"us": round(avg * 1e3, 2), "algorithmic_bytes": kb,
                             "frac_of_peak": round(kb / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    # algorithmic probes of the step: one table read per S tuple (W) and per R
    # tuple (counts), one key counted per T tuple (multiplicities)
    probes = 3 * n
    result = {
        "metric": "join input tuples/s (linear 3-way, per-A count)",
        "value": 3 * n / (ms * 1e-3),
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 keys / u64 counts",
        "data": "synthetic",
        "config": {"workload": "linear 3-way self-join F|x|F|x|F, power-law friends graph: "
                               "2^24 int32 edges, 2^20 vertices, Zipf(1.1) out-degrees capped "
                               "at 4096, preferential-attachment destinations, seed 2001",
                   "a_domain": a_domain, "log2_nb": plan.log2_nb, "log2_nc": plan.log2_nc,
                   "tables": "direct-indexed" if plan.flags & mj.PLAN_DENSE_KEYS else "hashed",
                   "b_domain": plan.b_domain, "c_domain": plan.c_domain,
                   "plan_ms": round(plan_ms, 2), "exact_sum_check": exact,
                   "ms_per_step_with_kernel_events": round(ms_profiled, 4),
                   "probes_per_s": probes / (ms * 1e-3),
                   "measured_copy_gbs": round(copy_gbs, 1),
                   "kernels_us": {k: round(v[0] * 1e3, 2) for k, v in kern.items()},
                   "kernels_roofline": per_kernel},
        "roofline": roof,
    }
    # The other paths never run in this process after the timed workload:
    # that sequence faulted the GPU (the first call after it), while each
    # path alone and the timed workload alone run cleanly.  By default the
    # other configurations (the small linear workload, the cyclic join, the
    # 512-join batch, the planners) and the gather-locality measurement run
    # after it, each as a child process of its own; --paths runs every leg.
    if not args.no_extra:
        del ws, out
        ctx.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        result["paths"] = child_paths(LEGS if args.paths else DEFAULT_LEGS)
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(F, a_domain)
        result["cpu_baseline"]["per_config"] = oracle_per_config()
    print(json.dumps(result), flush=True)


def oracle_per_config():
    """The oracle's time on every configuration: the small linear workload
    timed here (median of 5 runs, one thread), the others from the CPU
    seconds the oracle-only golden scripts recorded (one thread per slice
    or join, summed)."""
    import numpy as np
    import oracle
    from workloads import generators as G
    Fs = G.linear_small().view(np.uint32)
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.linear3_count(Fs, Fs, Fs, 4096)
        ts.append(time.perf_counter() - t0)
    out = {"linear_small_65536": {"seconds": round(float(np.median(ts)), 4), "runs": 5,
                                  "input_tuples_per_s": 3 * Fs.shape[0] / float(np.median(ts)),
                                  "where": "this host, one thread"}}
    gdir = os.path.join(ROOT, "tests", "golden")
    for key, fname, what in (("linear_powerlaw_2e24", "linear_powerlaw_2e24.json", "all 2^20 per-A counts"),
                             ("cyclic_rmat22", "triangle_rmat22.json", "the cyclic total"),
                             ("batch_512", "batch512.json", "every join of the batch")):
        path = os.path.join(gdir, fname)
        if os.path.exists(path):
            g = json.load(open(path))
            out[key] = {"cpu_seconds": g.get("oracle_cpu_seconds"), "computes": what,
                        "where": "recorded by " + g.get("command", fname) + " (one thread per task)"}
    return out


def time_call(fn, steps, warmup=1):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_and_profile(ctx, fn, steps, warmup=1, prof_calls=None):
    """Milliseconds per call of `fn` timed with the library's per-kernel
    events off, then per-kernel figures from further calls with them on:
    {kernel: (ms per call, launches per call)}."""
    import torch
    ms = time_call(fn, steps, warmup)
    n = prof_calls or steps
    ctx.profile(True)
    ctx.profile_read()
    for _ in range(n):
        fn()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    return ms, {k: (v[0] / n, v[1] / n) for k, v in prof.items()}


def star_path(mj, ctx):
    """The star join (Sec. 6): a 2^26-tuple fact relation with two 4096-tuple
    dimension relations, under the plan the planner picks (the star
    three-way join) and under the star cascade, the partitioned three-way
    join and the cascade of binary hash joins."""
    import numpy as np
    import torch
    from workloads import generators as G
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import brute
    log("generating the star schema (2^26 fact tuples, 4096-tuple dimensions)")
    R, S, T = G.star_schema()
    a_dom = G.STAR["a_domain"]
    Rd, Sd, Td = (torch.from_numpy(x).to("cuda") for x in (R, S, T))
    closed = brute.linear_closed_total(R, S, T)
    plan = ctx.plan(mj.LINEAR, Rd, Sd, Td, a_dom)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(a_dom, dtype=torch.int64, device="cuda")
    res = {"planned_algo": int(plan.algo), "fact_tuples": int(S.shape[0]),
           "est_ms": {"star": round(plan.est_ms_star, 3), "star_cascade": round(plan.est_ms_star_cascade, 3),
                      "3way": round(plan.est_ms_3way, 3), "cascade": round(plan.est_ms_cascade, 3)}}
    n_in = R.shape[0] + S.shape[0] + T.shape[0]
    for name, algo in (("star", mj.ALGO_STAR), ("star_cascade", mj.ALGO_STAR_CASCADE),
                       ("partitioned_3way", mj.ALGO_3WAY), ("cascade", mj.ALGO_CASCADE)):
        p = plan.copy()
        p.algo = algo
        if algo in (mj.ALGO_STAR, mj.ALGO_3WAY):
            fn = lambda: ctx.linear3_count(Rd, Sd, Td, a_dom, plan=p, out=cnt, workspace=ws)
        else:
            fn = lambda: ctx.cascade2_count(mj.LINEAR, Rd, Sd, Td, a_dom, plan=p, out=cnt, workspace=ws)
        ms, kp = time_and_profile(ctx, fn, 5)
        ok = int(mj.as_u64(cnt).sum(dtype=np.uint64)) == closed
        kern = {k: v[0] / max(v[1], 1) for k, v in kp.items()}          # ms per launch
        ent = {"ms": round(ms, 4), "tuples_per_s": n_in / (ms * 1e-3), "sum_equals_closed_form": ok,
               "kernels_us": {k: round(v * 1e3, 1) for k, v in sorted(kern.items(), key=lambda kv: -kv[1])[:6]}}
        kg = next((k for k in ("k_star_group_b", "k_star_group_a") if k in kern), None)
        if name == "star" and kg:
            us = kern[kg] * 1e3
            nbytes = 8 * S.shape[0]                      # the fact relation, read once
            ach = nbytes / (us * 1e-6) / 1e9
            ent["roofline"] = {"bound": "hbm", "kernel": kg, "achieved": round(ach, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                               "algorithmic_bytes": nbytes, "avg_launch_us": round(us, 2)}
        res[name] = ent
        log(f"star schema, {name}: {ms:.3f} ms, sum ok {ok}")
    res["speedup_star_over_star_cascade"] = round(res["star_cascade"]["ms"] / res["star"]["ms"], 2)
    res["speedup_star_over_partitioned"] = round(res["partitioned_3way"]["ms"] / res["star"]["ms"], 2)
    del ws, Rd, Sd, Td
    return res


def slarge_path(mj, ctx):
    """The S-largest form of the linear join (Sec. 4, after Algorithm 1): a
    2^26-tuple S with R and T of 2^16 tuples each (beyond the star plans),
    under the planner's S-largest plan and, on the same bucket counts, the
    partitioned three-way join and the cascade."""
    import numpy as np
    import torch
    from workloads import generators as G
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import brute
    log("generating the S-largest workload (2^26 S tuples, 2^16-tuple R and T)")
    R, S, T = G.star_schema(n_fact=1 << 26, k_r=1 << 16, k_t=1 << 16, a_domain=1 << 14, seed=5002)
    a_dom = 1 << 14
    Rd, Sd, Td = (torch.from_numpy(x).to("cuda") for x in (R, S, T))
    closed = brute.linear_closed_total(R, S, T)
    plan = ctx.plan(mj.LINEAR, Rd, Sd, Td, a_dom)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(a_dom, dtype=torch.int64, device="cuda")
    n_in = R.shape[0] + S.shape[0] + T.shape[0]
    res = {"planned_algo": int(plan.algo), "log2_nb": int(plan.log2_nb), "log2_nc": int(plan.log2_nc),
           "est_ms": {"slarge": round(plan.est_ms_slarge, 3), "3way": round(plan.est_ms_3way, 3),
                      "cascade": round(plan.est_ms_cascade, 3)}}
    clog2 = lambda x: max(0, (int(x) - 1).bit_length())
    for name, algo in (("s_largest", mj.ALGO_SLARGE), ("partitioned_3way", mj.ALGO_3WAY),
                       ("cascade", mj.ALGO_CASCADE)):
        p = plan.copy()
        p.algo = algo
        if algo != mj.ALGO_SLARGE:
            # the bucket counts the planner gives these plans (about 16K S
            # tuples per B bucket, 32K T tuples per C bucket)
            p.log2_nb = min(10, clog2((S.shape[0] + 16383) // 16384))
            p.log2_nc = min(10, clog2((T.shape[0] + 32767) // 32768))
        if algo == mj.ALGO_CASCADE:
            fn = lambda: ctx.cascade2_count(mj.LINEAR, Rd, Sd, Td, a_dom, plan=p, out=cnt, workspace=ws)
        else:
            fn = lambda: ctx.linear3_count(Rd, Sd, Td, a_dom, plan=p, out=cnt, workspace=ws)
        ms, kp = time_and_profile(ctx, fn, 5)
        ok = int(mj.as_u64(cnt).sum(dtype=np.uint64)) == closed
        res[name] = {"ms": round(ms, 4), "tuples_per_s": n_in / (ms * 1e-3), "sum_equals_closed_form": ok,
                     "kernels_us": {k: round(v[0] / max(v[1], 1) * 1e3, 1)
                                    for k, v in sorted(kp.items(), key=lambda kv: -kv[1][0])[:5]}}
        log(f"S-largest workload, {name}: {ms:.3f} ms, sum ok {ok}")
    res["speedup_over_partitioned"] = round(res["partitioned_3way"]["ms"] / res["s_largest"]["ms"], 2)
    return res


def skew_path(mj, ctx):
    """Heavy keys (Sec. 1.2's skew): the power-law graph of the benchmark
    (2^24 edges over 2^20 vertices) with its out-degree cap at 4096, 65536
    and none (the largest vertex then holds about 1.2 million edges), under
    the planner's plan (direct-indexed tables) and under hashed tables.  A
    range or bucket crowded beyond one workgroup's share runs as several."""
    import numpy as np
    import torch
    from workloads import generators as G
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import brute
    n = 1 << 20
    res = {}
    for cap in (4096, 1 << 16, n - 1):
        log(f"skew: power-law graph, out-degree cap {cap}")
        F = G.powerlaw_friends(n, 1 << 24, 1234, cap=cap)
        Fd = torch.from_numpy(F).to("cuda")
        closed = brute.linear_closed_total(F, F, F)
        cnt = torch.empty(n, dtype=torch.int64, device="cuda")
        p = ctx.plan(mj.LINEAR, Fd, Fd, Fd, n)
        q = p.copy()
        q.algo = mj.ALGO_3WAY
        q.flags = (q.flags & ~mj.PLAN_DENSE_KEYS) | mj.PLAN_NO_DENSE
        q = ctx.plan(mj.LINEAR, Fd, Fd, Fd, n, planner="fixed", fixed=q)
        row = {"max_out_degree": int(np.bincount(F[:, 0].astype(np.int64), minlength=n).max())}
        for name, plan in (("direct_indexed", p), ("hashed", q)):
            ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
            ms, kp = time_and_profile(ctx, lambda: ctx.linear3_count(Fd, Fd, Fd, n, plan=plan, out=cnt,
                                                                     workspace=ws), 5)
            row[name] = {"ms": round(ms, 4), "tuples_per_s": 3 * F.shape[0] / (ms * 1e-3),
                         "sum_equals_closed_form": int(mj.as_u64(cnt).sum(dtype=np.uint64)) == closed,
                         "kernels_us": {k: round(v[0] / max(v[1], 1) * 1e3, 1)
                                        for k, v in sorted(kp.items(), key=lambda kv: -kv[1][0])[:5]}}
            log(f"skew cap {cap} {name}: {ms:.3f} ms")
            del ws
        res[f"cap_{cap}"] = row
        del Fd
    return res


def gather_path(mj, ctx, F, a_domain):
    """What bounds the per-range sums: the benchmark step on its input, and
    on the same edges sorted by (source, destination) -- the same join, with
    each range's gathered keys in order, so that consecutive lanes read
    neighbouring entries.  The kernels' times on the two orders show what
    locality of the random table reads is worth."""
    import numpy as np
    import torch
    res = {}
    for name, E in (("benchmark_order", F), ("sorted_by_source_destination",
                                              F[np.lexsort((F[:, 1], F[:, 0]))])):
        Ed = torch.from_numpy(np.ascontiguousarray(E)).to("cuda")
        p = ctx.plan(mj.LINEAR, Ed, Ed, Ed, a_domain)
        ws = torch.empty(p.workspace_bytes, dtype=torch.uint8, device="cuda")
        out = torch.empty(a_domain, dtype=torch.int64, device="cuda")
        ms, kp = time_and_profile(ctx, lambda: ctx.linear3_count(Ed, Ed, Ed, a_domain, plan=p, out=out,
                                                                   workspace=ws), 20, 3)
        res[name] = {"ms_per_step": round(ms, 4),
                     "kernels_us": {k: round(v[0] / max(v[1], 1) * 1e3, 1) for k, v in kp.items()
                                    if k.startswith("k_range") or "scatter" in k},
                     "sum": int(mj.as_u64(out).sum(dtype=np.uint64))}
        del ws, Ed
        log(f"gather locality, {name}: {ms:.4f} ms")
    res["same_counts"] = res["benchmark_order"]["sum"] == res["sorted_by_source_destination"]["sum"]
    return res


def fm_exact_sizes(F, a_vals):
    """|D(a)| for the sampled a, by set operations on the edge list (for the
    accuracy figure of the distinct-count path)."""
    import numpy as np
    order = np.argsort(F[:, 0], kind="stable")
    src, dst = F[order, 0], F[order, 1]
    n_v = int(F.max()) + 1
    off = np.searchsorted(src, np.arange(n_v + 1, dtype=np.uint64))

    def nbrs(vs):
        lo, hi = off[vs], off[vs + 1]
        lens = (hi - lo).astype(np.int64)
        if lens.sum() == 0:
            return np.zeros(0, dtype=np.int64)
        first = np.repeat(lo.astype(np.int64) - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
        return np.unique(dst[first + np.arange(lens.sum())]).astype(np.int64)
    return [int(nbrs(nbrs(nbrs(np.array([a], dtype=np.int64)))).size) for a in a_vals]


def fm_path(mj, ctx, F, Fd, a_domain):
    """Flajolet-Martin distinct count of D per A (the non-decomposable
    aggregate of Sec. 1 / Sec. 6) on the power-law graph: one call sketches
    T per C, S per B and R per A and writes an estimate per A."""
    import numpy as np
    import torch
    log("distinct count (Flajolet-Martin) on the power-law graph")
    n = F.shape[0]
    sk = torch.empty((a_domain, 16), dtype=torch.int32, device="cuda")
    est = torch.empty(a_domain, dtype=torch.float64, device="cuda")
    fn = lambda: ctx.linear3_distinct(Fd, Fd, Fd, a_domain, seed=0x5EED, sketch=sk, est=est)
    ms, kp = time_and_profile(ctx, fn, 5, 2, 3)
    kern = {k: (v[0] / max(v[1], 1), v[1]) for k, v in kp.items()}     # (ms per launch, launches per call)
    e = est.cpu().numpy()
    rng = np.random.default_rng(11)
    outdeg = np.bincount(F[:, 0], minlength=a_domain)
    cand = np.flatnonzero(outdeg > 0)
    sample = rng.choice(cand, size=48, replace=False)
    exact = np.array(fm_exact_sizes(F, sample))
    big = exact >= 1000
    ratio = e[sample[big]] / exact[big]
    # bytes the path must move at least: R, S, T read once (8 B per tuple),
    # one 64-byte sketch per distinct C and per distinct B written and read
    # once, and the sketches and estimates per A written
    n_keys = int(np.unique(F[:, 0]).size)
    alg = 3 * 8 * n + 2 * 2 * 64 * n_keys + 72 * a_domain
    ach = alg / (ms * 1e-3) / 1e9
    res = {"ms": round(ms, 3), "tuples_per_s": 3 * n / (ms * 1e-3),
           "path_hbm": {"algorithmic_bytes": alg, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)},
           "est_over_exact": {"sampled_a": int(big.sum()), "median": round(float(np.median(ratio)), 4),
                              "p10": round(float(np.percentile(ratio, 10)), 4),
                              "p90": round(float(np.percentile(ratio, 90)), 4)},
           "kernels_us": {k: [round(v[0] * 1e3, 1), round(v[1], 2)]
                          for k, v in sorted(kern.items(), key=lambda kv: -kv[1][0] * kv[1][1])[:8]}}
    log(f"distinct count: {ms:.3f} ms, est/exact median {res['est_over_exact']['median']}")
    return res


def emit_path(mj, ctx, F, Fd):
    """The linear join's result written out (every (a, b, c, d) tuple of
    F |x| F |x| F, 4.36e9 of them, 70 GB, in nested-loop order) in one call;
    the total is checked against the closed form and sampled tuples against
    the edge list."""
    import numpy as np
    import torch
    n = F.shape[0]
    indeg = np.bincount(F[:, 1], minlength=1 << 20).astype(np.int64)
    outdeg = np.bincount(F[:, 0], minlength=1 << 20).astype(np.int64)
    closed = int((indeg[F[:, 0]] * outdeg[F[:, 1]]).sum())
    log(f"materialised output: {closed} tuples ({closed * 16 / 2**30:.1f} GiB)")
    total = torch.empty(1, dtype=torch.int64, device="cuda")
    out = torch.empty((closed, 4), dtype=torch.int32, device="cuda")
    fn = lambda: ctx.linear3_materialize(Fd, Fd, Fd, out=out, total=total)
    ms, kern = time_and_profile(ctx, fn, 3, 1, 2)
    got_total = int(total.item())
    rng = np.random.default_rng(3)
    pos = torch.from_numpy(rng.integers(0, closed, 2000)).to("cuda")
    smp = out[pos].cpu().numpy().view(np.uint32)
    del out
    torch.cuda.empty_cache()
    enc = lambda x, y: (x.astype(np.uint64) << np.uint64(32)) | y.astype(np.uint64)
    edges = enc(F[:, 0], F[:, 1])
    valid = bool(np.isin(enc(smp[:, 0], smp[:, 1]), edges).all() and
                 np.isin(enc(smp[:, 1], smp[:, 2]), edges).all() and
                 np.isin(enc(smp[:, 2], smp[:, 3]), edges).all())
    k_ms = kern.get("k_emit", (0.0, 0))[0]                           # ms per call, all chunks
    res = {"ms": round(ms, 3), "result_tuples": got_total, "total_equals_closed_form": got_total == closed,
           "sampled_tuples_are_join_results": valid,
           "result_tuples_per_s": got_total / (ms * 1e-3), "input_tuples_per_s": 3 * n / (ms * 1e-3),
           "kernels_ms_per_call": {k: round(v[0], 3) for k, v in
                                   sorted(kern.items(), key=lambda kv: -kv[1][0])[:6]}}
    if k_ms:
        nbytes = 16 * got_total                       # every result tuple written once
        ach = nbytes / (k_ms * 1e-3) / 1e9
        res["roofline"] = {"bound": "hbm", "kernel": "k_emit", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes": nbytes,
                           "ms_per_call": round(k_ms, 3)}
    log(f"materialised output: {ms:.2f} ms, total ok {got_total == closed}, samples ok {valid}")
    return res


LEGS = ("cascade", "small", "fm", "emit", "star", "slarge", "skew", "triangle", "batch", "planner", "gather")
DEFAULT_LEGS = ("small", "skew", "triangle", "batch", "planner", "gather")
OWN_WORKLOAD_LEGS = ("small", "star", "slarge", "skew", "triangle", "batch", "planner")


def child_paths(legs):
    """The named paths, each as `bench.py --only LEG` in a child process."""
    import subprocess
    out = {}
    for leg in legs:
        log(f"path {leg} (child process)")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--only", leg, "--no-cpu"],
                           capture_output=True, text=True, timeout=1200)
        lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
        if r.returncode == 0 and lines:
            out.update(json.loads(lines[-1])[leg])
        else:
            out[leg] = {"error": f"exit status {r.returncode}", "stderr_tail": r.stderr[-400:]}
    return out


def extra_paths(mj, ctx, F, Fd, a_domain, plan, ms_3way, only=None):
    """The other paths of the method, each on its own workload (all of them,
    or the one named by `only`)."""
    out = {}
    if only in (None, "cascade", "small"):
        out.update(linear_paths(mj, ctx, F, Fd, a_domain, plan, ms_3way, only))
    if only in (None, "fm"):
        out["distinct_fm"] = fm_path(mj, ctx, F, Fd, a_domain)
    if only in (None, "emit"):
        out["materialised"] = emit_path(mj, ctx, F, Fd)
    if only in (None, "star"):
        out["star"] = star_path(mj, ctx)
    if only in (None, "slarge"):
        out["s_largest"] = slarge_path(mj, ctx)
    if only in (None, "skew"):
        out["skew"] = skew_path(mj, ctx)
    if only in (None, "gather"):
        out["gather_locality"] = gather_path(mj, ctx, F, a_domain)
    if only in (None, "triangle"):
        out["triangle_rmat22"] = triangle_path(mj, ctx)
    if only in (None, "batch"):
        out["batch_512"] = batch_path(mj, ctx)
    if only in (None, "planner"):
        out["planner"] = planner_path(ctx)
    return out


def linear_paths(mj, ctx, F, Fd, a_domain, plan, ms_3way, only=None):
    """The cascade on the benchmarked input, and the small uniform input."""
    import numpy as np
    import torch
    from workloads import generators as G
    out = {}
    if only in (None, "cascade"):
        out["cascade_linear"] = cascade_path(mj, ctx, Fd, F.shape[0], a_domain, plan, ms_3way)
    if only == "cascade":
        return out
    # small uniform linear workload (65,536 tuples, keys in [0, 4096))
    Fs = G.linear_small()
    Fsd = torch.from_numpy(Fs.view(np.int32)).to("cuda")
    ps = ctx.plan(mj.LINEAR, Fsd, Fsd, Fsd, 4096)
    ws = torch.empty(ps.workspace_bytes, dtype=torch.uint8, device="cuda")
    cs = torch.empty(4096, dtype=torch.int64, device="cuda")
    ms_s = time_call(lambda: ctx.linear3_count(Fsd, Fsd, Fsd, 4096, plan=ps, out=cs, workspace=ws), 20, 3)
    ms_sc = time_call(lambda: ctx.cascade2_count(mj.LINEAR, Fsd, Fsd, Fsd, 4096, plan=ps, out=cs,
                                                 workspace=ws), 20, 3)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import brute
    closed = brute.linear_closed_total(Fs, Fs, Fs)
    got_c = int(mj.as_u64(cs).sum(dtype=np.uint64))
    ctx.linear3_count(Fsd, Fsd, Fsd, 4096, plan=ps, out=cs, workspace=ws)
    got_3 = int(mj.as_u64(cs).sum(dtype=np.uint64))
    out["linear_small"] = {"ms_3way": round(ms_s, 4), "ms_cascade": round(ms_sc, 4),
                           "tuples_per_s_3way": 3 * Fs.shape[0] / (ms_s * 1e-3),
                           "tuples_per_s_cascade": 3 * Fs.shape[0] / (ms_sc * 1e-3),
                           "sums_equal_closed_form": got_3 == closed and got_c == closed}
    del ws
    return out


def cascade_path(mj, ctx, Fd, n, a_domain, plan, ms_3way):
    """The cascade of binary joins on the benchmarked input (Sec. 6.3)."""
    import torch
    log("cascade on the power-law graph")
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(a_domain, dtype=torch.int64, device="cuda")
    ms_c = time_call(lambda: ctx.cascade2_count(mj.LINEAR, Fd, Fd, Fd, a_domain, plan=plan,
                                                out=cnt, workspace=ws), 3)
    del ws
    return {"ms": round(ms_c, 3), "tuples_per_s": 3 * n / (ms_c * 1e-3),
            "intermediate_pairs": plan.join2_size,
            "speedup_3way_over_cascade": round(ms_c / ms_3way, 2) if ms_3way else None}


def triangle_path(mj, ctx):
    """The cyclic join on the R-MAT scale-22 graph (Sec. 5): the general
    join at shares 1 / 4 / 16, and the planner's choice."""
    import torch
    from workloads import generators as G
    log("generating R-MAT scale 22 (2^26 undirected edges)")
    E = G.triangle_rmat()
    Ed = torch.from_numpy(E).to("cuda")
    golden = None
    gp = os.path.join(ROOT, "tests", "golden", "triangle_rmat22.json")
    if os.path.exists(gp):
        golden = json.load(open(gp))["total"]
    tri = {}
    tot = torch.empty(1, dtype=torch.int64, device="cuda")
    # the general join's list work: each S tuple (b, c) is handled once, by
    # the shorter of R's list of b and T's list of c, so it visits
    # sum over S of min(deg b, deg c) list elements (R = S = T symmetric)
    import numpy as np
    deg = np.bincount(E[:, 0].astype(np.int64))
    visits = int(np.minimum(deg[E[:, 0].astype(np.int64)], deg[E[:, 1].astype(np.int64)]).sum(dtype=np.int64))
    del deg
    tri["general_join_list_elements_visited"] = visits
    # shares 1, 4, 16 and the menu 8, 16, 32 of the workload statement (the
    # least number of A-slices of a hub list)
    for share in (0, 2, 3, 4, 5):
        p = mj.Plan()
        p.log2_share = share
        p.seed = 0x1B873593
        pt = ctx.plan(mj.TRIANGLE, Ed, Ed, Ed, 0, planner="fixed", fixed=p)
        ws = torch.empty(pt.workspace_bytes, dtype=torch.uint8, device="cuda")
        ms_t, kp = time_and_profile(ctx, lambda: ctx.triangle3_count(Ed, Ed, Ed, plan=pt, out=tot, workspace=ws),
                                    2, 1, 1)
        got = int(mj.as_u64(tot)[0])
        join_ms = sum(v[0] for k, v in kp.items() if k.startswith("k_tri_light") or k.startswith("k_tri_heavy"))
        tri[f"share_{1 << share}"] = {
            "ms": round(ms_t, 2), "tuples_per_s": 3 * E.shape[0] / (ms_t * 1e-3),
            "list_elements_per_s_in_join_kernels": visits / (join_ms * 1e-3) if join_ms else None,
            "total": got, "triangles": got // 6,
            "matches_oracle_total": (got == golden) if golden is not None else None,
            "kernels_ms_per_call": {k: round(v[0], 3) for k, v in sorted(kp.items(), key=lambda kv: -kv[1][0])[:8]}}
        log(f"cyclic share {1 << share}: {ms_t:.1f} ms total {got}")
        del ws
    # the planner's choice: it finds R = S = T symmetric and simple and picks
    # the degree-oriented join (each triangle once)
    t0 = time.perf_counter()
    po = ctx.plan(mj.TRIANGLE, Ed, Ed, Ed)
    plan_ms = (time.perf_counter() - t0) * 1e3
    ws = torch.empty(po.workspace_bytes, dtype=torch.uint8, device="cuda")
    ms_o, kp = time_and_profile(ctx, lambda: ctx.triangle3_count(Ed, Ed, Ed, plan=po, out=tot, workspace=ws), 3)
    got = int(mj.as_u64(tot)[0])
    tri["planned_oriented"] = {
        "algo": int(po.algo), "plan_ms": round(plan_ms, 1), "ms": round(ms_o, 2),
        "tuples_per_s": 3 * E.shape[0] / (ms_o * 1e-3), "total": got, "triangles": got // 6,
        "matches_oracle_total": (got == golden) if golden is not None else None,
        "speedup_over_share_1": round(tri["share_1"]["ms"] / ms_o, 2),
        "kernels_ms_per_call": {k: round(v[0], 3) for k, v in sorted(kp.items(), key=lambda kv: -kv[1][0])[:8]}}
    log(f"cyclic, planned (oriented): {ms_o:.1f} ms total {got}")
    del ws, Ed, E
    return tri


def planner_path(ctx, n=300):
    """Learned vs plain planners on held-out join instances (sizes 10^3 to
    10^5.5, the families the network was trained on, other seeds): the
    summed measured time of each planner's plans, with counts checked."""
    import numpy as np
    from paper_1905_13376_amd import learned
    log(f"planner comparison on {n} held-out instances")
    pl = learned.use_shipped(ctx)
    rows = [learned.label_instance(ctx, x) for x in learned.planner_instances(n, 7_000_000, 3.0, 5.5)]
    D = learned.rows_to_arrays(rows)
    res = learned.evaluate(pl, D)
    res["counts_exact_all_plans"] = bool(D["counts_exact"].all())
    res["plan_ms_median_analytic"] = round(float(np.median(D["plan_ms"])), 3)
    ctx.set_planner(None)
    return res


def batch_path(mj, ctx):
    """512 independent joins of uneven size (half linear, half cyclic; edge
    counts log-uniform in [10^3, 10^6]; uniform or Zipf(1.1) degrees): one
    mj_batch_count call (its kernel launches counted), its HIP-graph replay,
    and the same joins one call each for comparison."""
    import numpy as np
    import torch
    from workloads import generators as G
    log("generating the batch of 512 joins")
    inst = G.batch_instances()
    joins, keep = [], []
    for x in inst:
        Fd = torch.from_numpy(np.ascontiguousarray(x["F"]).view(np.int32)).to("cuda")
        keep.append(Fd)
        if x["kind"] == "linear":
            joins.append((mj.LINEAR, Fd, Fd, Fd, x["n"]))
        else:
            joins.append((mj.TRIANGLE, Fd, Fd, Fd, 0))
    tuples = 3 * sum(int(k.shape[0]) for k in keep)
    t0 = time.perf_counter()
    plans = [ctx.plan(k, R, S, T, a) for (k, R, S, T, a) in joins]
    plan_ms = (time.perf_counter() - t0) * 1e3
    b = ctx.batch(joins, plans=plans)
    ms_batch = time_call(lambda: b.run(), 3)
    _, kp = time_and_profile(ctx, lambda: b.run(), 1, 1)       # launches of one call
    launches = int(round(sum(v[1] for v in kp.values())))
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    b.run()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        b.run(stream=s)
    ms_graph = time_call(lambda: g.replay(), 3)
    outs_b = [mj.as_u64(o).copy() for o in b.outs]

    # one call per join (same plans), for comparison
    ws = torch.empty(max(p.workspace_bytes for p in plans), dtype=torch.uint8, device="cuda")
    outs = [torch.empty(max(a, 1), dtype=torch.int64, device="cuda") for (_, _, _, _, a) in joins]

    def seq():
        for (k, R, S, T, a), p, o in zip(joins, plans, outs):
            if k == mj.LINEAR:
                ctx.linear3_count(R, S, T, a, plan=p, out=o, workspace=ws)
            else:
                ctx.triangle3_count(R, S, T, plan=p, out=o, workspace=ws)
    ms_seq = time_call(seq, 2)
    same = all(np.array_equal(mj.as_u64(o)[:max(a, 1) if k == mj.LINEAR else 1][:len(ob)], ob)
               for (k, _, _, _, a), o, ob in zip(joins, outs, outs_b))
    log(f"batch of 512: {ms_batch:.2f} ms (graph {ms_graph:.2f} ms), one call per join {ms_seq:.2f} ms")
    return {"joins": len(joins), "input_tuples": tuples, "ms_batch": round(ms_batch, 3),
            "kernel_launches_per_call": launches,
            "ms_graph_replay": round(ms_graph, 3), "ms_one_call_per_join": round(ms_seq, 3),
            "tuples_per_s_batch": tuples / (ms_batch * 1e-3),
            "tuples_per_s_graph_replay": tuples / (ms_graph * 1e-3), "plan_ms_total": round(plan_ms, 1),
            "batch_equals_per_join_calls": bool(same)}


if __name__ == "__main__":
    main()
