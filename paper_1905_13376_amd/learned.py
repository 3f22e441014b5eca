"""Learned planner: a small network over degree sketches that predicts the
intermediate and output cardinalities of a join and chooses its plan among
the three-way join, the cascade, the star plans, the degree-oriented cyclic
join and the S-largest form (and the share on A of a cyclic join).

Everything numeric runs in libmj's kernels (k_deg_hist / k_sketch_features
for the sketch, k_mlp_fwd / k_mlp_loss / k_mlp_bwd / k_mlp_adamw for the
network); this module holds the parameter buffer, the training loop's
control flow, and the data pipeline that generates join instances, times
their candidate plans on the device and labels them.

    python -m paper_1905_13376_amd.learned label --count N --seed S --lo 3 --hi 5 --out rows.npz
    python -m paper_1905_13376_amd.learned train --train rows.npz ... --test heldout.npz \\
        --out paper_1905_13376_amd/planner_weights.npy --report paper_1905_13376_amd/planner_eval.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import _lib as L

IN, H, OUT = 100, 64, 11
SHAPES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (OUT, H)), ("b3", (OUT,))]
P = sum(int(np.prod(s)) for _, s in SHAPES)
SHARES = (0, 2, 4)                     # log2 of the shares 1, 4, 16 (the share head's classes)
CASCADE_CAP = 1 << 28                  # the planner never materialises more pairs
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "planner_weights.npy")


class LearnedPlanner:
    """The network's parameter buffer (device) and its training loop."""

    def __init__(self, ctx, device="cuda"):
        self.ctx = ctx
        self.buf = torch.zeros(L.mlp_param_bytes(), dtype=torch.uint8, device=device)
        self.master = self.buf[: 4 * P * 4].view(torch.float32)[:P]
        self.step = 0

    def init_weights(self, seed=0):
        rng = np.random.default_rng(seed)
        parts = []
        for name, shape in SHAPES:
            if name.startswith("W"):
                parts.append(rng.normal(0.0, math.sqrt(2.0 / shape[1]), size=shape).ravel())
            else:
                parts.append(np.zeros(int(np.prod(shape))))
        self.set_masters(np.concatenate(parts).astype(np.float32))

    def set_masters(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.shape == (P,)
        full = self.buf[: 4 * P * 4].view(torch.float32)
        full.zero_()                                   # masters, grads, Adam m, v
        self.master.copy_(torch.from_numpy(w))
        L.mlp_sync(self.ctx, self.buf)
        self.step = 0

    def masters(self) -> dict:
        w = self.master.detach().cpu().numpy()
        out, o = {}, 0
        for name, shape in SHAPES:
            k = int(np.prod(shape))
            out[name] = w[o:o + k].reshape(shape).copy()
            o += k
        return out

    def save(self, path=WEIGHTS):
        np.save(path, self.master.detach().cpu().numpy())

    def load(self, path=WEIGHTS):
        self.set_masters(np.load(path, allow_pickle=False))

    def predict(self, X: torch.Tensor) -> torch.Tensor:
        Y = torch.empty((X.shape[0], OUT), dtype=torch.float32, device=X.device)
        L.mlp_forward(self.ctx, self.buf, X.contiguous(), Y)
        return Y

    def train(self, X, targets, plan_label, share_label, epochs=60, batch=256, lr=2e-3,
              wd=1e-4, seed=0, log=None):
        """Mini-batch AdamW on the device; returns the mean loss per epoch."""
        n = X.shape[0]
        gen = torch.Generator(device="cpu").manual_seed(seed)
        ws = torch.empty(L.mlp_workspace_bytes(batch), dtype=torch.uint8, device=X.device)
        loss = torch.zeros(1, dtype=torch.float32, device=X.device)
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(n, generator=gen).to(X.device)
            loss.zero_()
            nb = 0
            for b0 in range(0, n, batch):
                idx = perm[b0:b0 + batch]
                L.mlp_grads(self.ctx, self.buf, X[idx].contiguous(), targets[idx].contiguous(),
                            plan_label[idx].contiguous(), share_label[idx].contiguous(), loss, ws)
                self.step += 1
                L.mlp_adamw(self.ctx, self.buf, lr, wd, self.step)
                nb += 1
            hist.append(float(loss.item()) / nb)
            if log and (ep % 10 == 0 or ep == epochs - 1):
                log(f"epoch {ep}: loss {hist[-1]:.4f}")
        return hist


def use_shipped(ctx, path=WEIGHTS):
    """Load the network trained by this module (planner_weights.npy) and
    make it the context's learned planner; returns the LearnedPlanner,
    which must stay alive while plans are made."""
    pl = LearnedPlanner(ctx)
    pl.load(path)
    ctx.set_planner(pl.buf)
    return pl


# ---------------------------------------------------------------- data
# plan classes of the network's plan head, in mj_algo order
PLANS = ("3way", "cascade", "star", "star_cascade", "oriented", "slarge")
COLS = PLANS + ("share0", "share2", "share4")      # measured-time columns


def planner_instances(count, base_seed, lo_exp=3.0, hi_exp=5.0):
    """Join instances shaped like the benchmark families: linear joins on
    uniform pairs of varying selectivity, on power-law friends graphs, on
    star schemas (small dimension relations) and on S-largest schemas
    (dimension relations beyond the star plans); cyclic joins on G(n, m),
    Chung-Lu and R-MAT graphs.  Each instance holds R, S, T (one relation
    for all three unless a schema) and a (the A domain; 0 for cyclic)."""
    from workloads import generators as G
    out = []
    for k in range(count):
        seed = base_seed + k
        g = np.random.default_rng(seed)
        m = int(round(10 ** g.uniform(lo_exp, hi_exp)))
        fam = int(g.integers(0, 8))
        if fam == 0:       # uniform, mean degree 1..64 (selectivity varies widely)
            n = max(16, int(m / (2 ** g.uniform(0, 6))))
            F = G.uniform_pairs(m, n, seed, dtype=np.int32)
            out.append(dict(kind="linear", R=F, S=F, T=F, a=n))
        elif fam == 1:     # uniform over a large domain: tiny intermediate
            n = int(m * 2 ** g.uniform(2, 8))
            F = G.uniform_pairs(m, n, seed, dtype=np.int32)
            out.append(dict(kind="linear", R=F, S=F, T=F, a=n))
        elif fam == 2:     # power-law friends graph, mean degree 16
            n = max(64, m // 16)
            F = G.powerlaw_friends(n, m, seed, cap=min(4096, n - 1))
            out.append(dict(kind="linear", R=F, S=F, T=F, a=n))
        elif fam == 3:
            n = max(64, m // 16)
            F = G.gnm_symmetric(n, m, seed)
            out.append(dict(kind="triangle", R=F, S=F, T=F, a=0))
        elif fam == 4:
            n = max(64, m // 16)
            F = G.chung_lu_symmetric(n, m, seed, cap=min(4096, n - 1))
            out.append(dict(kind="triangle", R=F, S=F, T=F, a=0))
        elif fam == 5:
            scale = max(6, int(round(math.log2(max(64, m // 16)))))
            F = G.rmat_symmetric(scale, min(m, (1 << scale) * 16), seed)
            out.append(dict(kind="triangle", R=F, S=F, T=F, a=0))
        elif fam == 6:     # star schema: dimension relations of 64..4096 tuples
            kr, kt = (int(2 ** g.uniform(6, 12)) for _ in range(2))
            a = int(2 ** g.uniform(4, 12))
            R, S, T = G.star_schema(n_fact=m, k_r=kr, k_t=kt, a_domain=a, seed=seed)
            out.append(dict(kind="linear", R=R, S=S, T=T, a=a))
        else:              # S-largest schema: dimension relations of 2^12..m/4 tuples
            hi = max(12.5, math.log2(max(m // 4, 1 << 12)))
            kr, kt = (int(2 ** g.uniform(12, hi)) for _ in range(2))
            a = int(2 ** g.uniform(6, 14))
            R, S, T = G.star_schema(n_fact=m, k_r=kr, k_t=kt, a_domain=a, seed=seed)
            out.append(dict(kind="linear", R=R, S=S, T=T, a=a))
    return out


def _time(fn, reps=2):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def label_instance(ctx, inst):
    """Features, exact cardinalities and measured times of every plan the
    instance is eligible for (infinity for the others); the plan label is
    the fastest measured plan (mj_algo value), the share label the fastest
    share of the cyclic three-way join.  Every plan's count is checked
    against the three-way join's."""
    kind = L.LINEAR if inst["kind"] == "linear" else L.TRIANGLE
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).to("cuda")
    same = inst["R"] is inst["S"] and inst["S"] is inst["T"]
    Rd = dev(inst["R"])
    Sd, Td = (Rd, Rd) if same else (dev(inst["S"]), dev(inst["T"]))
    a = inst["a"]
    feat = ctx.sketch(kind, Rd, Sd, Td)
    t0 = time.perf_counter()
    plan = ctx.plan(kind, Rd, Sd, Td, a)
    plan_ms = (time.perf_counter() - t0) * 1e3
    n_out = max(a, 1) if kind == L.LINEAR else 1
    out = torch.empty(n_out, dtype=torch.int64, device="cuda")
    times = {c: float("inf") for c in COLS}
    got = {}

    def run(name, p, reps=2):
        ws = ctx.workspace(p.workspace_bytes, Rd.device)
        if kind == L.LINEAR:
            if p.algo in (L.ALGO_CASCADE, L.ALGO_STAR_CASCADE):
                fn = lambda: ctx.cascade2_count(L.LINEAR, Rd, Sd, Td, a, plan=p, out=out, workspace=ws)
            else:
                fn = lambda: ctx.linear3_count(Rd, Sd, Td, a, plan=p, out=out, workspace=ws)
        elif p.algo == L.ALGO_CASCADE:
            fn = lambda: ctx.cascade2_count(L.TRIANGLE, Rd, Sd, Td, plan=p, out=out, workspace=ws)
        else:
            fn = lambda: ctx.triangle3_count(Rd, Sd, Td, plan=p, out=out, workspace=ws)
        times[name] = _time(fn, reps)
        got[name] = int(L.as_u64(out[:max(a, 1)] if kind == L.LINEAR else out).sum(dtype=np.uint64))

    def variant(algo, **fields):
        q = plan.copy()
        q.algo = algo
        for k, v in fields.items():
            setattr(q, k, v)
        return q

    if kind == L.LINEAR:
        run("3way", variant(L.ALGO_3WAY))
        if plan.join2_size <= CASCADE_CAP:
            run("cascade", variant(L.ALGO_CASCADE))
        if plan.est_ms_star > 0.0:
            run("star", variant(L.ALGO_STAR))
        if plan.est_ms_star_cascade > 0.0:
            run("star_cascade", variant(L.ALGO_STAR_CASCADE))
        if plan.est_ms_slarge > 0.0:
            lr, lt, _ = L.slarge_buckets(plan.n_r, plan.n_s, plan.n_t)
            run("slarge", variant(L.ALGO_SLARGE, log2_nb=lr, log2_nc=lt))
        ref = got["3way"]
    else:
        for k in SHARES:
            run(f"share{k}", variant(L.ALGO_3WAY, log2_share=k), 1)
        times["3way"] = min(times[f"share{k}"] for k in SHARES)
        ref = got["share0"]
        if plan.join2_size <= CASCADE_CAP:
            run("cascade", variant(L.ALGO_CASCADE), 1)
        if plan.flags & L.PLAN_SYMMETRIC_SIMPLE:
            run("oriented", variant(L.ALGO_ORIENTED), 1)
    exact = all(v == ref for v in got.values())
    plan_label = int(np.argmin([times[c] for c in PLANS]))
    share_label = int(np.argmin([times[f"share{k}"] for k in SHARES])) if kind == L.TRIANGLE else -1
    return dict(kind=kind, features=feat, join2=int(plan.join2_size), out=ref,
                times=np.array([times[c] for c in COLS], dtype=np.float64),
                plan_label=plan_label, share_label=share_label,
                analytic_algo=int(plan.algo), analytic_share=int(plan.log2_share), plan_ms=plan_ms,
                counts_exact=exact, n=int(Rd.shape[0] + (0 if same else Sd.shape[0] + Td.shape[0])))


def rows_to_arrays(rows):
    """Labelled instances as one dict of arrays (the form evaluate() takes)."""
    return dict(features=torch.stack([r["features"] for r in rows]).cpu().numpy(),
                join2=np.array([r["join2"] for r in rows], dtype=np.float64),
                out=np.array([r["out"] for r in rows], dtype=np.float64),
                times=np.stack([r["times"] for r in rows]),
                kind=np.array([r["kind"] for r in rows], dtype=np.int32),
                plan_label=np.array([r["plan_label"] for r in rows], dtype=np.int32),
                share_label=np.array([r["share_label"] for r in rows], dtype=np.int32),
                analytic_algo=np.array([r["analytic_algo"] for r in rows], dtype=np.int32),
                analytic_share=np.array([r["analytic_share"] for r in rows], dtype=np.int32),
                plan_ms=np.array([r["plan_ms"] for r in rows], dtype=np.float64),
                counts_exact=np.array([r["counts_exact"] for r in rows], dtype=bool),
                n=np.array([r["n"] for r in rows], dtype=np.int64))


def save_rows(rows, path):
    np.savez_compressed(path, **rows_to_arrays(rows))


def load_rows(paths):
    parts = [np.load(p, allow_pickle=False) for p in paths]
    return {k: np.concatenate([q[k] for q in parts]) for k in parts[0].files}


def as_tensors(D, device="cuda"):
    X = torch.from_numpy(np.ascontiguousarray(D["features"], dtype=np.float32)).to(device)
    targets = torch.from_numpy(np.stack([np.log2(1 + D["join2"]), np.log2(1 + D["out"])], 1)
                               .astype(np.float32)).to(device)
    pl = torch.from_numpy(D["plan_label"].astype(np.int32)).to(device)
    sl = torch.from_numpy(D["share_label"].astype(np.int32)).to(device)
    return X, targets, pl, sl


def nearest_share(k):
    """The timed share class closest to log2 share k."""
    return min(SHARES, key=lambda c: (abs(c - k), c))


def plan_time(times_row, kind, algo, share):
    """Measured time of a plan (the three-way plan of a cyclic join at the
    given share)."""
    if kind == L.TRIANGLE and algo == L.ALGO_3WAY:
        return times_row[COLS.index(f"share{share}")]
    return times_row[algo]


def evaluate(planner, D):
    """Held-out comparison of the learned plans with the analytic plans, the
    fixed plans and the best measured plan (regret), plus cardinality
    q-errors.  The network's plan is its largest logit among the plans the
    instance was eligible for (measured: finite time)."""
    X = torch.from_numpy(np.ascontiguousarray(D["features"], dtype=np.float32)).to("cuda")
    Y = planner.predict(X).cpu().numpy()
    T = D["times"]
    tot = {"learned": 0.0, "analytic": 0.0, "always_3way": 0.0, "always_cascade": 0.0, "best": 0.0}
    agree = {"learned": 0, "analytic": 0}
    qI, qO = [], []
    for i, y in enumerate(Y):
        kind = int(D["kind"][i])
        t = T[i]
        elig = np.isfinite(t[:len(PLANS)])
        logits = np.where(elig, y[2:2 + len(PLANS)], -np.inf)
        algo = int(np.argmax(logits))
        share = SHARES[int(np.argmax(y[2 + len(PLANS):]))]
        best = float(np.min(t[np.isfinite(t)]))
        tl = plan_time(t, kind, algo, share)
        ta = plan_time(t, kind, int(D["analytic_algo"][i]), nearest_share(int(D["analytic_share"][i])))
        tot["learned"] += tl
        tot["analytic"] += ta
        tot["always_3way"] += plan_time(t, kind, L.ALGO_3WAY, SHARES[0])
        tot["always_cascade"] += t[L.ALGO_CASCADE] if np.isfinite(t[L.ALGO_CASCADE]) else t[L.ALGO_3WAY]
        tot["best"] += best
        agree["learned"] += tl <= best
        agree["analytic"] += ta <= best
        qI.append(2 ** abs(float(y[0]) - math.log2(1 + D["join2"][i])))
        qO.append(2 ** abs(float(y[1]) - math.log2(1 + D["out"][i])))
    res = {k: round(v, 3) for k, v in tot.items()}
    res["regret_learned"] = round(tot["learned"] / tot["best"], 4)
    res["regret_analytic"] = round(tot["analytic"] / tot["best"], 4)
    res["best_plan_chosen_learned"] = int(agree["learned"])
    res["best_plan_chosen_analytic"] = int(agree["analytic"])
    res["qerror_join2_median"] = round(float(np.median(qI)), 3)
    res["qerror_join2_p95"] = round(float(np.percentile(qI, 95)), 3)
    res["qerror_out_median"] = round(float(np.median(qO)), 3)
    res["qerror_out_p95"] = round(float(np.percentile(qO, 95)), 3)
    res["instances"] = int(len(Y))
    res["plan_label_counts"] = {PLANS[k]: int((D["plan_label"] == k).sum()) for k in range(len(PLANS))}
    return res


def label(ctx, count, seed, lo_exp, hi_exp, path, log=None):
    """Label `count` instances (seeds seed..seed+count-1) and save them."""
    rows = []
    t0 = time.time()
    for i, x in enumerate(planner_instances(count, seed, lo_exp, hi_exp)):
        rows.append(label_instance(ctx, x))
        if log and (i + 1) % 250 == 0:
            log(f"{i + 1}/{count} instances labelled ({time.time() - t0:.0f} s)")
    save_rows(rows, path)
    return rows


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    la = sub.add_parser("label", help="label instances and save them (npz)")
    la.add_argument("--count", type=int, required=True)
    la.add_argument("--seed", type=int, required=True)
    la.add_argument("--lo", type=float, default=3.0)
    la.add_argument("--hi", type=float, default=5.0)
    la.add_argument("--out", required=True)
    tr = sub.add_parser("train", help="train on labelled sets, evaluate on a held-out set")
    tr.add_argument("--train", nargs="+", required=True)
    tr.add_argument("--test", required=True)
    tr.add_argument("--epochs", type=int, default=60)
    tr.add_argument("--out", default=WEIGHTS)
    tr.add_argument("--report", default=None)
    args = ap.parse_args()

    def log(m):
        print(f"[learned] {m}", file=sys.stderr, flush=True)
    ctx = L.Context()
    if args.cmd == "label":
        label(ctx, args.count, args.seed, args.lo, args.hi, args.out, log)
        return
    D = load_rows(args.train)
    X, targets, pl, sl = as_tensors(D)
    planner = LearnedPlanner(ctx)
    planner.init_weights(seed=0)
    hist = planner.train(X, targets, pl, sl, epochs=args.epochs, log=log)
    planner.save(args.out)
    rep = evaluate(planner, load_rows([args.test]))
    rep["train_loss_first_last"] = [round(hist[0], 4), round(hist[-1], 4)]
    rep["train_instances"] = int(X.shape[0])
    rep["train_plan_label_counts"] = {PLANS[k]: int((D["plan_label"] == k).sum()) for k in range(len(PLANS))}
    rep["counts_exact_all_plans"] = bool(D["counts_exact"].all())
    log(json.dumps(rep))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
