"""Learned planner: a small network over degree sketches that predicts the
intermediate and output cardinalities of a join and chooses between the
three-way join and the cascade (and the share on A of a cyclic join).

Everything numeric runs in libmj's kernels (k_deg_hist / k_sketch_features
for the sketch, k_mlp_fwd / k_mlp_loss / k_mlp_bwd / k_mlp_adamw for the
network); this module holds the parameter buffer, the training loop's
control flow, and the data pipeline that generates join instances, times
their candidate plans on the device and labels them.

    python -m paper_1905_13376_amd.learned --n-train 12000 --n-test 1000 \\
        --out paper_1905_13376_amd/planner_weights.npy --report planner_eval.json
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

IN, H, OUT = 100, 64, 7
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
def planner_instances(count, base_seed, lo_exp=3.0, hi_exp=5.0):
    """Join instances shaped like the benchmark families, at small sizes:
    linear joins on uniform pairs of varying selectivity and on power-law
    friends graphs; cyclic joins on G(n, m), Chung-Lu and R-MAT graphs."""
    from workloads import generators as G
    out = []
    for k in range(count):
        seed = base_seed + k
        g = np.random.default_rng(seed)
        m = int(round(10 ** g.uniform(lo_exp, hi_exp)))
        fam = int(g.integers(0, 6))
        if fam == 0:       # uniform, mean degree 1..64 (selectivity varies widely)
            n = max(16, int(m / (2 ** g.uniform(0, 6))))
            out.append(dict(kind="linear", F=G.uniform_pairs(m, n, seed, dtype=np.int32), a=n))
        elif fam == 1:     # uniform over a large domain: tiny intermediate
            n = int(m * 2 ** g.uniform(2, 8))
            out.append(dict(kind="linear", F=G.uniform_pairs(m, n, seed, dtype=np.int32), a=n))
        elif fam == 2:     # power-law friends graph, mean degree 16
            n = max(64, m // 16)
            out.append(dict(kind="linear", F=G.powerlaw_friends(n, m, seed, cap=min(4096, n - 1)), a=n))
        elif fam == 3:
            n = max(64, m // 16)
            out.append(dict(kind="triangle", F=G.gnm_symmetric(n, m, seed), a=0))
        elif fam == 4:
            n = max(64, m // 16)
            out.append(dict(kind="triangle", F=G.chung_lu_symmetric(n, m, seed, cap=min(4096, n - 1)), a=0))
        else:
            scale = max(6, int(round(math.log2(max(64, m // 16)))))
            out.append(dict(kind="triangle", F=G.rmat_symmetric(scale, min(m, (1 << scale) * 16), seed), a=0))
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
    """Features, exact cardinalities and measured times of the candidate
    plans of one instance."""
    kind = L.LINEAR if inst["kind"] == "linear" else L.TRIANGLE
    Fd = torch.from_numpy(np.ascontiguousarray(inst["F"]).view(np.int32)).to("cuda")
    a = inst["a"]
    feat = ctx.sketch(kind, Fd, Fd, Fd)
    t0 = time.perf_counter()
    plan = ctx.plan(kind, Fd, Fd, Fd, a)
    plan_ms = (time.perf_counter() - t0) * 1e3
    ws = ctx.workspace(plan.workspace_bytes, Fd.device)
    n_out = max(a, 1) if kind == L.LINEAR else 1
    out = torch.empty(n_out, dtype=torch.int64, device="cuda")
    times = {}
    if kind == L.LINEAR:
        p3 = plan.copy(); p3.algo = L.ALGO_3WAY
        times["3way"] = _time(lambda: ctx.linear3_count(Fd, Fd, Fd, a, plan=p3, out=out, workspace=ws))
        res = int(L.as_u64(out[:a]).sum(dtype=np.uint64))
        pc = plan.copy(); pc.algo = L.ALGO_CASCADE
        times["cascade"] = _time(lambda: ctx.cascade2_count(L.LINEAR, Fd, Fd, Fd, a, plan=pc, out=out, workspace=ws))
        exact = int(L.as_u64(out[:a]).sum(dtype=np.uint64)) == res
        # the star plans specialise the two when R is small (planner rule)
        if plan.est_ms_star > 0.0:
            pst = plan.copy(); pst.algo = L.ALGO_STAR
            times["star"] = _time(lambda: ctx.linear3_count(Fd, Fd, Fd, a, plan=pst, out=out, workspace=ws))
            exact = exact and int(L.as_u64(out[:a]).sum(dtype=np.uint64)) == res
        if plan.est_ms_star_cascade > 0.0:
            psc = plan.copy(); psc.algo = L.ALGO_STAR_CASCADE
            times["star_cascade"] = _time(lambda: ctx.cascade2_count(L.LINEAR, Fd, Fd, Fd, a, plan=psc, out=out,
                                                                     workspace=ws))
            exact = exact and int(L.as_u64(out[:a]).sum(dtype=np.uint64)) == res
    else:
        for k in SHARES:
            ps = plan.copy(); ps.algo = L.ALGO_3WAY; ps.log2_share = k
            times[f"share{k}"] = _time(lambda: ctx.triangle3_count(Fd, Fd, Fd, plan=ps, out=out, workspace=ws), 1)
        res = int(L.as_u64(out)[0])
        if plan.join2_size <= CASCADE_CAP:
            pc = plan.copy(); pc.algo = L.ALGO_CASCADE
            times["cascade"] = _time(lambda: ctx.cascade2_count(L.TRIANGLE, Fd, Fd, Fd, plan=pc, out=out, workspace=ws), 1)
            exact = int(L.as_u64(out)[0]) == res
        else:
            times["cascade"] = float("inf")      # never chosen: the planner caps the intermediate
            exact = True
        # one symmetric simple relation: the degree-oriented join (planner rule)
        if plan.flags & L.PLAN_SYMMETRIC_SIMPLE:
            po = plan.copy(); po.algo = L.ALGO_ORIENTED
            times["oriented"] = _time(lambda: ctx.triangle3_count(Fd, Fd, Fd, plan=po, out=out, workspace=ws), 1)
            exact = exact and int(L.as_u64(out)[0]) == res
    best3 = min(v for k, v in times.items() if k in ("3way", "star") or k.startswith("share"))
    bestc = min(v for k, v in times.items() if k in ("cascade", "star_cascade"))
    return dict(kind=kind, features=feat, join2=plan.join2_size, out=res, times=times,
                est=dict(star=plan.est_ms_star, star_cascade=plan.est_ms_star_cascade,
                         three=plan.est_ms_3way, cascade=plan.est_ms_cascade),
                plan_label=int(bestc < best3),
                share_label=(int(np.argmin([times[f"share{k}"] for k in SHARES])) if kind == L.TRIANGLE else -1),
                analytic=dict(algo=plan.algo, share=plan.log2_share), plan_ms=plan_ms,
                oriented_ok=bool(plan.flags & L.PLAN_SYMMETRIC_SIMPLE),
                cascade_equals_3way=exact, n=int(Fd.shape[0]))


def stack(rows):
    X = torch.stack([r["features"] for r in rows]).contiguous()
    targets = torch.tensor([[math.log2(1 + r["join2"]), math.log2(1 + r["out"])] for r in rows],
                           dtype=torch.float32, device=X.device)
    pl = torch.tensor([r["plan_label"] for r in rows], dtype=torch.int32, device=X.device)
    sl = torch.tensor([r["share_label"] for r in rows], dtype=torch.int32, device=X.device)
    return X, targets, pl, sl


def nearest_share(k):
    """The timed share class closest to log2 share k."""
    return min(SHARES, key=lambda c: (abs(c - k), c))


def plan_time(r, algo, share):
    t = r["times"]
    if algo == L.ALGO_ORIENTED:
        return t["oriented"]
    if algo == L.ALGO_STAR_CASCADE:
        return t["star_cascade"]
    if algo == L.ALGO_STAR:
        return t["star"]
    if algo == L.ALGO_CASCADE:
        return t["cascade"]
    return t["3way"] if r["kind"] == L.LINEAR else t[f"share{share}"]


# mj_plan's rule for the degree-oriented cyclic join (mj_plan_model.h)
ORIENT_MIN_N, ORIENT_MIN_WEDGES = 32768, 64


def specialise(r, algo):
    """mj_plan's rules: a cyclic join of one large, skewed, symmetric simple
    relation becomes the degree-oriented join; a three-way (cascade) choice becomes
    the star three-way join (star cascade) when that plan is eligible and
    rated faster by the analytic model."""
    if (r["kind"] == L.TRIANGLE and r.get("oriented_ok") and r["n"] >= ORIENT_MIN_N
            and r["join2"] >= ORIENT_MIN_WEDGES * r["n"]):
        return L.ALGO_ORIENTED
    e = r.get("est")
    if r["kind"] != L.LINEAR or not e:
        return algo
    if algo == L.ALGO_3WAY and 0.0 < e["star"] < e["three"]:
        return L.ALGO_STAR
    if algo == L.ALGO_CASCADE and 0.0 < e["star_cascade"] < e["cascade"]:
        return L.ALGO_STAR_CASCADE
    return algo


def evaluate(planner, rows):
    """Held-out comparison of the learned plan with the analytic plan, the
    fixed plans and the best measured plan (regret), plus cardinality
    q-errors."""
    X, targets, _, _ = stack(rows)
    Y = planner.predict(X).cpu().numpy()
    tot = {"learned": 0.0, "analytic": 0.0, "always_3way": 0.0, "always_cascade": 0.0, "best": 0.0}
    qI, qO = [], []
    for r, y in zip(rows, Y):
        algo = specialise(r, L.ALGO_CASCADE if (y[3] > y[2] and r["join2"] <= CASCADE_CAP) else L.ALGO_3WAY)
        share = SHARES[int(np.argmax(y[4:7]))]
        tot["learned"] += plan_time(r, algo, share)
        tot["analytic"] += plan_time(r, r["analytic"]["algo"], nearest_share(r["analytic"]["share"]))
        tot["always_3way"] += plan_time(r, L.ALGO_3WAY, SHARES[0])
        tot["always_cascade"] += r["times"]["cascade"]
        tot["best"] += min(r["times"].values())
        qI.append(2 ** abs(float(y[0]) - math.log2(1 + r["join2"])))
        qO.append(2 ** abs(float(y[1]) - math.log2(1 + r["out"])))
    res = {k: round(v, 3) for k, v in tot.items()}
    res["regret_learned"] = round(tot["learned"] / tot["best"], 4)
    res["regret_analytic"] = round(tot["analytic"] / tot["best"], 4)
    res["qerror_join2_median"] = round(float(np.median(qI)), 3)
    res["qerror_join2_p95"] = round(float(np.percentile(qI, 95)), 3)
    res["qerror_out_median"] = round(float(np.median(qO)), 3)
    res["qerror_out_p95"] = round(float(np.percentile(qO, 95)), 3)
    res["instances"] = len(rows)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=12000)
    ap.add_argument("--n-test", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()

    def log(m):
        print(f"[learned] {m}", file=sys.stderr, flush=True)
    ctx = L.Context()
    rows = {}
    for part, n, seed in (("train", args.n_train, 5_000_000), ("test", args.n_test, 6_000_000)):
        rows[part] = []
        t0 = time.time()
        inst = planner_instances(n, seed)
        for i, x in enumerate(inst):
            rows[part].append(label_instance(ctx, x))
            if (i + 1) % 1000 == 0:
                log(f"{part}: {i + 1}/{n} instances labelled ({time.time() - t0:.0f} s)")
    X, targets, pl, sl = stack(rows["train"])
    planner = LearnedPlanner(ctx)
    planner.init_weights(seed=0)
    hist = planner.train(X, targets, pl, sl, epochs=args.epochs, log=log)
    planner.save(args.out)
    rep = evaluate(planner, rows["test"])
    rep["train_loss_first_last"] = [round(hist[0], 4), round(hist[-1], 4)]
    rep["train_instances"] = len(rows["train"])
    rep["cascade_equals_3way_all"] = all(r["cascade_equals_3way"] for part in rows.values() for r in part)
    rep["train_plan_label_cascade_fraction"] = round(float(pl.float().mean().item()), 4)
    log(json.dumps(rep))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
