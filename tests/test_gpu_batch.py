"""Batched execution of many uneven joins (linear and cyclic, one batch):
every per-join result bit-exact against the oracle, and a HIP-graph
capture of the whole batch replayed several times with eager work in
between, each replay checked."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, dev, fixed_plan
from workloads import generators as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mj():
    import paper_1905_13376_amd as mj
    return mj


@pytest.fixture(scope="module")
def ctx(mj):
    c = mj.Context()
    yield c
    c.close()


def make_joins(mj, count, lo, hi, seed):
    inst = G.batch_instances(count=count, base_seed=seed, lo_exp=lo, hi_exp=hi)
    joins, want, keep = [], [], []
    for x in inst:
        F = x["F"]
        Fd = dev(F)
        keep.append(Fd)
        if x["kind"] == "linear":
            joins.append((mj.LINEAR, Fd, Fd, Fd, x["n"]))
            want.append(oracle.linear3_count(F, F, F, x["n"]))
        else:
            joins.append((mj.TRIANGLE, Fd, Fd, Fd, 0))
            want.append(oracle.triangle3_count(F, F, F))
    return joins, want, keep


def check(mj, outs, want):
    for o, w in zip(outs, want):
        got = mj.as_u64(o)
        if isinstance(w, int):
            assert int(got[0]) == w
        else:
            np.testing.assert_array_equal(got, w)


def test_batch_mixed(mj, ctx):
    banner("batch of 48 mixed joins, 10^3..10^4.5 edges")
    joins, want, keep = make_joins(mj, 48, 3.0, 4.5, 4000)
    b = ctx.batch(joins)
    check(mj, b.run(), want)
    check(mj, b.run(), want)            # a second run on the same buffers


def test_batch_with_cascade_items_and_empty(mj, ctx):
    banner("batch with cascade-planned and empty joins")
    joins, want, keep = make_joins(mj, 8, 3.0, 3.5, 4100)
    plans = [ctx.plan(k, R, S, T, a) for (k, R, S, T, a) in joins]
    plans[0].algo = mj.ALGO_CASCADE
    plans[5].algo = mj.ALGO_CASCADE
    e = dev(np.zeros((0, 2), dtype=np.uint32))
    joins.append((mj.LINEAR, e, e, e, 7))
    plans.append(ctx.plan(mj.LINEAR, e, e, e, 7))
    want.append(np.zeros(7, dtype=np.uint64))
    b = ctx.batch(joins, plans=plans)
    check(mj, b.run(), want)


def test_batch_graph_replay(mj, ctx):
    import torch
    banner("batch under HIP graph capture, replayed")
    joins, want, keep = make_joins(mj, 24, 3.0, 4.2, 4200)
    b = ctx.batch(joins)
    b.run()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        b.run(stream=s)
    for r in range(3):
        for o in b.outs:                 # scribble, so a replay must rewrite them
            o.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        check(mj, b.outs, want)
        # eager work between replays on the default stream
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()


def test_batch_ordered_on_callers_stream(mj, ctx):
    """The joins are prepared on the context's own streams, side by side.
    They must start after the work queued on the caller's stream before the
    call (here the copy that writes their inputs, queued behind a long
    product) and end before the work queued after it (the copy of their
    outputs).  Cascade and oriented items run on those streams too."""
    import torch
    banner("batch ordered on the caller's stream")
    joins, want, keep = make_joins(mj, 40, 3.0, 4.5, 4300)
    plans = [ctx.plan(k, R, S, T, a) for (k, R, S, T, a) in joins]
    plans[3].algo = mj.ALGO_CASCADE
    E = G.gnm_symmetric(3000, 30000, seed=14)
    Ed = dev(E)
    joins.append((mj.TRIANGLE, Ed, Ed, Ed, 0))
    plans.append(fixed_plan(mj, ctx, mj.TRIANGLE, Ed, Ed, Ed, seed=0x1B873593, algo=mj.ALGO_ORIENTED))
    assert plans[-1].algo == mj.ALGO_ORIENTED
    want.append(oracle.triangle3_count(E, E, E))
    keep.append(Ed)
    b = ctx.batch(joins, plans=plans)
    staged = [x.clone() for x in keep]
    res = [torch.full_like(o, -1) for o in b.outs]
    for x in keep:
        x.zero_()                        # wrong inputs until the caller's copy lands
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = torch.randn(4096, 4096, device="cuda")
        for _ in range(6):
            a = (a @ a) * 1e-3
        for x, y in zip(keep, staged):
            x.copy_(y)
        b.run(stream=s)
        for r, o in zip(res, b.outs):
            r.copy_(o)
    torch.cuda.synchronize()
    check(mj, res, want)


def test_batch_staging_reused(mj, ctx):
    """Eager calls share one staging buffer for their argument tables: two
    batches of different sizes run back to back without a synchronisation
    between them (the second call must not overwrite tables the first
    one's copy has not read), alternately, each result checked."""
    banner("batch staging buffer reused across calls")
    j1, w1, k1 = make_joins(mj, 6, 3.0, 3.5, 4400)
    j2, w2, k2 = make_joins(mj, 30, 3.0, 4.0, 4500)
    b1, b2 = ctx.batch(j1), ctx.batch(j2)
    for _ in range(2):
        o1 = [o.clone() for o in b1.run()]
        o2 = [o.clone() for o in b2.run()]
        check(mj, o1, w1)
        check(mj, o2, w2)


def _check_golden(mj, outs, gold):
    import hashlib
    for o, g in zip(outs, gold):
        got = mj.as_u64(o)
        if g["kind"] == "linear":
            got = got[:g["a_domain"]].astype("<u8")
            assert int(got.sum(dtype=np.uint64)) == g["sum"], g["k"]
            assert hashlib.sha256(got.tobytes()).hexdigest() == g["sha256_u64_le"], g["k"]
        else:
            assert int(got[0]) == g["total"], g["k"]


def test_batch_512_full_golden(mj, ctx):
    """The full 512-join batch (seeds 4000 + k, 10^3..10^6 edges, half linear
    and half cyclic) under the planner's plans: every join's result equals
    the oracle's, stored by tests/golden/make_batch_golden.py, for the eager
    call (which launches at most 512 kernels: one per merged step) and for
    three replays of its HIP-graph capture."""
    import json
    import os
    import torch
    banner("batch of 512 joins, full size, against the oracle's results")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch512.json")))["joins"]
    joins, keep = [], []
    for k in range(512):
        x = G.batch_instance(k)
        Fd = dev(x["F"])
        keep.append(Fd)
        joins.append((mj.LINEAR, Fd, Fd, Fd, x["n"]) if x["kind"] == "linear" else (mj.TRIANGLE, Fd, Fd, Fd, 0))
    b = ctx.batch(joins)
    _check_golden(mj, b.run(), gold)
    torch.cuda.synchronize()
    # one call issues merged steps: a few hundred launches, not each join's own
    ctx.profile(True)
    ctx.profile_read()
    _check_golden(mj, b.run(), gold)
    torch.cuda.synchronize()
    launches = sum(v[1] for v in ctx.profile_read().values())
    ctx.profile(False)
    assert 0 < launches <= 512, launches
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        b.run(stream=s)
    for _ in range(3):
        for o in b.outs:
            o.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        _check_golden(mj, b.outs, gold)
