"""The learned planner's kernels against the float64 reference (same BF16
weights), its training, the degree sketch against numpy degree
histograms, and plans chosen by the network giving exact counts."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp_ref as M
from tests.gpu_util import banner, dev
from workloads import generators as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import paper_1905_13376_amd as mj
    from paper_1905_13376_amd import learned
    import paper_1905_13376_amd._lib as L
    return mj, learned, L


@pytest.fixture(scope="module")
def ctx(mods):
    mj = mods[0]
    c = mj.Context()
    yield c
    c.close()


def bf16_params(masters):
    return {k: (M.bf16_round(v) if k.startswith("W") else v).astype(np.float64)
            for k, v in masters.items()}


def test_forward_parity(mods, ctx):
    import torch
    mj, learned, L = mods
    banner("mlp forward vs float64 reference")
    pl = learned.LearnedPlanner(ctx)
    pl.init_weights(seed=3)
    rng = np.random.default_rng(0)
    X = rng.normal(0, 1, (37, M.IN)).astype(np.float32)
    Y = pl.predict(torch.from_numpy(X).cuda()).cpu().numpy()
    ref, _ = M.forward(bf16_params(pl.masters()), X)
    np.testing.assert_allclose(Y, ref, rtol=2e-4, atol=2e-5)


def test_gradient_and_adamw_parity(mods, ctx):
    import torch
    mj, learned, L = mods
    banner("mlp gradients and AdamW vs float64 reference")
    pl = learned.LearnedPlanner(ctx)
    pl.init_weights(seed=5)
    rng = np.random.default_rng(1)
    B = 70
    X = rng.normal(0, 1, (B, M.IN)).astype(np.float32)
    t = rng.normal(8, 3, (B, 2)).astype(np.float32)
    plab = rng.integers(0, M.NPLAN, B).astype(np.int32)
    slab = rng.integers(-1, 3, B).astype(np.int32)
    dX, dt = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    dp, ds = torch.from_numpy(plab).cuda(), torch.from_numpy(slab).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = torch.empty(L.mlp_workspace_bytes(B), dtype=torch.uint8, device="cuda")
    masters = pl.masters()
    L.mlp_grads(ctx, pl.buf, dX, dt, dp, ds, loss, ws)
    grad = pl.buf[: 4 * learned.P * 4].view(torch.float32)[learned.P:2 * learned.P].cpu().numpy()
    p64 = bf16_params(masters)
    y, cache = M.forward(p64, X)
    assert float(loss.item()) == pytest.approx(M.loss(y, t, plab, slab), rel=1e-4)
    g = M.backward(p64, cache, M.loss_grad_y(y, t, plab, slab))
    ref = np.concatenate([g[k].ravel() for k, _ in learned.SHAPES])
    np.testing.assert_allclose(grad, ref, rtol=2e-3, atol=2e-5)
    # one AdamW step from these gradients
    L.mlp_adamw(ctx, pl.buf, 1e-3, 1e-2, 1)
    w0 = np.concatenate([masters[k].ravel() for k, _ in learned.SHAPES]).astype(np.float64)
    w1, _, _ = M.adamw(w0, grad.astype(np.float64), np.zeros_like(w0), np.zeros_like(w0), 1, 1e-3, 1e-2)
    got = np.concatenate([v.ravel() for v in pl.masters().values()])
    np.testing.assert_allclose(got, w1, rtol=1e-5, atol=1e-7)


def test_training_reduces_loss(mods, ctx):
    import torch
    mj, learned, L = mods
    banner("mlp training on a synthetic task")
    rng = np.random.default_rng(2)
    N = 4096
    X = rng.normal(0, 1, (N, M.IN)).astype(np.float32)
    t = np.stack([X[:, :10].sum(1) * 2 + 10, X[:, 10:20].sum(1) + 5], 1).astype(np.float32)
    plab = (X[:, 0] > 0).astype(np.int32)
    slab = np.where(X[:, 1] > 0.5, 2, np.where(X[:, 1] < -0.5, 0, 1)).astype(np.int32)
    d = [torch.from_numpy(a).cuda() for a in (X, t, plab, slab)]
    pl = learned.LearnedPlanner(ctx)
    pl.init_weights(seed=0)
    hist = pl.train(*d, epochs=40, batch=256, lr=3e-3)
    assert hist[-1] < 0.25 * hist[0]
    Y = pl.predict(d[0]).cpu().numpy()
    assert ((Y[:, M.PLAN0 + 1] > Y[:, M.PLAN0]) == (plab == 1)).mean() > 0.85


def numpy_sketch(R, S, T, kind):
    f = np.zeros(100)
    for h, col in enumerate((np.asarray(R)[:, 1], np.asarray(S)[:, 0], np.asarray(T)[:, 0])):
        _, cnt = np.unique(np.asarray(col).view(np.uint32), return_counts=True)
        bins = np.bincount(np.floor(np.log2(cnt)).astype(int), minlength=32)
        f[32 * h:32 * h + 32] = np.log2(1 + bins) / 32
    f[96:99] = [math.log2(1 + len(R)) / 32, math.log2(1 + len(S)) / 32, math.log2(1 + len(T)) / 32]
    f[99] = kind
    return f


def test_sketch_matches_numpy(mods, ctx):
    mj, learned, L = mods
    banner("degree sketch vs numpy")
    F = G.linear_powerlaw(seed=7, n_vertices=1 << 13, m=1 << 17)
    rng = np.random.default_rng(3)
    T = rng.integers(0, 500, size=(3000, 2)).astype(np.uint32)
    T[:5, 0] = 0xFFFFFFFF
    got = ctx.sketch(mj.TRIANGLE, dev(F), dev(F), dev(T)).cpu().numpy()
    np.testing.assert_allclose(got, numpy_sketch(F, F, T, 1), rtol=1e-6, atol=1e-7)


def test_learned_plans_give_exact_counts(mods, ctx):
    mj, learned, L = mods
    banner("plans chosen by the network: exact counts")
    pl = learned.LearnedPlanner(ctx)
    pl.init_weights(seed=11)
    ctx.set_planner(pl.buf)
    F = G.linear_powerlaw(seed=12, n_vertices=1 << 12, m=1 << 16)
    Fd = dev(F)
    p = ctx.plan(mj.LINEAR, Fd, Fd, Fd, 1 << 12, planner="learned")
    assert p.pred_log2_out != 0.0 or p.pred_log2_join2 != 0.0
    want = oracle.linear3_count(F, F, F, 1 << 12)
    run = p.algo in (mj.ALGO_CASCADE, mj.ALGO_STAR_CASCADE)
    got = (mj.as_u64(ctx.cascade2_count(mj.LINEAR, Fd, Fd, Fd, 1 << 12, plan=p)) if run
           else mj.as_u64(ctx.linear3_count(Fd, Fd, Fd, 1 << 12, plan=p)))
    np.testing.assert_array_equal(got, want)
    E = G.gnm_symmetric(2000, 30000, seed=2)
    Ed = dev(E)
    q = ctx.plan(mj.TRIANGLE, Ed, Ed, Ed, planner="learned")
    assert q.log2_share in (0, 2, 4)
    tot = (ctx.cascade2_count(mj.TRIANGLE, Ed, Ed, Ed, plan=q) if q.algo == mj.ALGO_CASCADE
           else ctx.triangle3_count(Ed, Ed, Ed, plan=q))
    assert int(mj.as_u64(tot)[0]) == oracle.triangle3_count(E, E, E)
    ctx.set_planner(None)


def test_shipped_planner_beats_analytic_on_held_out(mods, ctx):
    """The shipped network on join instances it was not trained on (other
    seeds, 10^3..10^6 edges, every family): every plan of every instance
    is timed on the device and its count checked against the three-way
    join's; the network's plans take less summed time than the analytic
    planner's, on the same measured times."""
    mj, learned, L = mods
    banner("shipped learned planner vs analytic planner, held-out instances")
    pl = learned.use_shipped(ctx)
    rows = [learned.label_instance(ctx, x) for x in learned.planner_instances(400, 7_500_000, 3.0, 6.0)]
    D = learned.rows_to_arrays(rows)
    assert D["counts_exact"].all()
    res = learned.evaluate(pl, D)
    print(res)
    assert res["learned"] < res["analytic"]
    ctx.set_planner(None)
