"""GPU parity of the materialised linear join (the join of Sec. 4 with its
result written out) against the oracle: the tuples (a, b, c, d) in
nested-loop order, element by element, order included."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, dev
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


def emit(ctx, R, S, T, first=0, cap=None):
    import torch
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    if cap is None:
        out, total = ctx.linear3_materialize(Rd, Sd, Td, first=first)
        return out.cpu().numpy().view(np.uint32), int(total.item())
    out = torch.full((max(cap, 1), 4), -7, dtype=torch.int32, device="cuda")
    _, total = ctx.linear3_materialize(Rd, Sd, Td, first=first, out=out[:cap] if cap else out[:0])
    return out.cpu().numpy().view(np.uint32)[:cap], int(total.item())


def rel(rng, n, dom):
    return rng.integers(0, dom, size=(n, 2)).astype(np.uint32)


def test_emit_uniform(mj, ctx):
    banner("emit uniform 3000 tuples over [0, 100)")
    rng = np.random.default_rng(1)
    R, S, T = rel(rng, 3000, 100), rel(rng, 3000, 100), rel(rng, 3000, 100)
    got, total = emit(ctx, R, S, T)
    want, wtotal = oracle.linear3_materialize(R, S, T)
    assert total == wtotal and total > 20 * 16384        # many tiles and a ragged last one
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("seed", range(5))
def test_emit_random_bags_special_keys(mj, ctx, seed):
    banner(f"emit random bags seed={seed}")
    rng = np.random.default_rng(100 + seed)
    dom = [60, 40, 700, 90, 25000][seed]
    nr, ns, nt = (int(x) for x in rng.integers(1, 6000, size=3))
    R, S, T = rel(rng, nr, dom), rel(rng, ns, dom), rel(rng, nt, dom)
    special = np.array([0xFFFFFFFF, 0x80000000, 0xFFFFFFFE], dtype=np.uint32)
    for X, col in ((R, 0), (R, 1), (S, 0), (S, 1), (T, 0), (T, 1)):
        m = rng.random(X.shape[0]) < 0.05
        X[m, col] = special[rng.integers(0, 3, size=m.sum())]
    want, wtotal = oracle.linear3_materialize(R, S, T)
    got, total = emit(ctx, R, S, T)
    assert total == wtotal
    np.testing.assert_array_equal(got, want)


def test_emit_windows(mj, ctx):
    banner("emit windows")
    rng = np.random.default_rng(7)
    R, S, T = rel(rng, 1500, 60), rel(rng, 1500, 60), rel(rng, 1500, 60)
    want, total = oracle.linear3_materialize(R, S, T)
    for first, cap in ((0, 1), (5, 16384), (16383, 2), (16380, 40000), (total - 3, 10), (total, 5),
                       (total + 100, 3), (12345, 0)):
        got, t = emit(ctx, R, S, T, first, cap)
        assert t == total
        n = max(0, min(cap, total - first))
        np.testing.assert_array_equal(got[:n], want[first:first + n])
        assert (got[n:] == np.uint32(0xFFFFFFF9)).all()        # rows past the end untouched


def test_emit_hubs_sparse_r_and_empty_pairs(mj, ctx):
    """One R tuple whose results span many tiles; long stretches of R tuples
    without results and of R tuples with one result each (a tile then covers
    more R tuples than its LDS window holds); S tuples whose C is not in T."""
    banner("emit hubs / sparse R / empty pairs")
    rng = np.random.default_rng(3)
    hub_s = np.stack([np.full(400, 5), rng.integers(0, 50, 400)], 1)      # b = 5: 400 S tuples
    hub_t = np.stack([rng.integers(0, 50, 3000), rng.integers(0, 1 << 30, 3000)], 1)
    one_s = np.stack([np.arange(1000, 1200), np.full(200, 77)], 1)         # b in [1000, 1200): c = 77
    one_t = np.array([[77, 4242]])                                        # one t for c = 77
    dead_s = np.stack([np.full(50, 9), np.full(50, 999999)], 1)          # c = 999999: no t
    S = np.concatenate([hub_s, one_s, dead_s]).astype(np.uint32)
    T = np.concatenate([hub_t, one_t]).astype(np.uint32)
    R = np.concatenate([
        np.stack([rng.integers(0, 1 << 31, 30000), np.full(30000, 31337)], 1),   # no s
        np.stack([rng.integers(0, 1 << 31, 20000), rng.integers(1000, 1200, 20000)], 1),  # one result
        np.stack([np.arange(3), np.full(3, 5)], 1),                              # hubs
        np.stack([rng.integers(0, 1 << 31, 5000), np.full(5000, 9)], 1),         # empty pairs only
        np.stack([rng.integers(0, 1 << 31, 20000), rng.integers(1000, 1200, 20000)], 1),
    ]).astype(np.uint32)
    R = R[rng.permutation(R.shape[0])]
    want, wtotal = oracle.linear3_materialize(R, S, T)
    got, total = emit(ctx, R, S, T)
    assert total == wtotal
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n", [2, 8191, 8192, 8193, 16383, 16384, 16385, 131072, 131073])
def test_emit_sort_sizes(mj, ctx, n):
    """S and T of n tuples with long runs of equal B and of equal C, whose
    order in the output is the relations' own order; n at the edges of the
    one-workgroup sort (8192 keys) and of the one-launch scan (32 tiles)."""
    banner(f"emit, S and T of {n} tuples")
    rng = np.random.default_rng(n)
    S = np.stack([rng.integers(0, 1000, n), rng.integers(0, 50000, n)], 1).astype(np.uint32)
    T = np.stack([rng.integers(0, 50000, n), rng.integers(0, 1 << 32, n)], 1).astype(np.uint32)
    R = np.stack([rng.integers(0, 1 << 32, 50), rng.integers(0, 1000, 50)], 1).astype(np.uint32)
    want, wtotal = oracle.linear3_materialize(R, S, T)
    got, total = emit(ctx, R, S, T)
    assert total == wtotal
    np.testing.assert_array_equal(got, want)


def test_emit_empty_and_sizing(mj, ctx):
    banner("emit empty inputs and sizing")
    e = np.zeros((0, 2), dtype=np.uint32)
    F = np.array([[0, 1], [1, 2], [2, 3]], dtype=np.uint32)
    for R, S, T in ((e, F, F), (F, e, F), (F, F, e), (F, F + 10, F)):
        got, total = emit(ctx, R, S, T, 0, 4)
        assert total == 0 and (got == np.uint32(0xFFFFFFF9)).all()
    got, total = emit(ctx, F, F, F, 0, 0)
    assert total == oracle.linear3_materialize(F, F, F)[1] == 1


def test_emit_column_layouts(mj, ctx):
    import torch
    banner("emit column layouts")
    rng = np.random.default_rng(9)
    F = rel(rng, 4000, 300)
    want, total = oracle.linear3_materialize(F, F, F)
    Fd = dev(F)
    soa = torch.stack([Fd[:, 0].contiguous(), Fd[:, 1].contiguous()], 0).t()   # strides (1, n)
    out, t = ctx.linear3_materialize(soa, soa, soa)
    assert int(t.item()) == total
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), want)


def test_emit_errors(mj, ctx):
    import torch
    banner("emit argument errors")
    Fd = dev(np.array([[1, 2]], dtype=np.uint32))
    with pytest.raises(ValueError):
        ctx.linear3_materialize(Fd, Fd, Fd, out=torch.empty((4, 3), dtype=torch.int32, device="cuda"))
    with pytest.raises(mj.MJError) as e:
        ctx.linear3_materialize(Fd, Fd, Fd, workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert "WORKSPACE" in str(e.value)


def test_emit_powerlaw_full_sampled(mj, ctx):
    """The benchmarked friends graph (2^24 edges): all 4.36e9 result tuples
    written in one call (several launch chunks of 2^30 positions); sampled
    positions, the chunk and tile boundaries among them, against the
    oracle."""
    import torch
    banner("emit power-law full size (4.36e9 tuples, 70 GB)")
    F = G.linear_powerlaw()
    Fd = dev(F)
    out, total = ctx.linear3_materialize(Fd, Fd, Fd)
    n = int(total.item())
    rng = np.random.default_rng(5)
    pos = np.concatenate([rng.integers(0, n, 400), [0, n - 1],
                          [k * (1 << 30) + d for k in range(1, n >> 30) for d in (-1, 0)],
                          [k * 16384 + d for k in (1, 7, 100003) for d in (-1, 0)]]).astype(np.int64)
    idx = torch.from_numpy(pos).to("cuda")
    got = out[idx].cpu().numpy().view(np.uint32)
    del out
    torch.cuda.empty_cache()
    want, wtotal = oracle.linear3_materialize_at(F, F, F, pos.astype(np.uint64))
    assert n == wtotal
    np.testing.assert_array_equal(got, want)
