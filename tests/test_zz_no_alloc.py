"""The allocation-free linear join (mj_linear3_count_static): the library's
per-device scratch array as the workspace.  Two calls in a row, the second on
a smaller input, each equal element by element to mj_linear3_count with a
workspace of the caller's; a plan whose path needs more than the array is
refused before any launch."""
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


def test_static_scratch_equals_workspace_call_twice(mj, ctx):
    import torch
    banner("allocation-free linear join: two calls, the second smaller")
    F = G.linear_powerlaw(seed=2001, n_vertices=1 << 16, m=1 << 20).view(np.uint32)
    for m, a_dom in ((1 << 20, 1 << 16), (50_000, 1 << 16)):
        Fm = np.ascontiguousarray(F[:m])
        Fd = dev(Fm)
        p = ctx.plan(mj.LINEAR, Fd, Fd, Fd, a_dom)
        assert p.flags & mj.PLAN_DENSE_KEYS
        want = mj.as_u64(ctx.linear3_count(Fd, Fd, Fd, a_dom, plan=p)).copy()
        out = torch.full((a_dom,), 7, dtype=torch.int64, device="cuda")
        got = mj.as_u64(ctx.linear3_count_static(Fd, Fd, Fd, a_dom, plan=p, out=out))
        np.testing.assert_array_equal(got, want)
        np.testing.assert_array_equal(got, oracle.linear3_count(Fm, Fm, Fm, a_dom))


def test_static_scratch_hashed_tables(mj, ctx):
    banner("allocation-free linear join, hashed tables")
    rng = np.random.default_rng(3)
    R = rng.integers(0, 3000, size=(30000, 2)).astype(np.uint32)
    R[:, 1] = rng.integers(0, 2 ** 31, size=30000)               # sparse B
    S = np.stack([R[rng.integers(0, 30000, 40000), 1], rng.integers(0, 2 ** 31, 40000)], 1).astype(np.uint32)
    T = np.stack([S[rng.integers(0, 40000, 20000), 1], rng.integers(0, 9, 20000)], 1).astype(np.uint32)
    Rd, Sd, Td = dev(R), dev(S), dev(T)
    p = fixed_plan(mj, ctx, mj.LINEAR, Rd, Sd, Td, 3000, log2_nb=6, log2_nc=6, seed=11, flags=mj.PLAN_NO_DENSE)
    got = mj.as_u64(ctx.linear3_count_static(Rd, Sd, Td, 3000, plan=p))
    np.testing.assert_array_equal(got, oracle.linear3_count(R, S, T, 3000))


def test_static_scratch_refuses_a_larger_plan(mj, ctx):
    import torch
    banner("allocation-free linear join: a plan beyond the scratch array")
    n = 1 << 23
    Fd = torch.randint(0, 1 << 24, (n, 2), dtype=torch.int32, device="cuda")
    p = fixed_plan(mj, ctx, mj.LINEAR, Fd, Fd, Fd, 1 << 24, log2_nb=10, log2_nc=10, seed=1,
                   flags=mj.PLAN_NO_DENSE)
    out = torch.full((1 << 24,), 5, dtype=torch.int64, device="cuda")
    with pytest.raises(mj.MJError) as e:
        ctx.linear3_count_static(Fd, Fd, Fd, 1 << 24, plan=p, out=out)
    assert "WORKSPACE" in str(e.value)
    assert int((out != 5).sum()) == 0                              # untouched
