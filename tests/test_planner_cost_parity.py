"""The planner's cost formulas (C++, inside libmj) against the oracle's
restatement of the paper's formulas, and the worked examples -- no GPU."""
import math

import numpy as np
import pytest

from oracle import cost_model as cm


@pytest.fixture(scope="module")
def mj():
    import paper_1905_13376_amd as mj
    return mj


CASES = [
    ("linear_tuples", cm.linear_tuples_read, 4),
    ("cascade_tuples", cm.cascade_tuples_moved, 1),
    ("linear_break_even_M", cm.linear_threshold, 4),
    ("cyclic_tuples", cm.cyclic_tuples_read, 5),
    ("cyclic_optimal_H", cm.cyclic_optimal_H, 4),
    ("cyclic_min", cm.cyclic_min_tuples_read, 4),
    ("join2_uniform", cm.join2_size_uniform, 3),
    ("branch_hit", cm.branch_hit_probability, 2),
]


@pytest.mark.parametrize("name,ref,k", CASES)
def test_formula_parity(mj, name, ref, k):
    rng = np.random.default_rng(abs(hash(name)) % 2**32)
    for _ in range(200):
        args = list(10 ** rng.uniform(0, 12, size=k))
        want = ref(*args)
        got = mj.cost_model(name, *args)
        if math.isinf(want):
            assert math.isinf(got)
        else:
            assert got == pytest.approx(want, rel=1e-12)


def test_worked_examples_through_the_planner(mj):
    F = 6e11
    assert mj.cost_model("linear_break_even_M", F, F, F, 1.8e14) == pytest.approx(1.00334e9, rel=1e-4)
    # Sec. 5.2 derived form of Example 4
    M = 2.6845e7
    assert mj.cost_model("cyclic_min", F, F, F, M * 1.001) < 1.8e14 < \
        mj.cost_model("cyclic_min", F, F, F, M * 0.999)


def test_bad_formula_id_rejected(mj):
    import ctypes
    import paper_1905_13376_amd._lib as L
    arr = (ctypes.c_double * 1)(1.0)
    out = ctypes.c_double()
    assert L._lib.mj_cost_model(99, arr, 1, ctypes.byref(out)) == -1
    assert L._lib.mj_cost_model(0, arr, 1, ctypes.byref(out)) == -1   # too few arguments


def test_slarge_buckets(mj):
    """The S-largest plan's bucket counts (host only): parts of R of about
    1024 tuples, at most 2^12 cells, larger T split further; R beyond 2^12
    parts of 1024 is refused."""
    lr, lt, ms = mj.slarge_buckets(1 << 16, 1 << 26, 1 << 16)
    assert lr == 6 and lr + lt <= 12 and ms > 0
    lr2, lt2, _ = mj.slarge_buckets(1 << 12, 1 << 26, 1 << 22)
    assert lr2 == 2 and lt2 > lt and lr2 + lt2 <= 12
    assert mj.slarge_buckets(1025, 1 << 20, 10)[0] == 1
    assert mj.slarge_buckets(1, 1 << 20, 1)[:2] == (0, 0)
    with pytest.raises(mj.MJError):
        mj.slarge_buckets((1 << 22) + 1, 1 << 26, 1 << 10)
    # the modelled time grows with S
    assert mj.slarge_buckets(1 << 16, 1 << 27, 1 << 16)[2] > ms
