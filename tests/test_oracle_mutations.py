"""The pins are strong enough to catch plausible mistakes: each test plants
one mistake in a copy of the oracle's C source (on the CPU), builds it, and
checks that the pins reject the mutant."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import brute

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTATIONS = {
    "linear_uses_T_column_D": ("tc[i] = t0[i * tstride];", "tc[i] = t0[i * tstride + 1];"),
    "linear_transposed_S": ("pair_t* s = load_pairs(s0, s1, sstride, ns, 0);",
                            "pair_t* s = load_pairs(s0, s1, sstride, ns, 1);"),
    "linear_drops_first_match": ("for (uint64_t j = lo; j < hi; ++j) {            /* s with s.b = r.b */",
                                 "for (uint64_t j = lo + (hi > lo); j < hi; ++j) {"),
    "linear_ignores_T_multiplicity": ("acc[a] += nmatch;", "acc[a] += nmatch > 0;"),
    "triangle_R_keyed_by_A": ("pair_t* R = load_pairs(r0, r1, rstride, nr, 1);",
                              "pair_t* R = load_pairs(r0, r1, rstride, nr, 0);"),
    "triangle_set_semantics": ("total += hi - lo;", "total += hi > lo;"),
    "triangle_T_keyed_by_A": ("pair_t* T = load_pairs(t0, t1, tstride, nt, 0);",
                              "pair_t* T = load_pairs(t0, t1, tstride, nt, 1);"),
    "join2_uses_R_column_A": ("uint32_t b = r1[i * rstride];\n        total += upper_u32",
                              "uint32_t b = r0[i * rstride];\n        total += upper_u32"),
}


def _pins_pass():
    """A compact subset of the pins; True when all hold."""
    for seed in range(6):
        rng = np.random.default_rng(seed)
        dom = [2, 3, 5][seed % 3]
        R, S, T = (rng.integers(0, dom, size=(30, 2)).astype(np.uint32) for _ in range(3))
        if not np.array_equal(oracle.linear3_count(R, S, T, dom),
                              brute.linear_bruteforce(R, S, T, dom)):
            return False
        if oracle.triangle3_count(R, S, T) != brute.triangle_bruteforce(R, S, T):
            return False
        if oracle.join2_size(R, S) != brute.join2_bruteforce(R, S):
            return False
    return True


def test_unmutated_passes():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mutant = src.replace(old, new, 1)
    c = tmp_path / "mutant.c"
    so = tmp_path / "mutant.so"
    c.write_text(mutant)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(c)])
    lib = oracle.bind(ctypes.CDLL(str(so)))
    monkeypatch.setattr(oracle, "_lib", lib)
    assert not _pins_pass(), f"pins did not catch mutant {name}"
