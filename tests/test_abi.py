"""The C ABI without a GPU: the library loads, exports every function that
include/mj.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mj.h")
LIB = os.path.join(ROOT, "paper_1905_13376_amd", "libmj.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(mj_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmj.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("mj_plan", "mj_linear3_count", "mj_triangle3_count", "mj_cascade2_count",
                 "mj_ctx_create", "mj_ctx_destroy", "mj_status_str"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_1905_13376_amd._lib as L
    assert set(declared_functions()) <= set(L.exported_symbols())


def test_status_strings(lib):
    lib.mj_status_str.restype = ctypes.c_char_p
    assert lib.mj_status_str(0) == b"MJ_OK"
    assert lib.mj_status_str(-3) == b"MJ_ERR_WORKSPACE"
    assert lib.mj_status_str(-99) == b"MJ_ERR_UNKNOWN"


def test_null_arguments_rejected_without_device(lib):
    INVALID = -1
    vp = ctypes.c_void_p
    assert lib.mj_ctx_create(0, None) == INVALID
    assert lib.mj_ctx_destroy(None) == INVALID
    f = lib.mj_linear3_count
    f.argtypes = [vp] * 5 + [vp, vp, vp, ctypes.c_uint64, vp]
    f.argtypes = [vp, vp, vp, vp, ctypes.c_uint32, vp, vp, vp, ctypes.c_uint64, vp]
    assert f(None, None, None, None, 0, None, None, None, 0, None) == INVALID
    g = lib.mj_plan
    g.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_uint32, ctypes.c_int, vp, vp, ctypes.c_uint64, vp]
    assert g(None, 0, None, None, None, 0, 0, None, None, 0, None) == INVALID


def test_planning_workspace_size(lib):
    """mj_plan's workspace (the library allocates none): it grows with the
    relations and covers the cyclic kind's symmetry check."""
    f = lib.mj_plan_workspace
    f.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    f.restype = ctypes.c_uint64
    small, big = f(0, 1000, 1000, 1000), f(0, 1 << 24, 1 << 24, 1 << 24)
    assert 0 < small < big
    assert f(1, 1 << 20, 1 << 20, 1 << 20) >= f(0, 1 << 20, 1 << 20, 1 << 20)
    assert f(0, 0, 0, 0) > 0


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of mj_rel, mj_plan_t and mj_batch_item have the C
    layout: every field offset and the struct sizes, as a C compiler reads
    include/mj.h."""
    import subprocess
    import paper_1905_13376_amd._lib as L
    structs = {"mj_rel": L.Rel, "mj_plan_t": L.Plan, "mj_batch_item": L.BatchItem}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mj.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
