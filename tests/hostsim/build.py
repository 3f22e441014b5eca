"""Host build of libmj under AddressSanitizer and UndefinedBehaviorSanitizer
(test infrastructure only; the product library is built by hipcc for gfx950).

    python tests/hostsim/build.py [--no-sanitize] [-j N]

The library's sources are copied to _build/hostsim/src with one mechanical
change -- a dynamic LDS declaration `extern __shared__ T name[];` becomes a
pointer to the workgroup's dynamic LDS buffer -- and compiled as C++ for the
CPU against the stand-in runtime of tests/hostsim (hip/hip_runtime.h,
sim.cpp).  Output: _build/hostsim/replay (the benchmark's call sequence,
replay.cpp), _build/hostsim/abi_check (argument checks that need a
context, abi_check.cpp) and _build/hostsim/multi_check (merged launches'
block search, multi_check.cpp).
"""
from __future__ import annotations

import argparse
import glob
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1905_13376_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(ROOT, "_build", "hostsim")
CXX = "/opt/rocm/llvm/bin/clang++"

DYN = re.compile(r"extern\s+__shared__\s+([A-Za-z_][\w\s]*?)\s+(\w+)\s*\[\s*\]\s*;")


def transform(text: str) -> str:
    return DYN.sub(lambda m: f"{m.group(1)}* {m.group(2)} = "
                             f"reinterpret_cast<{m.group(1)}*>(::hipsim::dyn_smem());", text)


def build(sanitize: bool = True, jobs: int = 8, verbose: bool = False) -> str:
    src_dir = os.path.join(OUT, "src")
    obj_dir = os.path.join(OUT, "obj" if sanitize else "obj_plain")
    os.makedirs(src_dir, exist_ok=True)
    os.makedirs(obj_dir, exist_ok=True)
    units = []
    for path in sorted(glob.glob(os.path.join(CSRC, "*"))):
        name = os.path.basename(path)
        if not name.endswith((".hip", ".cpp", ".h")):
            continue
        text = transform(open(path).read())
        dst = os.path.join(src_dir, name)
        if not os.path.exists(dst) or open(dst).read() != text:
            with open(dst, "w") as f:
                f.write(text)
        if name.endswith((".hip", ".cpp")):
            units.append(dst)
    units += [os.path.join(HERE, "sim.cpp")]
    mains = [os.path.join(HERE, "replay.cpp"), os.path.join(HERE, "abi_check.cpp"),
             os.path.join(HERE, "multi_check.cpp")]
    # uninitialised locals (kernel argument structs among them) hold a
    # non-zero pattern, so a field left unset reads as a wild value, not 0
    flags = ["-x", "c++", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-pthread",
             "-ftrivial-auto-var-init=pattern",
             "-I" + HERE, "-I" + src_dir, "-I" + INCLUDE, "-Wno-unused-command-line-argument",
             "-Wno-ignored-attributes", "-Wno-unknown-pragmas", "-Wno-pass-failed"]
    if sanitize:
        flags += ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

    def cc(u):
        o = os.path.join(obj_dir, os.path.basename(u) + ".o")
        deps = [u] + glob.glob(os.path.join(src_dir, "*.h")) + [os.path.join(HERE, "hip", "hip_runtime.h")]
        if os.path.exists(o) and all(os.path.getmtime(d) <= os.path.getmtime(o) for d in deps):
            return o
        cmd = [CXX] + flags + ["-c", u, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {u}\n{r.stderr[-6000:]}")
        return o

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(cc, units + mains))
    lib_objs, main_objs = objs[:len(units)], objs[len(units):]
    suffix = "" if sanitize else "_plain"
    for m, mo in zip(mains, main_objs):
        exe = os.path.join(OUT, os.path.splitext(os.path.basename(m))[0] + suffix)
        link = [CXX, "-pthread", "-g"] + (["-fsanitize=address,undefined"] if sanitize else []) + lib_objs + \
               [mo, "-o", exe]
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed\n{r.stderr[-6000:]}")
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--no-sanitize", action="store_true")
    ap.add_argument("-j", type=int, default=8)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(not a.no_sanitize, a.j, a.v))
    sys.exit(0)
