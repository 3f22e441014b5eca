"""The library's host build under AddressSanitizer and UndefinedBehaviorSanitizer
(tests/hostsim): every kernel and the host code run on the CPU, every caller
buffer is an exact-size allocation pre-filled with a non-zero byte.

- abi_check: argument checks that need a context (a planning workspace one
  byte short, a plan given other relations of the same sizes, a count
  workspace too small);
- multi_check: merged launches (one grid for launches of one kernel from
  several joins): every workgroup finds its own launch, block index and
  grid size, for 1..6000 launches;
- replay: the benchmark's sequence of calls on one context (the three-way
  join with per-kernel events, the cascade on the same plan, the small
  workload, the distinct count, windows of the materialised result, the
  star schema under its four plans, a batch of eighty small joins of both
  kinds under every plan form) on scaled-down inputs, each result checked
  against a closed form, the oracle or another algorithm, under two fill
  bytes.
Any access outside a buffer, undefined behaviour, a deadlock at a barrier
or a differing result fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOSTSIM = os.path.join(ROOT, "tests", "hostsim")


@pytest.fixture(scope="module")
def built():
    sys.path.insert(0, HOSTSIM)
    import build as hostsim_build
    return hostsim_build.build(sanitize=True, jobs=8)


def _run(cmd, env_extra=None, timeout=600):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.update(env_extra or {})
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    return r.returncode, r.stdout + r.stderr


def test_abi_checks_under_sanitizers(built):
    rc, out = _run([os.path.join(built, "abi_check")])
    assert rc == 0 and "all checks passed" in out, out[-3000:]


def test_merged_launch_block_search(built):
    rc, out = _run([os.path.join(built, "multi_check")])
    assert rc == 0 and "all checks passed" in out, out[-3000:]


def test_batch_on_a_small_device(built, tmp_path_factory):
    """The batch leg with a one-CU device: persistent grids of a few waves,
    each taking its work items in runs of several."""
    data = tmp_path_factory.getbasetemp() / "hostsim_tiny"
    if not (data / "meta.txt").exists():
        subprocess.run([sys.executable, os.path.join(HOSTSIM, "make_inputs.py"), str(data), "--tiny"],
                       check=True, capture_output=True)
    rc, out = _run([os.path.join(built, "replay"), str(data), "batch"], {"HIPSIM_CUS": "1"})
    assert rc == 0 and "all checks passed" in out, out[-3000:]


@pytest.mark.parametrize("fill", ["0xA5", "0x00"])
def test_replay_of_the_benchmark_sequence(built, tmp_path_factory, fill):
    data = tmp_path_factory.getbasetemp() / "hostsim_tiny"
    if not (data / "meta.txt").exists():
        subprocess.run([sys.executable, os.path.join(HOSTSIM, "make_inputs.py"), str(data), "--tiny"],
                       check=True, capture_output=True)
    rc, out = _run([os.path.join(built, "replay"), str(data)], {"HIPSIM_FILL": fill, "HIPSIM_STEPS": "1"})
    assert rc == 0 and "all checks passed" in out, out[-3000:]
    assert "inactive lane" not in out, out[-3000:]
