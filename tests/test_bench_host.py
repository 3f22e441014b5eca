"""Host logic of bench.py (no GPU): the algorithmic byte counts behind the
roofline entry, and the --paths mode that runs every other path as a child
process of its own and gathers their JSON lines."""
import json
import subprocess
import sys

import pytest

import bench


def test_range_kernel_bytes():
    """Per launch: the pairs read once, one 2-byte table read per tuple, the
    outputs (and their 2-byte copies) written once."""
    n, a, b, c = 1 << 24, 1 << 20, 1 << 20, 1 << 20
    assert bench.kernel_bytes("k_range_count", n, n, n, 0, 0, a, b, c) == 10 * n + 8 * a
    assert bench.kernel_bytes("k_range_w", n, n, n, 0, 0, a, b, c) == 10 * n + 10 * b
    assert bench.kernel_bytes("k_range_deg", n, n, n, 0, 0, a, b, c) == 8 * n + 6 * c


def test_child_paths_runs_every_leg_alone(monkeypatch):
    calls = []

    def fake_run(cmd, capture_output, text, timeout):
        calls.append(cmd)
        leg = cmd[cmd.index("--only") + 1]
        if leg == "emit":                      # a leg that fails is reported, not fatal
            return subprocess.CompletedProcess(cmd, 1, stdout="", stderr="boom")
        body = {leg: {f"{leg}_result": {"ms": 1.0}}}
        return subprocess.CompletedProcess(cmd, 0, stdout="noise\n" + json.dumps(body) + "\n", stderr="")

    monkeypatch.setattr(subprocess, "run", fake_run)
    out = bench.child_paths(bench.LEGS)
    assert [c[c.index("--only") + 1] for c in calls] == list(bench.LEGS)
    for c in calls:
        assert c[0] == sys.executable and c[1].endswith("bench.py") and "--no-cpu" in c
    assert out["emit"]["error"] == "exit status 1" and "boom" in out["emit"]["stderr_tail"]
    for leg in bench.LEGS:
        if leg != "emit":
            assert out[f"{leg}_result"] == {"ms": 1.0}


def test_default_legs_are_configurations_other_than_the_main_one():
    assert set(bench.DEFAULT_LEGS) <= set(bench.LEGS)
    assert {"small", "triangle", "batch", "planner"} <= set(bench.DEFAULT_LEGS)


def test_shared_partition_bytes():
    """R = S = T one relation: its partition by range of its first column is
    made once, so the partition launches move one relation."""
    n = 1 << 24
    assert bench.kernel_bytes("dense:k_part_scatter", n, n, n, 0, 0, 0, shared_partition=True) == 16 * n
    assert bench.kernel_bytes("dense:k_part_scatter", n, n, n, 0, 0, 0) == 40 * n
    assert bench.kernel_bytes("dense:k_part_hist", n, n, n, 0, 0, 0, shared_partition=True) == 4 * n


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU only" in capsys.readouterr().err
