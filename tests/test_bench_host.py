"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
byte count of the roofline, and the rule that a stored HBM traffic figure is
reported only for the kernel source and list parameters it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_are_list_plus_state_per_particle():
    assert bench.algorithmic_bytes(270.0, 4, "mixed_fixed") == 4 * (270.0 + 168)
    assert bench.algorithmic_bytes(270.0, 4, "fp64") == 4 * (270.0 + 48)


def _record():
    kv = {}
    with open(bench.TRAFFIC_FILE) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
    return kv


def test_stored_traffic_only_for_the_measured_configuration():
    kv = _record()
    skin, div, prec, n = float(kv["skin"]), int(kv["cell_div"]), kv["precision"], int(kv["n_atoms"])
    if kv["source_digest"] != bench.source_digest():
        pytest.skip("the force-kernel sources changed since the counters were taken")
    assert bench.stored_traffic(skin, div, prec, n) == float(kv["hbm_bytes_per_launch"])
    assert bench.stored_traffic(skin + 0.1, div, prec, n) is None
    assert bench.stored_traffic(skin, div + 1, prec, n) is None
    assert bench.stored_traffic(skin, div, "fp64", n) is None
    assert bench.stored_traffic(skin, div, prec, n + 64) is None
