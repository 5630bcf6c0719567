"""Host-side logic of bench.py (no GPU): the one-GPU guard, the roofline
pricing, and the rule that a stored HBM traffic figure is reported only for
the kernel source and list parameters it was measured on."""
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


def test_roofline_prices_useful_pair_flops_against_the_fp32_peak():
    """achieved = ordered in-cutoff pairs x 19 FLOP / mean launch time, over
    157.3 TFLOP/s; issued work counts the entries the kernel walks (padding
    included); the HBM view
    counts 150 bytes per atom-step."""
    prof = {"force_ms": 0.25, "pairs": 67216584.0}
    stats = {"mean_list_len": 104.0, "skin": 0.4, "cell_div": 1.0, "windows": 1.0, "wg_size": 128.0,
             "mean_walked": 126.0}
    n = 1 << 20
    r = bench.roofline(prof, stats, n, "mixed_fixed")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(67216584.0 * 19 / 0.25e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["issued_tflops"] == pytest.approx(126.0 * n * 19 / 0.25e-3 / 1e12)
    assert r["list_candidates_per_launch"] == 104.0 * n
    assert r["hbm_view"]["achieved_gbs"] == pytest.approx(n * 150 / 0.25e-3 / 1e9)
    assert r["kernel"] == "k_force_mixed<true,false,true,true,2>"
    assert bench.kernel_name("fp64") == "k_force_fp64<false,true,4>"
    assert bench.kernel_name("mixed", 0, 64) == "k_force_mixed<false,false,true,false,1>"


def test_stored_traffic_only_for_the_measured_configuration():
    recs = bench.traffic_records()
    assert recs, "no record in the committed counter summary"
    kv = recs[0]
    skin, div, prec, n = float(kv["skin"]), int(kv["cell_div"]), kv["precision"], int(kv["n_atoms"])
    if kv["source_digest"] != bench.source_digest():
        pytest.skip("the force-kernel sources changed since the counters were taken")
    k = kv.get("kernel")
    assert bench.stored_traffic(skin, div, prec, n, k) == float(kv["hbm_bytes_per_launch"])
    assert bench.stored_traffic(skin + 0.01, div, prec, n, k) is None
    assert bench.stored_traffic(skin, div + 1, prec, n, k) is None
    assert bench.stored_traffic(skin, div, "fp64", n, k) is None
    assert bench.stored_traffic(skin, div, prec, n + 64, k) is None
    assert bench.stored_traffic(skin, div, prec, n, "another kernel") is None


def test_traffic_records_parse_sections(tmp_path):
    p = tmp_path / "t.md"
    p.write_text("text\n- ignored: 1\n### Record A\n- skin: 0.3\n- kernel: `k<a>`\n"
                 "### Record B\n- skin: 0.4\nprose\n- hbm_bytes_per_launch: 5\n")
    recs = bench.traffic_records(str(p))
    assert recs == [{"skin": "0.3", "kernel": "k<a>"}, {"skin": "0.4", "hbm_bytes_per_launch": "5"}]
