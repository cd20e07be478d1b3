"""Host-side checks of the benchmark script: argument contract and the HBM traffic figure it
reports next to the roofline (no GPU needed)."""
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


def test_code_digest_ignores_comments_and_whitespace_only():
    src = "int f(int a) {\n  return a + 1;  // add one\n}\n"
    same = "// header\nint f(int a)\n{\n\treturn a + 1;\n}\n"
    other = "int f(int a) {\n  return a + 2;\n}\n"
    assert bench.near_code_digest(src) == bench.near_code_digest(same)
    assert bench.near_code_digest(src) != bench.near_code_digest(other)


def _counter_total(path):
    """Near-phase bytes recomputed from the per-kernel averages and the copy calibration."""
    text = open(path).read()
    fetch_factor = float(re.search(r"FETCH_SIZE is scaled by ([0-9.]+)", text).group(1))
    write_factor = float(re.search(r"WRITE_SIZE by ([0-9.]+)", text).group(1))
    total = 0.0
    for counter, kib in re.findall(r"^\S.*? (FETCH_SIZE|WRITE_SIZE) KiB: .*\(avg ([0-9.]+)\)$", text, re.M):
        total += float(kib) * 1024 * (fetch_factor if counter == "FETCH_SIZE" else write_factor)
    return total


def test_traffic_is_the_calibrated_counter_sum_while_the_kernel_is_unchanged():
    val, src = bench.near_traffic()
    recorded = re.search(r"code sha1: ([0-9a-f]+)", open(bench.NEAR_COUNTERS).read()).group(1)
    current = bench.near_code_digest(open(bench.NEAR_SOURCE).read())
    if recorded != current:
        assert val is None
        return
    assert src.startswith("rocprofv3")
    assert abs(val - _counter_total(bench.NEAR_COUNTERS)) < 1e-3 * val
    # the near kernel writes one float64 reverse partial sum per slot and component: at least
    # the 1.23 GB the counters attribute to it
    assert val > 1.2e9


def test_traffic_is_dropped_once_the_kernel_changes(tmp_path, monkeypatch):
    changed = tmp_path / "kernels_p2p.hip"
    changed.write_text(open(bench.NEAR_SOURCE).read() + "\nstatic int one_more_line;\n")
    monkeypatch.setattr(bench, "NEAR_SOURCE", str(changed))
    val, why = bench.near_traffic()
    assert val is None and "changed" in why
