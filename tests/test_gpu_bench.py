"""The bench line's contract on the GPU: one JSON line with the metric, throughput, timing,
roofline (achieved over peak, with the committed PMC traffic while the kernel source is
unchanged) and configuration, from a short fixed-shape run of the default workload."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--no-tune", "--launch",
                        "512,4,8", "--steps", "20", "--warmup", "9", "--no-cpu", *args],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    return json.loads(lines[0])


def test_default_bench_line():
    d = run_bench()
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 9
    assert d["value"] > 0 and d["higher_is_better"] is True and d["dtype"] == "f64"
    assert d["config"]["workload"] == "two_stream" and d["config"]["n"] == 1 << 20
    assert d["config"]["state_finite_after_run"] is True
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["achieved"] == pytest.approx(36 * (1 << 20) / (rf["kernel_us"] * 1e-6) / 1e9)
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"])
    # the counters stand for the kernel only while its source is the one they were taken on
    if committed_counters_current("two_stream"):
        assert rf["traffic"] is not None and rf["traffic"] > 36 * (1 << 20)
    else:
        assert rf["traffic"] is None


def committed_counters_current(workload):
    """True when the committed counters stand for this test's runs: the same kernel source,
    fp32c, and the launch shape the runs fix (512, 4, 8)."""
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(bench.pmc_path(workload, [512, 4, 8])))
    return (rec["kernel_src_sha"] == bench.kernel_src_sha() and rec["precision"] == "fp32c"
            and rec["launch"] == [512, 4, 8])


def test_fp64_line_reports_no_fp32_counters():
    """The counters were taken on float32 storage: a float64 run moves other bytes and must
    not report them."""
    d = run_bench("--precision", "fp64")
    assert d["config"]["precision"] == "fp64" and d["dtype"] == "f64"
    rf = d["roofline"]
    assert rf["traffic"] is None
    assert rf["achieved"] == pytest.approx(72 * (1 << 20) / (rf["kernel_us"] * 1e-6) / 1e9)


def test_p2_bench_line():
    d = run_bench("--element-order", "2")
    assert d["config"]["workload"] == "two_stream_p2" and d["config"]["element_order"] == 2
    assert d["value"] > 0
    assert (d["roofline"]["traffic"] is not None) == committed_counters_current("two_stream_p2")


def test_persistent_bench_line():
    """The persistent kernel's line: one launch of the timed steps, the algorithmic bytes of
    all of them over that launch's duration, the note on what they count, and no counter
    traffic for a step count the counters were not taken at."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--no-tune", "--launch",
                        "1024,4,4,1", "--steps", "100", "--warmup", "9", "--no-cpu",
                        "--no-served"], capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    d = json.loads([ln for ln in r.stdout.splitlines() if ln.strip()][-1])
    assert d["config"]["timed_launches"] == "persistent launches"
    rf = d["roofline"]
    assert rf["kernel"] == "k_persist" and rf["steps_per_launch"] == 100
    assert rf["bytes_per_launch"] == 36 * (1 << 20) * 100
    assert rf["achieved"] == pytest.approx(rf["bytes_per_launch"] / (rf["kernel_us"] * 1e-6) / 1e9)
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"])
    assert "registers" in rf["note"]
    assert rf["traffic"] is None
