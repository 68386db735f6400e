"""Host logic of bench.py (CPU): the one-GPU refusal, the workload-name suffixes, the PMC
summary's per-dispatch means and copy scaling, and the gate on the traffic figure (a
changed kernel source, another precision or another launch shape reports no traffic)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workload_suffixes():
    assert bench.base_workload("two_stream") == "two_stream"
    assert bench.base_workload("two_stream_monopole") == "two_stream"
    assert bench.base_workload("two_stream_p2") == "two_stream"
    assert bench.base_workload("two_stream_monopole_p2") == "two_stream"


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for disp, name, value in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


def test_pmc_summary_scales_by_the_copy(tmp_path, monkeypatch):
    """Per-dispatch means of the fused kernel only (other kernels and per-channel rows of one
    dispatch summed first), each scaled by known bytes over the copy's reading."""
    src = tmp_path / "paper_2605_21794_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "vp_kernels.hip").write_text("// kernel source stand-in\nint k = 1;\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    k = "void vpk::k_fused<1, 512, true, false, false>(...)"
    _write_counters(tmp_path / "f", "FETCH_SIZE", [(1, k, 100.0), (1, k, 50.0), (2, k, 250.0),
                                                   (3, "k_ring", 1e9)])
    _write_counters(tmp_path / "w", "WRITE_SIZE", [(1, k, 400.0), (2, k, 600.0)])
    gib_kib = (1 << 30) / 1024.0
    _write_counters(tmp_path / "cf", "FETCH_SIZE", [(1, "copy", gib_kib / 2), (2, "fill", 3.0)])
    _write_counters(tmp_path / "cw", "WRITE_SIZE", [(1, "copy", gib_kib)])
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                      str(tmp_path / "cw"), "two_stream", "fp32c", [512, 4, 8])
    rec = json.load(open(tmp_path / "profiles" / "pmc_k_fused_two_stream_512x4x8.json"))
    assert rec["dispatches"] == [2, 2]
    assert rec["fetch_kib_per_dispatch"] == pytest.approx(200.0)
    assert rec["write_kib_per_dispatch"] == pytest.approx(500.0)
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["traffic_bytes_per_launch"] == pytest.approx((2 * 200.0 + 500.0) * 1024.0)
    n = rec["n"]
    assert rec["traffic_bytes_per_particle"] == pytest.approx(rec["traffic_bytes_per_launch"] / n)
    assert rec["precision"] == "fp32c" and rec["launch"] == [512, 4, 8]
    # the traffic figure is served only while the kernel source, the particle count, the
    # precision and the launch shape are those of the counter runs
    shape = [512, 4, 8]
    assert bench.load_traffic("two_stream", n, "fp32c", shape) == pytest.approx(
        rec["traffic_bytes_per_launch"])
    assert bench.load_traffic("two_stream", n + 1, "fp32c", shape) is None
    assert bench.load_traffic("two_stream", n, "fp64", shape) is None
    assert bench.load_traffic("two_stream", n, "fp32c", [1024, 4, 8]) is None
    assert bench.load_traffic("two_stream", n, "fp32c", [512, 4, 4]) is None
    (src / "vp_kernels.hip").write_text("// a comment edited\nint k = 1;  /* and one added */\n")
    assert bench.load_traffic("two_stream", n, "fp32c", shape) == pytest.approx(
        rec["traffic_bytes_per_launch"])
    (src / "vp_kernels.hip").write_text("// kernel source stand-in\nint k = 2;\n")
    assert bench.load_traffic("two_stream", n, "fp32c", shape) is None


def test_launch_key():
    assert bench.launch_key({"threads": 512, "ppt": 4, "acc_copies": 8, "use_graph": 1,
                             "graph_steps": 99, "persistent": 0}) == [512, 4, 8]


def test_committed_counters_name_their_settings():
    """Every committed counter summary records the precision and launch shape it was taken
    at, so that no other run reports its bytes."""
    import glob
    files = glob.glob(os.path.join(ROOT, "profiles", "pmc_k_*.json"))
    assert files
    for f in files:
        rec = json.load(open(f))
        assert rec["kernel"] in ("k_fused", "k_persist"), f
        assert rec["precision"] in ("fp64", "fp32c", "fp32ts", "fp32"), f
        assert len(rec["launch"]) == 3 and all(isinstance(v, int) for v in rec["launch"]), f
        assert os.path.basename(f) == os.path.basename(
            bench.pmc_path(rec["workload"], rec["launch"], rec["kernel"])), f
        if rec["kernel"] == "k_persist":
            assert rec["steps_per_launch"] >= 1, f


def test_pmc_summary_of_the_persistent_kernel(tmp_path, monkeypatch):
    """A persistent launch runs many steps: its summary names the kernel and its steps per
    launch, and a run with another step count reports none of its bytes."""
    src = tmp_path / "paper_2605_21794_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "vp_kernels.hip").write_text("// kernel source stand-in\nint k = 1;\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    k = "void vpk::k_persist<1, 1024, 4, false>(...)"
    _write_counters(tmp_path / "f", "FETCH_SIZE", [(1, k, 300.0), (2, "k_fused<1>", 9e9)])
    _write_counters(tmp_path / "w", "WRITE_SIZE", [(1, k, 700.0)])
    gib_kib = (1 << 30) / 1024.0
    _write_counters(tmp_path / "cf", "FETCH_SIZE", [(1, "copy", gib_kib / 2)])
    _write_counters(tmp_path / "cw", "WRITE_SIZE", [(1, "copy", gib_kib)])
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                      str(tmp_path / "cw"), "two_stream", "fp32c", [1024, 4, 4],
                      "k_persist", 1000)
    rec = json.load(open(tmp_path / "profiles" / "pmc_k_persist_two_stream_1024x4x4.json"))
    assert rec["kernel"] == "k_persist" and rec["steps_per_launch"] == 1000
    assert rec["dispatches"] == [1, 1]
    tb = (2 * 300.0 + 700.0) * 1024.0
    assert rec["traffic_bytes_per_launch"] == pytest.approx(tb)
    assert rec["traffic_bytes_per_update"] == pytest.approx(tb / (rec["n"] * 1000))
    n, shape = rec["n"], [1024, 4, 4]
    assert bench.load_traffic("two_stream", n, "fp32c", shape, "k_persist", 1000) == \
        pytest.approx(tb)
    assert bench.load_traffic("two_stream", n, "fp32c", shape, "k_persist", 20) is None
    assert bench.load_traffic("two_stream", n, "fp32c", shape, "k_fused", 1) is None
    assert bench.kernel_of({"persistent": 1}) == "k_persist"
    assert bench.kernel_of({"persistent": 0}) == "k_fused"


def test_source_hash_ignores_comments_and_layout():
    """The counters' source hash follows the code only: comments and whitespace may change,
    string literals and code may not."""
    base = 'int a = 1; /* x */ const char* s = "a // b";\nint f() { return a; } // tail\n'
    same = ('int a = 1;\n// one more comment\nconst char* s = "a // b";  int f() {\n'
            '    return a;  /* inside */\n}\n')
    assert bench.code_tokens(base) == bench.code_tokens(same)
    assert bench.code_tokens(base) != bench.code_tokens(base.replace('"a // b"', '"a  b"'))
    assert bench.code_tokens(base) != bench.code_tokens(base.replace("return a", "return -a"))
    assert bench.code_tokens("char c = '/'; int x; // y") == "char c = '/'; int x;"
