"""bench.py's command-line contract and its use of committed profiles (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def run_bench(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=e,
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_exits_with_a_message():
    r = run_bench(["--gpus", "2"])
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU" in r.stderr


def test_more_than_one_rank_exits_with_a_message():
    r = run_bench([], env={"WORLD_SIZE": "4"})
    assert r.returncode == 2 and r.stdout == "" and "one GPU" in r.stderr


def test_measured_traffic_is_used_only_for_the_profiled_kernel(monkeypatch):
    name = "rmat24skew-p0.25-q4-r4-L80"
    t = json.load(open(os.path.join(ROOT, "profiles", f"traffic_{name}.json")))
    assert t["bytes_per_launch"] == t["fetch_bytes"] + t["write_bytes"] > 0
    monkeypatch.setattr(bench, "kernel_sha", lambda: t["kernel_sha"])
    assert bench.load_traffic(name)["bytes_per_launch"] == t["bytes_per_launch"]
    for sha in t.get("same_code_shas", []):
        # sources whose persistent kernel compiles to the profiled instructions
        monkeypatch.setattr(bench, "kernel_sha", lambda: sha)
        assert bench.load_traffic(name)["bytes_per_launch"] == t["bytes_per_launch"]
        assert "k_persistent" in t["same_code_check"]
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 16)
    assert bench.load_traffic(name) is None
    assert bench.load_traffic("no-such-workload") is None


def test_profiles_name_their_commands_and_kernel():
    txt = open(os.path.join(ROOT, "profiles", "k_persistent_rmat24skew_hbm_counters.txt")).read()
    assert "rocprofv3 --pmc FETCH_SIZE" in txt and "rocprofv3 --pmc WRITE_SIZE" in txt
    trace = open(os.path.join(ROOT, "profiles", "k_persistent_rmat24skew_kernel_trace.txt")).read()
    assert "rocprofv3 --kernel-trace --stats" in trace and "k_persistent" in trace


def test_unknown_workload_name_exits_with_a_message():
    r = run_bench(["--workload", "skewy"])
    assert r.returncode == 2 and r.stdout == "" and "not a paper workload" in r.stderr
    r = run_bench(["--workload", "er20.5"])
    assert r.returncode == 2 and "integer scale" in r.stderr


def test_paper_context_names_the_papers_figures():
    from paper_1805_00280_amd import workloads as WL
    c = bench.paper_context(WL.skew(3.0))
    assert c["fn_base_seconds"] == 811.1 and c["table1_max_degree"] == 8420
    assert "fn_base_seconds" not in bench.paper_context(WL.skew(3.0, 2.0, 0.5))
    assert bench.paper_context(WL.C3) == {}


def test_skew_profile_names_its_commands():
    txt = open(os.path.join(ROOT, "profiles", "k_persistent_skew5_kernel_trace.txt")).read()
    assert txt.count("rocprofv3 --kernel-trace --stats") == 2 and "--workload skew5 --approx 1000" in txt


def test_output_line_is_strict_json():
    # non-finite values are reported as null, never as NaN or Infinity
    line = {"a": float("nan"), "b": [1.0, float("inf")], "c": {"d": -float("inf"), "e": 2}}
    assert bench.finite(line) == {"a": None, "b": [1.0, None], "c": {"d": None, "e": 2}}
