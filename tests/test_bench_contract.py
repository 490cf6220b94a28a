"""bench.py's contract without a GPU: one GPU only, and measured traffic taken
only from counter runs of the current kernel sources."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_from_the_current_kernel_sources(tmp_path, monkeypatch):
    bench = load_bench()
    from paper_1209_6007_amd import kernel_source_hash

    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"bytes_per_launch": 1.5e12, "kernel": "ms_team_kernel"}
    data = {"rmat17": {"team64": dict(entry, kernel_sha=kernel_source_hash()),
                       "far64": dict(entry, kernel_sha="0" * 16)}}
    (prof / "hbm_traffic.json").write_text(json.dumps(data))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("rmat17", 4) == 1.5e12          # team64, current sources
    assert bench.load_traffic("rmat17", "far64") is None      # taken on other sources
    assert bench.load_traffic("grid512", 3) is None           # never measured
    assert bench.CLASS_NAMES[4] == "team64" and set(bench.KERNEL_SYMBOLS) == set(range(len(bench.CLASS_NAMES)))


def test_committed_traffic_entries_name_their_kernel_and_sources():
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
        d = json.load(f)
    for workload, per in d.items():
        for cls, e in per.items():
            assert e["bytes_per_launch"] > 0 and len(e["kernel_sha"]) == 16 and e["kernel"], (workload, cls)
