"""Host logic of bench.py (no GPU): the committed HBM-traffic record is used
only for the timed window it was taken over and only while the fit kernel's
sources hash to the recorded digest; the CPU description of the baseline."""
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_record_is_keyed_by_window_and_sources():
    b = load_bench()
    with open(os.path.join(ROOT, "profiles", "k_fit_c4096_traffic.json")) as fh:
        rec = json.load(fh)
    wins = rec["windows"]
    assert wins, "the record holds at least one window"
    w = wins[0]
    got = b.fit_traffic("c4096", w["warmup"], w["steps"])
    if w["fit_sources_sha256"] == b.fit_source_digest():
        assert got == w["bytes_per_launch"]
    else:
        assert got is None
    # another window, another workload: no figure
    assert b.fit_traffic("c4096", w["warmup"] + 1, w["steps"]) is None
    assert b.fit_traffic("c4096", w["warmup"], w["steps"] + 7) is None
    assert b.fit_traffic("c1024", w["warmup"], w["steps"]) is None


def test_traffic_record_ignored_when_sources_change(monkeypatch):
    b = load_bench()
    monkeypatch.setattr(b, "fit_source_digest", lambda: "0" * 64)
    with open(os.path.join(ROOT, "profiles", "k_fit_c4096_traffic.json")) as fh:
        w = json.load(fh)["windows"][0]
    assert b.fit_traffic("c4096", w["warmup"], w["steps"]) is None


def test_cpu_info_fields():
    b = load_bench()
    info = b.cpu_info()
    assert set(info) == {"cpu_model", "nproc", "cpus_allowed"}
    assert info["nproc"] >= 1 and 1 <= info["cpus_allowed"] <= info["nproc"]


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
