"""The benchmark's contract, on the CPU: one GPU only (a multi-GPU request
exits with a message before anything touches a device), the default
steps, and the traffic record's hash inputs (a source file renamed away
would make the hash skip it silently)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location(
        "bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_defaults(monkeypatch):
    b = _bench()
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = b.parse()
    assert (a.gpus, a.steps, a.warmup) == (1, 20, 5)
    assert a.only is None and not a.no_extras


def test_traffic_hash_covers_existing_sources():
    b = _bench()
    for f in b.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_2604_22228_amd", f)), f
    h = b.kernel_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    with open(b.PROFILE_TRAFFIC) as f:
        rec = json.load(f)
    # the record states what it was measured on and how it was scaled
    assert rec["algorithmic_bytes_per_launch"] == 36 * (1 << 26)
    assert 0.99 < rec["traffic_over_algorithmic"] < 1.1
    assert abs(rec["copy_probe"]["fetch_scale"] - 2.0) < 0.01
    assert abs(rec["copy_probe"]["write_scale"] - 1.0) < 0.01
