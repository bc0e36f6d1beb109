"""The benchmark script on the host: it imports with every module-level name
defined, its defaults are the documented ones, and asking for more than one
GPU exits with a message (no GPU is touched on that path)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_module_constants_and_defaults(monkeypatch):
    b = _load()
    assert b.METRIC.startswith("MVF subdomain bounds/sec")
    assert abs(b.FP64_ISSUE_PEAK - 39.3216e12) < 1e6
    assert isinstance(b.TRAFFIC, dict)
    for key, val in b.TRAFFIC.items():
        # (engine, grad, tape hash, code-object bytes): a rebuilt kernel finds no stale entry
        assert len(key) == 4 and key[0] in ("spec", "interp") and key[1] in ("fwd", "rev") and val > 0
        assert isinstance(key[3], int) and key in b.TRAFFIC_SOURCE
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = b.parse()
    assert (a.gpus, a.steps, a.warmup, a.engine, a.grad) == (1, 200, 200, "spec", "fwd")


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
