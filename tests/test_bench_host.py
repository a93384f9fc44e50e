"""Host logic of bench.py (CPU): the one-GPU contract, and the counter-based
traffic lookup, which applies only to the workload, solve mode, kernel class
and source digest it was measured on."""
import hashlib
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2, (r.returncode, r.stderr)
    assert "one GPU" in r.stderr


def test_traffic_lookup_applies_only_where_measured(monkeypatch):
    b = _bench()
    t = b.MEASURED_TRAFFIC
    k = "block_inner_kernel<float>"
    assert k in t["bytes_per_launch"]
    assert b.measured_traffic(k, "graded4096_k1e6_p0.5", t["mode"]) is None
    assert b.measured_traffic(k, t["workload"], "fp64") is None
    assert b.measured_traffic("pair_step_kernel", t["workload"], t["mode"]) is None
    # the stored figure, when the sources still hash to the stored digest
    h = hashlib.sha256()
    for src in t["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    monkeypatch.setitem(t, "sha256", h.hexdigest())
    assert b.measured_traffic(k, t["workload"], t["mode"]) == t["bytes_per_launch"][k]
    # any other digest (a changed source) voids it
    monkeypatch.setitem(t, "sha256", "0" * 64)
    assert b.measured_traffic(k, t["workload"], t["mode"]) is None
