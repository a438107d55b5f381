"""CPU checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message, and the module-level names the JSON line uses exist."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_module_constants():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    assert m.METRIC.startswith("element-steps/s")
    assert m.HBM_PEAK_GBS == 8000.0
    assert callable(m.measured_traffic) and callable(m.run_ensemble) and callable(m.run_serving)
