"""Host logic of bench.py (no GPU): the traffic figure it reports comes from the committed
rocprofv3 summary only while the Vanka step's sources are the ones the counters were taken
from; more than one GPU is refused with a message before anything touches a device; the
Poisson ratio of a parameter set given by Lame parameters."""
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


def test_traffic_is_taken_only_for_the_profiled_sources(monkeypatch, tmp_path):
    b = _bench()
    prof = tmp_path / "summary.md"
    prof.write_text("kernel_source_sha256: %s\ntraffic_bytes_per_launch: 123456\n" % b.kernel_source_hash())
    assert b.measured_traffic(str(prof)) == 123456
    monkeypatch.setattr(b, "kernel_source_hash", lambda: "0" * 64)
    assert b.measured_traffic(str(prof)) is None
    assert b.measured_traffic(str(tmp_path / "missing.md")) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_poisson_ratio_from_lame():
    b = _bench()
    assert b.poisson({"lam": 1.0, "mu": 1.0}) == 0.25
    E, nu = 1.0, 0.49
    lam, mu = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
    assert abs(b.poisson({"lam": lam, "mu": mu}) - nu) < 1e-6
