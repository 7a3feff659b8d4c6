"""Host-side checks of bench.py: the one-GPU contract and the rule that a
stored HBM-traffic figure is only reported for the kernel source it was
measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_only_for_the_measured_source(tmp_path, monkeypatch):
    import bench
    digest = bench.kernel_source_digest()
    rec = {"k|w|m": {"source_digest": digest, "bytes_per_launch": 123}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: digest)
    assert bench.load_traffic("k", "w", "m") == 123
    assert bench.load_traffic("k", "w", "other") is None
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 16)
    assert bench.load_traffic("k", "w", "m") is None
