"""bench.py's command line on the host: more than one GPU is refused before
anything touches a device, and the traffic figure is withheld once the
simulate kernel's sources no longer match the counters it came from."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_traffic_figure_follows_the_kernel_sources(tmp_path, monkeypatch):
    import bench

    rec = {"source_hash": bench.sim_source_hash(), "bytes_per_launch": 123.0}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.traffic_per_launch() == 123.0
    f.write_text(json.dumps(dict(rec, source_hash="0" * 16)))
    assert bench.traffic_per_launch() is None
    f.write_text("{damaged")
    assert bench.traffic_per_launch() is None
