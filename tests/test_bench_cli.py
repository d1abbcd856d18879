"""bench.py's command-line contract (no GPU): one GPU only, and the HBM
traffic figure is reported only for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_entry_follows_the_kernel_sources(tmp_path, monkeypatch):
    import bench
    rec = json.load(open(bench.TRAFFIC_FILE))
    entry = rec["helmholtz16_p4"]
    assert entry["bytes_per_launch"] > 0
    fresh = dict(rec)
    fresh["helmholtz16_p4"] = dict(entry, kernel_source_hash=bench.kernel_source_hash())
    f = tmp_path / "t.json"
    f.write_text(json.dumps(fresh))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.traffic_entry("helmholtz16_p4") == entry["bytes_per_launch"]
    stale = {k: dict(v, kernel_source_hash="0" * 16) for k, v in rec.items()}
    f.write_text(json.dumps(stale))
    assert bench.traffic_entry("helmholtz16_p4") is None
    assert bench.traffic_entry("helmholtz32_p4") is None
    f.write_text(json.dumps({}))
    assert bench.traffic_entry("helmholtz32_p4") is None
