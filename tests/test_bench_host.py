"""Host-side checks of bench.py: the one-GPU contract and the rule that
stored HBM counters are reported only for the kernel source they were
taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_stored_traffic_follows_the_kernel_source_hash(tmp_path, monkeypatch):
    good = {"kernel": "k_step", "source_sha256": bench.kernel_source_hash(), "read_bytes": 300, "write_bytes": 100,
            "per": "launch"}
    p = tmp_path / "profile.md"
    p.write_text("# summary\n\ntraffic_json: " + json.dumps(good) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", "profile.md")
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: good["source_sha256"])
    t = bench.measured_traffic(200)
    assert t["total_bytes"] == 400 and t["vs_algorithmic"] == 2.0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.measured_traffic(200) is None



def test_every_workload_traffic_profile_holds_counters_of_the_current_source():
    """each committed per-workload counter profile exists and carries one
    traffic_json record; when it was taken on the step source in the tree the
    bench reports it (a profile older than the source is reported as null by
    the bench, and skipped here with that reason)"""
    import pytest
    stale = []
    for workload, rel in bench.TRAFFIC_PROFILES.items():
        path = os.path.join(ROOT, rel)
        assert os.path.exists(path), rel
        recs = [json.loads(l.split(":", 1)[1]) for l in open(path) if l.startswith("traffic_json:")]
        assert len(recs) == 1, rel
        assert recs[0]["read_bytes"] > 0 and recs[0]["write_bytes"] > 0
        if recs[0]["source_sha256"] != bench.kernel_source_hash():
            stale.append(rel)
            assert bench.measured_traffic(1, rel) is None
        else:
            assert bench.measured_traffic(1, rel) is not None
    if stale:
        pytest.skip(f"counters predate the current step source (traffic reported as null): {stale}")
