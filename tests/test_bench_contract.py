"""bench.py's command-line contract on the host: one GPU only, refused
before anything touches a device; the traffic summary is read only for the
sources it was taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "single" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_summary_matches_its_sources():
    sys.path.insert(0, ROOT)
    import bench
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    got = bench.measured_traffic("chimera::k_event_smooth32", "precision_300ev")
    # the committed summary is either current (then it is used) or stale (then ignored)
    assert got is None or got == t["kernels"]["chimera::k_event_smooth32"]["traffic_bytes"]
    assert bench.measured_traffic("chimera::k_event_smooth32", "another_workload") is None
    assert bench.measured_traffic("no_such_kernel", "precision_300ev") is None
