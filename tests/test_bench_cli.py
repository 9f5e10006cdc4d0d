"""Host-side checks of bench.py that need no GPU: a multi-GPU request is
refused with a message (the path runs on one GPU), and the traffic record
is read only while the kernel sources hash to the recorded value."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_is_tied_to_the_kernel_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0000000000000000")
    assert bench.measured_traffic() is None
