"""bench.py's host-side contract (no GPU): it refuses more than one GPU
before touching one, and the hash that keys its stored traffic figure finds
the projector source regions it covers."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_projector_source_hash_covers_its_regions():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.projector_src_hash()
    assert h is not None and len(h) == 16
    int(h, 16)
