"""bench.py's contract checks that need no device: more than one GPU is
refused with a message, and the extra legs report failures as records."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_cholesky_leg_reports_failure_as_a_record():
    # without a device the leg cannot run; it must say so, not raise
    sys.path.insert(0, ROOT)
    import bench
    import torch
    if torch.cuda.is_available():
        return
    rec = bench.cholesky_leg(16, 1, lambda *a: None)
    assert set(rec) == {"error"}
