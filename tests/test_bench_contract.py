"""The benchmark's command-line contract (CPU only: nothing here touches a GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_byte_counts():
    sys.path.insert(0, ROOT)
    import bench
    # stage 1 moves 9 FP32 values per cell, stages 2 and 3 twelve, the physics seven: 160 B per cell-step
    assert (sum(bench.VALUES_STAGE.values()) + bench.VALUES_PHYSICS) * 4 == 160
    assert bench.MLP_FLOPS_PER_COL == 944128
    assert bench.PAPER_RW_K20X_S[(256, 256, 512)] == 2.16
