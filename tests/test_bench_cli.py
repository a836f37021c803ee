"""bench.py's command line on the CPU: it runs on one GPU only and says so for --gpus N > 1
(before touching a device), and every study mode it documents is accepted by its parser."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_help_lists_the_study_modes():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 0
    for flag in ("--steps", "--warmup", "--precision", "--ksweep", "--learned", "--multi", "--window-sweep",
                 "--kernel-only", "--proj-only", "--net-only"):
        assert flag in p.stdout, flag
