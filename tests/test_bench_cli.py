"""CPU checks of bench.py's command line: one GPU only (a request for more
exits with status 2 and says so, before touching a device)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_studies():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for flag in ["--workload", "--tree-study", "--qr-node", "--qr-pod", "--right-vectors", "--block-gram",
                 "--calibrate-copy"]:
        assert flag in r.stdout
