"""bench.py's command line on the CPU: more than one GPU is refused with a
message before any device work starts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    msg = r.stdout + r.stderr
    assert "one GPU" in msg
    assert "{" not in r.stdout          # no JSON line is printed
