"""Host check of the benchmark's command-line contract: more than one GPU is
refused with a message and a non-zero status, before any device work."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300, cwd=ROOT)
    assert p.returncode != 0
    line = p.stdout.strip().splitlines()[-1]
    msg = json.loads(line)
    assert "error" in msg and "one GPU" in msg["error"]
