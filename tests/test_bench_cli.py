"""The benchmark's command-line contract on the host: a request for more
than one GPU ends with a message (this build measures one GPU), and every
workload name is accepted by the parser."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_workloads_are_listed():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 0
    for name in ("satellite_spacetime", "batched_uneven", "surrogate_plane", "sweep", "predict",
                 "neighbours", "attributes_18d", "grouped_plane", "pipeline"):
        assert name in p.stdout
