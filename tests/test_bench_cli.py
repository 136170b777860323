"""The benchmark's command line without a GPU: more than one GPU is refused
with a JSON message (the library and benchmark use one GPU), and the
workload table names every benchmark workload with its sizes."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_workloads_and_default():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.DEFAULT_WORKLOAD == "perm4"
    assert {"plain1", "plain2", "plain3", "perm4", "uneven5", "pairs3", "quads2"} <= set(bench.WORKLOADS)
    for name, wl in bench.WORKLOADS.items():
        assert wl["desc"], name
