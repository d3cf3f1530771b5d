"""The benchmark's command line without a GPU: more than one GPU is refused
with a message, and an oracle worker of the all-cores CPU baseline runs its
(iteration, T_inner, packet range) jobs and reports counters that add up."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_cpu_worker_reports_its_range():
    def run(jobs):
        r = subprocess.run([sys.executable, BENCH, "--cpu-worker", json.dumps(jobs)],
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr
        return json.loads(r.stdout.strip().splitlines()[-1])

    # two iterations at different temperatures, split at packet 40
    a = run([[0, 9000.0, 0, 40], [3, 30000.0, 0, 40]])
    b = run([[0, 9000.0, 40, 100], [3, 30000.0, 40, 100]])
    ab = run([[0, 9000.0, 0, 100], [3, 30000.0, 0, 100]])
    for k in ("segments", "line_events", "escatters", "escaped", "reabsorbed"):
        assert a["counters"][k] + b["counters"][k] == ab["counters"][k], k
    assert ab["counters"]["escaped"] + ab["counters"]["reabsorbed"] == 200
    assert ab["seconds"] > 0.0
    hot = run([[3, 30000.0, 0, 100]])
    cold = run([[0, 9000.0, 0, 100]])
    for k in ("segments", "line_events"):
        assert hot["counters"][k] + cold["counters"][k] == ab["counters"][k], k
