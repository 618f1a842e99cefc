"""The benchmark's host-side contract (CPU only): one GPU only, and the
tuned 11-level leg has a pick to run from the committed table."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_tuned_leg_has_a_pick():
    with open(os.path.join(ROOT, "paper_2606_10477_amd", "tuning_mi355x_bts11.json")) as f:
        rep = json.load(f)
    top = max(int(l) for l in rep["table"])
    pick = rep["table"][str(top)]["3.1e-08"]
    assert top == 11 and pick is not None and pick["mre"] <= 3.1e-8
