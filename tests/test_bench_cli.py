"""Host-side checks of the benchmark's command line (no GPU needed): more
than one GPU is refused with a message and exit status 2 before anything
touches a device, and the scheme option is known."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_bench_help_lists_the_options():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--workload", "--precision", "--scheme", "--midplane-bins"):
        assert opt in r.stdout, opt


def test_oracle_child_job_writes_its_sample(tmp_path):
    """The benchmark's CPU baseline runs the oracle in a child interpreter:
    on the small 2D workload it writes the state after the warm-up step and
    the timed steps, the last record and the three timings."""
    import json

    import numpy as np
    out = str(tmp_path / "o.npz")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-job", "c1", "2", "0", out],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    assert "timed step 2 of 2 done" in r.stderr
    z = np.load(out)
    d = json.loads(str(z["diag"]))
    assert d["step"] == 3 and z["state"][0] == 3
    assert z["times"].shape == (3,) and (z["times"] > 0).all() and int(z["steps"]) == 2
