"""Host logic of bench.py (no GPU): more than one GPU is refused with a message, and the
HBM traffic figure is read from the committed counter summary only while the evaluate
kernel's source is the one those counters were taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_profiled_source():
    t = bench.measured_traffic("phimvs_kernels.hip", "eval_kernel_highres_hbm.md")
    # the committed counter summary belongs to the committed kernel (re-profile after a change)
    assert t is not None and t > 1e9
    # any other source (here the PHI kernels) does not match the recorded hash
    assert bench.measured_traffic("phimvs_phi.hip", "eval_kernel_highres_hbm.md") is None
    assert bench.measured_traffic("phimvs_kernels.hip", "no_such_summary.md") is None
