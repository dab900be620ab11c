"""CPU checks of bench.py's contract: one GPU only, and the hardware-counter
profiles under profiles/ belong to the kernel sources and cell parameters the
benchmark runs (their HBM bytes are reported only then)."""

import os
import subprocess
import sys

import bench
import workloads
from paper_1508_00115_amd import tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_profiles_match_the_kernels():
    params = tune.lookup(workloads.sedov())["best"]
    for kname in ("k_density", "k_force"):
        t = bench._traffic(kname, params)
        assert t is not None, "%s: profiles/ was taken from other sources or parameters" % kname
        assert t["bytes"] > 1e6


def test_traffic_needs_the_same_parameters():
    params = dict(tune.lookup(workloads.sedov())["best"])
    params["h_margin"] = 1.3
    assert bench._traffic("k_density", params) is None
