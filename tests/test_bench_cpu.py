"""CPU checks of bench.py's contract: one GPU only, and the hardware-counter
profiles under profiles/ are used only for the kernel sources and cell
parameters they were taken with (their HBM bytes are reported only then,
null otherwise)."""

import glob
import json
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


def _fields(path):
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "\t", "#", "|")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def test_traffic_profiles_are_well_formed():
    paths = glob.glob(os.path.join(ROOT, "profiles", "*_traffic.txt"))
    assert paths, "no counter profile under profiles/"
    for p in paths:
        kv = _fields(p)
        for k in ("kernel", "params", "kernel_sources_sha256", "fetch_bytes_per_launch",
                  "write_bytes_per_launch", "copy_factor_fetch", "copy_factor_write"):
            assert k in kv, (p, k)
        with open(p) as fh:
            assert "rocprofv3 --pmc FETCH_SIZE" in fh.read(), p
        json.loads(kv["params"])
        tag = os.path.basename(p)[len(kv["kernel"]) + 1:-len("_traffic.txt")]
        t = bench._traffic(kv["kernel"], tag, json.loads(kv["params"]))
        # current sources: the bytes are reported; changed sources: null
        if kv["kernel_sources_sha256"] == bench._kernel_hash(kv["kernel"]):
            assert t is not None and t["bytes"] > 1e6
        else:
            assert t is None


def test_traffic_needs_the_same_parameters():
    params = dict(tune.lookup(workloads.batched())["best"])
    params["h_margin"] = 1.3
    assert bench._traffic("k_density", "batched", params) is None
    assert bench._traffic("k_force", "batched", params) is None
