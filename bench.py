"""Benchmark: particle-neighbour interactions per second of one SPH
density + force pass on one MI355X.

A step is one full pass of the hot path over the Sedov-blast set (64^3
particles on a jittered lattice in a periodic unit box, u = 1e-5 except
total energy 1 in the 32 central particles, v = 0): the density loop with
the smoothing-length solve to convergence, then the ghost step and the force
loop, issued as one sph_pass (a captured launch sequence with one host
synchronisation). The cells are built once before timing (the build is
reported separately), the starting h is restored before every step, and all
inputs are resident in HBM. The roofline's kernel durations are averages
over as many passes with the same kernels, launched uncaptured by a timing
context with HIP events on their stream. The interaction count of a pass is

    #{(i, j), j != i: r_ij < h_i}  +  #{(i, j), j != i: r_ij < max(h_i, h_j)}

counted once per pass however many Newton sweeps h needed. The same pass in
the plain FP64 form is timed beside it, and the FP64 CPU oracle on the
host's cores.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-neighbour interactions/s (density+force), FP32 batched vs FP64 plain"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (public figure)
PEAK_HBM_GBS = 8000.0

# Algorithmic FLOPs per unit of work (FMA = 2, add/mul/min = 1; sqrt and
# reciprocals listed apart and not counted):
#   a candidate pair tested and rejected            8   (3 sub, r^2, compare)
#   a density interaction at one trial h           26   (+1 sqrt)
#   a force interaction, gather form (per side)    61   (+1 rsqrt, +1 rcp)
FLOP_REJECT = 8
FLOP_DENSITY = 26
FLOP_FORCE = 61


def _workload(name: str):
    import workloads
    if name == "sedov":
        return workloads.sedov(), ("sedov blast 64^3: 262,144 equal-mass particles, jittered lattice, "
                                   "periodic unit box, u=1e-5 with total energy 1 in the 32 central "
                                   "particles, v=0, gamma=5/3, cubic spline, 48 weighted neighbours")
    if name == "small":
        return workloads.small(), "small 16^3 jittered lattice, u=1, v=0"
    if name == "batched":
        return workloads.batched(), "256 periodic boxes of 20^3..40^3 jittered-lattice particles, v~N(0,0.1)"
    if name == "clustered":
        return workloads.clustered(), "2^19 uniform + 64 Plummer spheres x 8192, periodic unit box"
    if name == "large":
        return workloads.lognormal(), "256^3 particles from a log-normal density field"
    raise SystemExit("unknown workload " + name)


def cpu_baseline(d: dict, min_seconds: float) -> dict:
    import oracle
    reps, t_tot, inter = 0, 0.0, 0
    while reps < 1 or (t_tot < min_seconds and reps < 200):
        r = oracle.run(d)
        t_tot += r["t_density"] + r["t_force"]
        inter = int(r["nngb"].sum() + r["npair"].sum())
        reps += 1
    return {"value": inter * reps / t_tot, "unit": "interactions/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": "the full workload (every particle, density with h solved to 1e-13 + force), "
                      "%d repetition(s), %.1f s" % (reps, t_tot)}


KERNEL_SOURCES = {
    "k_density": ["density.hip", "tiles.h", "common.h"],
    "k_force": ["force.hip", "tiles.h", "common.h"],
}


def _kernel_hash(kname: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kname]:
        with open(os.path.join(ROOT, "paper_1508_00115_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic(kname: str, params: dict):
    """HBM bytes per launch of kernel kname from its committed counter profile
    (FETCH_SIZE and WRITE_SIZE, each divided by the factor the same counter
    reads for a device copy of known size), or None when there is no profile,
    or the kernel sources or cell parameters changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_sedov64_traffic.txt" % kname)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "\t", "#", "|")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv["kernel_sources_sha256"] != _kernel_hash(kname) or json.loads(kv["params"]) != params:
            return None
        fetch = float(kv["fetch_bytes_per_launch"]) / float(kv["copy_factor_fetch"])
        write = float(kv["write_bytes_per_launch"]) / float(kv["copy_factor_write"])
    except (KeyError, ValueError):
        return None
    return {"bytes": fetch + write}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sedov")
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--leapfrog-steps", type=int, default=10,
                    help="leapfrog steps timed after the pass (0: none)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="library defaults instead of the autotuner")
    ap.add_argument("--tune", action="store_true", help="re-run the autotuner instead of the stored table")
    ap.add_argument("--tune-out", default=None, help="merge a fresh tuning result into this JSON file")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="MiB of an untimed device copy to calibrate hardware byte counters")
    ap.add_argument("--params", default=None,
                    help='cell parameters as JSON instead of the autotuner, e.g. '
                         '\'{"h_margin": 1.18, "cell_ratio": 0.5, "leaf_target": 32, "schedule": 1}\'')
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only (--gpus %d requested): the library "
              "has no multi-GPU path" % args.gpus, file=sys.stderr)
        return 2

    import torch
    import paper_1508_00115_amd as sph

    dev = torch.device("cuda:0")
    if args.copy_probe > 0:
        # a device-to-device copy of known size, outside the timed region: the
        # hardware byte counters of its kernel calibrate those of the others
        words = int(args.copy_probe * 2 ** 20) // 4
        src = torch.ones(words, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    d, desc = _workload(args.workload)
    n = d["pos"].shape[0]
    stream = torch.cuda.current_stream(dev)
    pos = torch.from_numpy(d["pos"]).to(dev)
    h0 = torch.from_numpy(d["h0"]).to(dev)
    mass = torch.from_numpy(d["mass"]).to(dev)
    vel = torch.from_numpy(d["vel"]).to(dev)
    u = torch.from_numpy(d["u"]).to(dev)
    h = h0.clone()
    rho = torch.empty_like(h)
    f = torch.empty_like(h)
    acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    dudt = torch.empty_like(h)

    tuned = None
    params = {}
    tune_source = "library defaults"
    if args.params:
        params = json.loads(args.params)
        tune_source = "--params"
    elif not args.no_tune:
        from paper_1508_00115_amd import tune
        tuned = None if args.tune else tune.lookup(d)
        tune_source = "stored tuning table"
        if tuned is None:
            tuned = tune.autotune(d, 0)
            tune_source = "autotuned in this run"
            if args.tune_out:
                tune.save(d, tuned, args.tune_out)
        params = tuned["best"]
    # the timed region: density + force as one captured launch sequence (the
    # production configuration)
    ctx = sph.Context(0, **params)
    ctx.build_cells(pos, h0, d["box_first"], d["box_len"])

    def step(c):
        h.copy_(h0)
        return c.pass_(mass, h, vel, u, rho=rho, f=f, acc=acc, dudt=dudt)["stats"]

    for _ in range(args.warmup):
        step(ctx)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        sp = step(ctx)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    inter = sp["interactions_density"] + sp["interactions_force"]
    value = inter / (ms_step * 1e-3)

    # kernel durations: the same passes (the same kernels, the ghost step in
    # the density kernels) launched uncaptured by a timing context, with HIP
    # events on the stream they run on; averages over as many steps
    ctx_t = sph.Context(0, timing=1, **params)
    ctx_t.build_cells(pos, h0, d["box_first"], d["box_len"])
    build_ms = ctx_t.timings()["build_ms"]
    for _ in range(max(args.warmup, 1)):
        step(ctx_t)
    dk, dr, fk, pc = [], [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st_t = step(ctx_t)
        t = ctx_t.timings()
        dk.append(t["density_kernel_ms"] - t["density_rescan_ms"])
        dr.append(t["density_rescan_ms"])
        fk.append(t["force_kernel_ms"])
        pc.append(t["pass_call_ms"])
    torch.cuda.synchronize()
    ms_step_uncaptured = (time.perf_counter() - t0) * 1e3 / args.steps
    ctx_t.close()
    assert st_t["interactions_density"] == sp["interactions_density"]
    assert st_t["interactions_force"] == sp["interactions_force"]
    sd = sf = sp

    # ---- plain FP64 form on the same cells -------------------------------------------
    mass64, vel64, u64 = mass.double(), vel.double(), u.double()
    h0_64 = h0.double()
    h64 = h0_64.clone()
    rho64, f64 = torch.empty_like(h64), torch.empty_like(h64)
    acc64 = torch.empty((n, 3), dtype=torch.float64, device=dev)
    dudt64 = torch.empty_like(h64)

    def step64():
        h64.copy_(h0_64)
        ctx.density_f64(mass64, h64, rho64, f64)
        ctx.force_f64(vel64, u64, acc64, dudt64, cons=False)

    step64()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.fp64_steps):
        step64()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step64 = e0.elapsed_time(e1) / args.fp64_steps
    value64 = inter / (ms_step64 * 1e-3)

    # ---- the same captured pass with the Balsara switch (not part of `value`):
    #      the div/curl pass, the packing and the four-float4 force loop ------------
    ctx_b = sph.Context(0, balsara=1, **params)
    ctx_b.build_cells(pos, h0, d["box_first"], d["box_len"])
    for _ in range(max(args.warmup, 1)):
        step(ctx_b)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step(ctx_b)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_bal = e0.elapsed_time(e1) / args.steps
    ctx_b.close()
    bal = {"ms_per_step": ms_bal, "vs_pass": ms_bal / ms_step, "steps": args.steps,
           "note": "the timed pass with sph_params.balsara = 1 on the same cells"}

    # ---- one leapfrog step (not part of `value`): half kick, drift, prediction,
    #      cell build, pass, half kick and the Courant step, on a context that
    #      records signal velocities --------------------------------------------------------
    lf = None
    if args.leapfrog_steps > 0:
        ctx_l = sph.Context(0, signal_velocity=1, **params)
        pos_l, vel_l, u_l, h_l = pos.clone(), vel.clone(), u.clone(), h0.clone()
        ctx_l.build_cells(pos_l, h_l, d["box_first"], d["box_len"])
        rl = ctx_l.pass_(mass, h_l, vel_l, u_l)
        acc_l, dudt_l, rho_l = rl["acc"], rl["dudt"], rl["rho"]

        def leap():
            dt = ctx_l.timestep(0.3)
            ctx_l.step(dt, pos_l, mass, h_l, vel_l, u_l, acc_l, dudt_l, rho=rho_l)
            return dt

        leap()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.leapfrog_steps):
            dt_last = leap()
        torch.cuda.synchronize()
        lf = {"ms_per_step": (time.perf_counter() - t0) * 1e3 / args.leapfrog_steps,
              "steps": args.leapfrog_steps, "courant": 0.3, "last_dt": dt_last,
              "build_ms": ctx_l.timings()["build_ms"],
              "note": "wall time per step from the host (kick, drift, kick, pass with a cell rebuild "
                      "when the drift bound requires one, kick, time step), after one untimed step"}
        ctx_l.close()

    # ---- roofline of the dominant kernel ------------------------------------------------
    dens_ms = float(np.mean(dk))  # the list kernel alone (the re-scan kernel is timed apart)
    force_ms = float(np.mean(fk))
    dens_alg = FLOP_DENSITY * sd["sweep_interactions_density"] + \
        FLOP_REJECT * (sd["candidates_density"] - sd["sweep_interactions_density"])
    force_alg = FLOP_FORCE * sf["interactions_force"] + \
        FLOP_REJECT * (sf["candidates_force"] - sf["interactions_force"])
    if dens_ms >= force_ms:
        kname, kms, alg = "k_density", dens_ms, dens_alg
    else:
        kname, kms, alg = "k_force", force_ms, force_alg
    achieved = alg / (kms * 1e-3) / 1e12
    traffic = _traffic(kname, params)
    useful = (FLOP_DENSITY * sd["sweep_interactions_density"] + FLOP_FORCE * sf["interactions_force"]) / \
        ((dens_ms + force_ms) * 1e-3) / 1e12

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "particles": n, "interactions_per_pass": inter,
                   "density_interactions": sd["interactions_density"],
                   "force_interactions": sf["interactions_force"], "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": None if traffic is None else traffic["bytes"],
                     "traffic_unit": "bytes per launch (HBM, from hardware counters)",
                     "traffic_gbs": None if traffic is None else traffic["bytes"] / (kms * 1e-3) / 1e9,
                     "avg_kernel_ms": kms, "algorithmic_flop_per_launch": alg},
        "ms_per_step_uncaptured_with_events": ms_step_uncaptured,
        "kernels_ms": {"density_kernel": dens_ms, "density_rescan_kernel": float(np.mean(dr)),
                       "force_kernel": force_ms, "pass_gpu": float(np.mean(pc)), "build": build_ms},
        "useful_tflops": useful,
        "density": {"sweeps": sd["sweeps"], "rebuilds": sd["rebuilds"],
                    "candidates": sd["candidates_density"],
                    "sweep_interactions": sd["sweep_interactions_density"],
                    "candidates_per_interaction": sd["candidates_density"] / max(1, sd["interactions_density"]),
                    "cells": sd["n_cells"], "cell_pairs": sd["n_pairs"]},
        "force": {"candidates": sf["candidates_force"],
                  "candidates_per_interaction": sf["candidates_force"] / max(1, sf["interactions_force"])},
        "fp64_plain": {"value": value64, "ms_per_step": ms_step64, "steps": args.fp64_steps},
        "speedup_vs_fp64_plain": value / value64,
        "leapfrog": lf,
        "balsara": bal,
        "cell_params": params or "library defaults",
        "cell_params_from": tune_source,
        "autotune_top5": None if tuned is None else [
            {**t["params"], "ms": t["ms"], "rebuilds": t.get("rebuilds")}
            for t in sorted((t for t in tuned["table"] if t["ms"] is not None), key=lambda t: t["ms"])[:5]],
        "autotune_settings": None if tuned is None else len(tuned["table"]),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
