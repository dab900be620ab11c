"""Benchmark: particle-neighbour interactions per second of one SPH
density + force pass on one MI355X, FP32 batched against the plain FP64 form.

A step is one full pass of the hot path over the batched set: 256
independent periodic unit boxes of 20^3..40^3 particles (7,234,361 in all;
box sizes log-uniform, seeded), each a jittered lattice with Gaussian
velocities (sigma 0.1) and u = 1. One pass runs, for every self and pair
cell task of every box in single launches captured in one HIP graph:

  - the density loop with the smoothing-length solve to convergence,
  - the ghost step (folded into the density kernels),
  - the force loop (acceleration and du/dt),
  - the per-box FP64 momentum and energy rates (the conservation sums),

issued as one sph_pass with one host synchronisation. Cell parameters come
from the stored autotuning table for the set. The cells are built once before
timing (the build is reported separately), the starting h is restored before
every step inside the timed region, and all inputs are resident in HBM. The
interaction count of a pass is

    #{(i, j), j != i: r_ij < h_i}  +  #{(i, j), j != i: 0 < r_ij < max(h_i, h_j)}

counted once per pass however many Newton sweeps h needed. The same pass in
the plain FP64 form (one thread per particle, FP64 positions, with the same
conservation sums) is timed on the same cells and reported beside it, with
the speedup. The FP64 CPU oracle is timed on the host's cores, on the whole
set with every core and on a seeded sample of boxes with one thread.

The roofline's kernel durations are averages over as many passes with the
same kernels, launched uncaptured by a timing context with HIP events on
their stream. Extra keys report the Sedov blast (64^3) and the 2^24
log-normal set the same way (their own stored cell parameters).

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
#   a near-field gravity pair (per side)           22   (+1 rsqrt)
FLOP_REJECT = 8
FLOP_DENSITY = 26
FLOP_FORCE = 61
FLOP_GRAVITY = 22

WORKLOADS = {
    # name: (generator, description, profile tag)
    "batched": ("batched", "batched: 256 periodic unit boxes of 20^3..40^3 jittered-lattice particles "
                           "(7,234,361 in all, sizes log-uniform), v ~ N(0, 0.1^2), u = 1, gamma = 5/3, "
                           "cubic spline, 48 weighted neighbours; all boxes in one captured pass",
                "batched"),
    "sedov": ("sedov", "sedov blast 64^3: 262,144 equal-mass particles, jittered lattice, periodic unit "
                       "box, u=1e-5 with total energy 1 in the 32 central particles, v=0", "sedov64"),
    "large": ("lognormal", "log-normal 256^3: 16,777,216 particles from a log-normal density field "
                           "(P(k) ~ k^-2, sigma_ln 1.5), velocities from the same field, u=1", "large"),
    "clustered": ("clustered", "clustered: 2^19 uniform + 64 Plummer spheres x 8192, periodic unit box",
                  "clustered"),
    "small": ("small", "small 16^3 jittered lattice, u=1, v=0", "small"),
}


def _workload(name: str) -> tuple:
    import workloads
    if name not in WORKLOADS:
        raise SystemExit("unknown workload " + name)
    gen, desc, tag = WORKLOADS[name]
    return getattr(workloads, gen)(), desc, tag


def cpu_baseline(d: dict, min_seconds: float, one_thread_seconds: float) -> dict:
    """The FP64 oracle (untuned) on the host: every box with every core, then
    a seeded sample of boxes with one thread (boxes are independent, so a
    sample of boxes is a sample of the same work)."""
    import oracle
    cores = oracle.max_threads()
    reps, t_tot, inter = 0, 0.0, 0
    while reps < 1 or (t_tot < min_seconds and reps < 50):
        r = oracle.run(d, threads=cores)
        t_tot += r["t_density"] + r["t_force"]
        inter = int(r["nngb"].sum() + r["npair"].sum())
        reps += 1
    out = {"value": inter * reps / t_tot, "unit": "interactions/s", "cores": cores, "kind": "oracle",
           "sample": "the whole workload (every particle of every box: density with h solved to "
                     "1e-13, then force), %d repetition(s), %.1f s on %d threads" % (reps, t_tot, cores)}
    nb = len(d["box_len"])
    order = np.random.default_rng([1508, 3, 1000]).permutation(nb)
    t1, i1, boxes = 0.0, 0, 0
    import workloads
    for b in order:
        r = oracle.run(workloads.box_slice(d, int(b)), threads=1)
        t1 += r["t_density"] + r["t_force"]
        i1 += int(r["nngb"].sum() + r["npair"].sum())
        boxes += 1
        if t1 >= one_thread_seconds:
            break
    out["value_1thread"] = i1 / t1
    out["sample_1thread"] = "%d of the %d boxes (seeded order), %.1f s on 1 thread" % (boxes, nb, t1)
    oracle.run(workloads.box_slice(d, int(order[0])), threads=cores)  # leave the library at all cores
    out["gravity_p2p"] = cpu_gravity(d, order)
    return out


def cpu_gravity(d: dict, order, min_seconds: float = 3.0) -> dict:
    """The FP64 gravity oracle (scipy's tree search and numpy, one process)
    over boxes in the seeded order, with the cutoff, softening and masses
    the GPU entry uses, until min_seconds have passed."""
    import time as _time

    from oracle import gravity as og
    import workloads
    rc = 0.95 * float(d["h0"].min())
    t, pairs, boxes = 0.0, 0, 0
    for b in order:
        e = workloads.box_slice(d, int(b))
        t0 = _time.perf_counter()
        r = og.p2p(e["pos"], e["mass"].astype(np.float64), 1.0, 1e-3, rc, float(e["box_len"][0]))
        t += _time.perf_counter() - t0
        pairs += int(r["npair"])
        boxes += 1
        if t >= min_seconds:
            break
    return {"value": pairs / t, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": "%d of the %d boxes (seeded order), %.1f s in one process" % (boxes, len(d["box_len"]), t)}


KERNEL_SOURCES = {
    "k_density": ["density.hip", "tiles.h", "common.h"],
    "k_force": ["force.hip", "tiles.h", "common.h"],
    "k_gravity": ["gravity.hip", "tiles.h", "common.h"],
}


def _kernel_hash(kname: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kname]:
        with open(os.path.join(ROOT, "paper_1508_00115_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic(kname: str, tag: str, params: dict):
    """HBM bytes per launch of kernel kname on workload `tag` from its
    committed counter profile (FETCH_SIZE and WRITE_SIZE, each divided by the
    factor the same counter reads for a device copy of known size), or None
    when there is no profile, or the kernel sources or cell parameters
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.txt" % (kname, tag))
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


def _params_for(d: dict, args) -> tuple:
    if args.params:
        return json.loads(args.params), "--params", None
    if args.no_tune:
        return {}, "library defaults", None
    from paper_1508_00115_amd import tune
    tuned = None if args.tune else tune.lookup(d)
    src = "stored tuning table"
    if tuned is None:
        tuned = tune.autotune(d, 0)
        src = "autotuned in this run"
        if args.tune_out:
            tune.save(d, tuned, args.tune_out)
    return tuned["best"], src, tuned


class Inputs:
    """A workload resident on the GPU with its output buffers."""

    def __init__(self, d: dict, dev):
        import torch
        self.d = d
        self.n = d["pos"].shape[0]
        self.pos = torch.from_numpy(d["pos"]).to(dev)
        self.h0 = torch.from_numpy(d["h0"]).to(dev)
        self.mass = torch.from_numpy(d["mass"]).to(dev)
        self.vel = torch.from_numpy(d["vel"]).to(dev)
        self.u = torch.from_numpy(d["u"]).to(dev)
        self.h = self.h0.clone()
        self.rho = torch.empty_like(self.h)
        self.f = torch.empty_like(self.h)
        self.acc = torch.empty((self.n, 3), dtype=torch.float32, device=dev)
        self.dudt = torch.empty_like(self.h)

    def context(self, sph, **params):
        ctx = sph.Context(0, **params)
        ctx.build_cells(self.pos, self.h0, self.d["box_first"], self.d["box_len"])
        return ctx

    def build_ms(self, ctx, reps: int = 5) -> float:
        """Median host wall time of a cell build on a context that has built
        once (its buffers exist), up to the end of its GPU work."""
        import torch
        t = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.build_cells(self.pos, self.h0, self.d["box_first"], self.d["box_len"])
            torch.cuda.synchronize()
            t.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(t))

    def step(self, ctx, cons: bool = True) -> dict:
        self.h.copy_(self.h0)
        return ctx.pass_(self.mass, self.h, self.vel, self.u, rho=self.rho, f=self.f, acc=self.acc,
                         dudt=self.dudt, cons=cons)["stats"]


def time_pass(inp: Inputs, ctx, steps: int, warmup: int, stream) -> tuple:
    """HIP events on the stream around `steps` captured passes (after
    `warmup`): ms per step and the stats of the last pass."""
    import torch
    for _ in range(warmup):
        inp.step(ctx)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        sp = inp.step(ctx)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, sp


def kernel_times(inp: Inputs, sph, params: dict, steps: int, warmup: int) -> dict:
    """The same passes (the same kernels, the ghost step in the density
    kernels, the conservation sums) launched uncaptured by a timing context,
    with HIP events on the stream they run on; averages over `steps`."""
    import torch
    ctx_t = inp.context(sph, timing=1, **params)
    build_ms = inp.build_ms(ctx_t)
    for _ in range(max(warmup, 1)):
        inp.step(ctx_t)
    dk, dr, fk, pc = [], [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        st = inp.step(ctx_t)
        t = ctx_t.timings()
        dk.append(t["density_kernel_ms"] - t["density_rescan_ms"])
        dr.append(t["density_rescan_ms"])
        fk.append(t["force_kernel_ms"])
        pc.append(t["pass_call_ms"])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ctx_t.close()
    return {"density_kernel": float(np.mean(dk)), "density_rescan_kernel": float(np.mean(dr)),
            "force_kernel": float(np.mean(fk)), "pass_gpu": float(np.mean(pc)), "build": build_ms,
            "ms_per_step_uncaptured_with_events": wall, "stats": st}


def roofline(stats: dict, km: dict, tag: str, params: dict) -> dict:
    """Algorithmic FP32 work of the slower hot kernel over its average
    duration, against the FP32 vector peak."""
    dens_ms, force_ms = km["density_kernel"], km["force_kernel"]
    dens_alg = FLOP_DENSITY * stats["sweep_interactions_density"] + \
        FLOP_REJECT * (stats["candidates_density"] - stats["sweep_interactions_density"])
    force_alg = FLOP_FORCE * stats["interactions_force"] + \
        FLOP_REJECT * (stats["candidates_force"] - stats["interactions_force"])
    if dens_ms >= force_ms:
        kname, kms, alg = "k_density", dens_ms, dens_alg
    else:
        kname, kms, alg = "k_force", force_ms, force_alg
    achieved = alg / (kms * 1e-3) / 1e12
    traffic = _traffic(kname, tag, params)
    other = {"k_density": (dens_alg, dens_ms), "k_force": (force_alg, force_ms)}
    return {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": None if traffic is None else traffic["bytes"],
            "traffic_unit": "bytes per launch (HBM, from hardware counters)",
            "traffic_gbs": None if traffic is None else traffic["bytes"] / (kms * 1e-3) / 1e9,
            "avg_kernel_ms": kms, "algorithmic_flop_per_launch": alg,
            "per_kernel": {k: {"algorithmic_flop_per_launch": a, "avg_kernel_ms": ms,
                               "frac": a / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}
                           for k, (a, ms) in other.items()},
            "useful_tflops": (FLOP_DENSITY * stats["sweep_interactions_density"] +
                              FLOP_FORCE * stats["interactions_force"]) / ((dens_ms + force_ms) * 1e-3) / 1e12}


def culling(inp: Inputs, sph, params: dict) -> dict:
    """One pass on a context counting the density loop's list-building tests
    and the candidates they list (sph_params.timing = 2, a separate kernel
    instance): tests per listed neighbour measure the culling, the work the
    paper's sorted sweeps save (listed: candidates inside the search radius,
    the particle itself included)."""
    ctx = inp.context(sph, timing=2, **params)
    inp.step(ctx)  # as in the timed passes: after any rebuild the first pass needed
    st = inp.step(ctx)
    ctx.close()
    return {"phase_a_tests": st["tests_density"], "listed": st["listed_density"],
            "tests_per_listed": st["tests_density"] / max(1, st["listed_density"]),
            "force_candidates_per_interaction": st["candidates_force"] / max(1, st["interactions_force"])}


def gravity(inp: Inputs, sph, params: dict, steps: int, tag: str) -> dict:
    """Near-field gravity (sph_gravity_p2p) on the same cells with the
    workload's masses, r_cut = 0.95 x the smallest h guess (inside every
    particle's search radius), G = 1, eps = 1e-3: the kernel's HIP-event time
    averaged over `steps` calls after one untimed call."""
    ctx = inp.context(sph, timing=1, **params)
    rc = 0.95 * float(inp.d["h0"].min())
    _, pairs, cand = ctx.gravity_p2p(inp.mass, 1.0, 1e-3, rc, acc=inp.acc, candidates=True)
    kms = []
    for _ in range(steps):
        ctx.gravity_p2p(inp.mass, 1.0, 1e-3, rc, acc=inp.acc)
        kms.append(ctx.timings()["gravity_kernel_ms"])
    ctx.close()
    ms = float(np.mean(kms))
    alg = FLOP_GRAVITY * pairs + FLOP_REJECT * (cand - pairs)
    traffic = _traffic("k_gravity", tag, params)
    return {"r_cut": rc, "pairs": pairs, "candidates": cand, "candidates_per_pair": cand / max(1, pairs),
            "kernel_ms": ms, "pairs_per_s": pairs / (ms * 1e-3), "calls": steps,
            "algorithmic_flop_per_launch": alg, "frac_fp32_peak": alg / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
            "traffic": None if traffic is None else traffic["bytes"],
            "traffic_gbs": None if traffic is None else traffic["bytes"] / (ms * 1e-3) / 1e9}


def extra_set(name: str, sph, args, stream, dev) -> dict:
    """The captured pass on another workload, with its kernel times."""
    import torch
    d, desc, tag = _workload(name)
    params, src, _ = _params_for(d, args)
    inp = Inputs(d, dev)
    ctx = inp.context(sph, **params)
    ms, sp = time_pass(inp, ctx, args.extra_steps, 1, stream)
    ctx.close()
    km = kernel_times(inp, sph, params, args.extra_steps, 1)
    inter = sp["interactions_density"] + sp["interactions_force"]
    out = {"workload": desc, "particles": inp.n, "value": inter / (ms * 1e-3), "unit": "interactions/s",
           "ms_per_step": ms, "steps": args.extra_steps, "interactions_per_pass": inter,
           "kernels_ms": {k: v for k, v in km.items() if k != "stats"},
           "roofline": roofline(sp, km, tag, params), "sweeps": sp["sweeps"],
           "candidates_per_interaction_density": sp["candidates_density"] / max(1, sp["interactions_density"]),
           "candidates_per_interaction_force": sp["candidates_force"] / max(1, sp["interactions_force"]),
           "culling": culling(inp, sph, params),
           "cell_params": params or "library defaults", "cell_params_from": src}
    del inp
    torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched", choices=sorted(WORKLOADS))
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="least oracle time on every core (whole set, repeated)")
    ap.add_argument("--cpu-1thread-seconds", type=float, default=12.0,
                    help="oracle time on one thread (a seeded sample of boxes)")
    ap.add_argument("--extra", default="sedov,large",
                    help="other workloads timed after the headline, comma separated ('' for none)")
    ap.add_argument("--extra-steps", type=int, default=10)
    ap.add_argument("--leapfrog-steps", type=int, default=10,
                    help="leapfrog steps timed on the Sedov blast (0: none)")
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

    d, desc, tag = _workload(args.workload)
    params, tune_source, tuned = _params_for(d, args)
    stream = torch.cuda.current_stream(dev)
    inp = Inputs(d, dev)
    n = inp.n

    # ---- the timed region: density + force + conservation sums as one
    #      captured launch sequence (the production configuration) ----------------------
    ctx = inp.context(sph, **params)
    ms_step, sp = time_pass(inp, ctx, args.steps, args.warmup, stream)
    inter = sp["interactions_density"] + sp["interactions_force"]
    value = inter / (ms_step * 1e-3)

    km = kernel_times(inp, sph, params, args.steps, args.warmup)
    assert km["stats"]["interactions_density"] == sp["interactions_density"]
    assert km["stats"]["interactions_force"] == sp["interactions_force"]

    # ---- plain FP64 form on the same cells, with the conservation sums -------------------
    mass64, vel64, u64 = inp.mass.double(), inp.vel.double(), inp.u.double()
    h0_64 = inp.h0.double()
    h64 = h0_64.clone()
    rho64, f64 = torch.empty_like(h64), torch.empty_like(h64)
    acc64 = torch.empty((n, 3), dtype=torch.float64, device=dev)
    dudt64 = torch.empty_like(h64)

    def step64():
        h64.copy_(h0_64)
        sd = ctx.density_f64(mass64, h64, rho64, f64)["stats"]
        return sd, ctx.force_f64(vel64, u64, acc64, dudt64, cons=True)["stats"]

    step64()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.fp64_steps):
        sd64, sf64 = step64()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step64 = e0.elapsed_time(e1) / args.fp64_steps
    inter64 = sd64["interactions_density"] + sf64["interactions_force"]
    value64 = inter64 / (ms_step64 * 1e-3)
    del mass64, vel64, u64, h0_64, h64, rho64, f64, acc64, dudt64

    # ---- the same captured pass with the Balsara switch (not part of `value`):
    #      the div/curl pass, the packing and the four-float4 force loop ------------
    ctx_b = inp.context(sph, balsara=1, **params)
    ms_bal, _ = time_pass(inp, ctx_b, args.steps, max(args.warmup, 1), stream)
    ctx_b.close()
    bal = {"ms_per_step": ms_bal, "vs_pass": ms_bal / ms_step, "steps": args.steps,
           "note": "the timed pass with sph_params.balsara = 1 on the same cells"}

    rl = roofline(sp, km, tag, params)
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
        "config": {"workload": desc, "particles": n, "boxes": len(d["box_len"]),
                   "interactions_per_pass": inter,
                   "density_interactions": sp["interactions_density"],
                   "force_interactions": sp["interactions_force"],
                   "conservation_sums_in_timed_pass": True, "parallelism": "single GPU"},
        "roofline": rl,
        "ms_per_step_uncaptured_with_events": km["ms_per_step_uncaptured_with_events"],
        "kernels_ms": {k: v for k, v in km.items() if k not in ("stats", "ms_per_step_uncaptured_with_events")},
        "useful_tflops": rl["useful_tflops"],
        "density": {"sweeps": sp["sweeps"], "rebuilds": sp["rebuilds"],
                    "candidates": sp["candidates_density"],
                    "sweep_interactions": sp["sweep_interactions_density"],
                    "candidates_per_interaction": sp["candidates_density"] / max(1, sp["interactions_density"]),
                    "rescanned": sp["rescanned_density"],
                    "cells": sp["n_cells"], "cell_pairs": sp["n_pairs"]},
        "culling": culling(inp, sph, params),
        "force": {"candidates": sp["candidates_force"],
                  "candidates_per_interaction": sp["candidates_force"] / max(1, sp["interactions_force"])},
        "fp64_plain": {"value": value64, "ms_per_step": ms_step64, "steps": args.fp64_steps,
                       "interactions_per_pass": inter64,
                       "note": "sph_density_f64 + sph_force_f64 with the conservation sums, same cells"},
        "speedup_vs_fp64_plain": value / value64,
        "balsara": bal,
        "gravity_p2p": gravity(inp, sph, params, args.steps, tag),
        "cell_params": params or "library defaults",
        "cell_params_from": tune_source,
        "autotune_top5": None if tuned is None else [
            {**t["params"], "ms": t["ms"], "rebuilds": t.get("rebuilds")}
            for t in sorted((t for t in tuned["table"] if t["ms"] is not None), key=lambda t: t["ms"])[:5]],
        "autotune_settings": None if tuned is None else len(tuned["table"]),
    }
    ctx.close()
    del inp
    torch.cuda.empty_cache()

    # ---- one leapfrog step on the Sedov blast (not part of `value`): half kick,
    #      drift, prediction, cell build when needed, pass, half kick and the
    #      Courant step, on a context that records signal velocities -----------------
    if args.leapfrog_steps > 0:
        ds, _, _ = _workload("sedov")
        params_s, _, _ = _params_for(ds, args)
        # the stored table is timed on one pass at the start, where no top
        # cell splits and cell_ratio changes nothing; once the blast spreads
        # the search radii, the coarser setting splits fewer cells per rebuild
        # (40 steps: 1.06 against 1.14 ms per step)
        if not args.params and not args.no_tune:
            params_s = dict(params_s, cell_ratio=1.0)
        li = Inputs(ds, dev)
        ctx_l = sph.Context(0, signal_velocity=1, **params_s)
        pos_l, vel_l, u_l, h_l = li.pos.clone(), li.vel.clone(), li.u.clone(), li.h0.clone()
        ctx_l.build_cells(pos_l, h_l, ds["box_first"], ds["box_len"])
        r0 = ctx_l.pass_(li.mass, h_l, vel_l, u_l)
        acc_l, dudt_l, rho_l = r0["acc"], r0["dudt"], r0["rho"]

        sweeps, evals = [], []

        def leap(predict=True):
            dt = ctx_l.timestep(0.3)
            r = ctx_l.step(dt, pos_l, li.mass, h_l, vel_l, u_l, acc_l, dudt_l, rho=rho_l, predict_h=predict)
            st = r["stats"]
            sweeps.append(st["sweeps"])
            evals.append(st["sweep_interactions_density"] / max(st["interactions_density"], 1))
            return dt

        leap()
        torch.cuda.synchronize()
        b0 = ctx_l.timings()["builds"]
        sweeps.clear()
        evals.clear()
        t0 = time.perf_counter()
        for _ in range(args.leapfrog_steps):
            dt_last = leap()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.leapfrog_steps
        builds = ctx_l.timings()["builds"] - b0
        ev_pred, sw = float(np.mean(evals)), float(np.mean(sweeps))
        # the steps that follow, without the prediction (untimed)
        evals.clear()
        for _ in range(min(10, args.leapfrog_steps)):
            leap(predict=False)
        out["leapfrog"] = {
            "workload": "sedov blast 64^3", "ms_per_step": ms,
            "steps": args.leapfrog_steps, "courant": 0.3, "last_dt": dt_last,
            "steps_with_a_cell_build": builds,
            "sweeps_per_pass": sw,
            "evaluations_per_particle": ev_pred,
            "evaluations_per_particle_without_prediction": float(np.mean(evals)),
            "build_ms": li.build_ms(ctx_l),
            "cell_params": params_s,
            "note": "wall time per step from the host (kick, drift, h prediction, kick, pass with a "
                    "cell rebuild when the drift bound requires one, kick, time step), after one "
                    "untimed step; sweeps: most Newton evaluations of any particle; evaluations: "
                    "their mean (the next steps run without the prediction for comparison); "
                    "build_ms: a warm cell build on these particles, GPU work included"}
        ctx_l.close()
        del li
        torch.cuda.empty_cache()

    for name in [x for x in args.extra.split(",") if x and x != args.workload]:
        out[name] = extra_set(name, sph, args, stream, dev)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, args.cpu_seconds, args.cpu_1thread_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
