"""Autotuner for the cell parameters of the library.

The parameters it searches change only how the work is cut, never the
result (h is the unique root, and every pair within reach is found for any
legal cell layout):

    h_margin     search radius over the starting h: candidates per particle
                 grow like h_margin^3, but h may grow by this factor before
                 the cells must be rebuilt
    cell_ratio   smallest cell width below the top grid, in search radii
    leaf_target  cells holding more particles than this are split
    schedule     hardware dispatch or persistent per-XCD queues
    tile_cap     candidates the density kernel keeps resident in LDS
    cell_order   cells by decreasing cost (balance), in Morton order (L2 reuse), or
                 Morton ranges per XCD each ordered by cost

Each setting is timed on the caller's particles as whole density + force
passes (sph_pass, after a warm-up, HIP events around the calls); the fastest
wins, where settings within 1% of it count as equal and the XCD-local cell
orders win such ties (less traffic beyond the L2 at the same speed). Results are
kept in a JSON file keyed by a signature of the particle set; ``tuned.json``
beside this module holds the results shipped with the library.

    python -m paper_1508_00115_amd.tune --workload sedov --out FILE

re-tunes a named synthetic workload on GPU 0 and merges the result into FILE.
"""

from __future__ import annotations

import hashlib
import json
import os

import numpy as np

DEFAULT_GRID = [
    {"h_margin": m, "cell_ratio": cr, "leaf_target": lt, "schedule": s, "tile_cap": tc, "cell_order": co}
    for m in (1.05, 1.1, 1.18, 1.26)
    for cr in (1.0, 0.5)
    for lt in (64, 32)
    for s in (0, 1)
    for tc in (128, 512)
    for co in (0, 1, 2)
]


STORE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def signature(d: dict) -> str:
    """Key of a particle set: sizes, box layout and summary statistics of h0."""
    h = np.asarray(d["h0"], dtype=np.float64)
    parts = [d["pos"].shape[0], len(d["box_len"]), float(h.min()), float(h.max()), float(h.mean()),
             hashlib.sha1(np.ascontiguousarray(d["box_first"]).tobytes()).hexdigest()[:12]]
    return json.dumps(parts)


def lookup(d: dict, store: str = STORE) -> dict | None:
    """The stored tuning result of particle set ``d``, or None."""
    try:
        with open(store) as fh:
            return json.load(fh).get(signature(d))
    except (OSError, ValueError):
        return None


def save(d: dict, result: dict, store: str) -> None:
    """Merge a tuning result for particle set ``d`` into the JSON file ``store``."""
    try:
        with open(store) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        table = {}
    table[signature(d)] = result
    with open(store, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)


def autotune(d: dict, device: int = 0, grid=None, reps: int = 5, cache: str | None = None,
             progress: bool = False) -> dict:
    """Time every setting of ``grid`` on workload ``d`` (a dict as produced by
    the ``workloads`` package) and return {"best": params, "table": [...]}.
    progress: print one line per setting as it is timed."""
    import torch

    from . import Context

    grid = DEFAULT_GRID if grid is None else grid
    if cache:
        hit = lookup(d, cache)
        if hit is not None:
            return hit
    dev = torch.device("cuda", device)
    pos = torch.from_numpy(d["pos"]).to(dev)
    h0 = torch.from_numpy(d["h0"]).to(dev)
    mass = torch.from_numpy(d["mass"]).to(dev)
    vel = torch.from_numpy(d["vel"]).to(dev)
    u = torch.from_numpy(d["u"]).to(dev)
    n = pos.shape[0]
    h = h0.clone()
    rho, f = torch.empty_like(h), torch.empty_like(h)
    acc, dudt = torch.empty((n, 3), dtype=torch.float32, device=dev), torch.empty_like(h)
    table = []
    stream = torch.cuda.current_stream(dev)
    for params in grid:
        ctx = Context(device, **params)
        try:
            ctx.build_cells(pos, h0, d["box_first"], d["box_len"])
            times = []
            for r in range(reps + 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                h.copy_(h0)
                e0.record(stream)
                st = ctx.pass_(mass, h, vel, u, rho=rho, f=f, acc=acc, dudt=dudt)["stats"]
                e1.record(stream)
                torch.cuda.synchronize()
                if r > 0:  # the first pass warms up (and captures the launch sequence)
                    times.append(e0.elapsed_time(e1))
            table.append({"params": params, "ms": float(np.median(times)), "rebuilds": st["rebuilds"],
                          "cells": st["n_cells"]})
        except RuntimeError as e:  # e.g. a margin too large for a small box
            table.append({"params": params, "ms": None, "error": str(e)})
        finally:
            ctx.close()
        if progress:
            print("tune %d/%d %s ms %s" % (len(table), len(grid), json.dumps(params, sort_keys=True),
                                           table[-1]["ms"]), flush=True)
    ok = [t for t in table if t["ms"] is not None]
    if not ok:
        raise RuntimeError("no cell setting ran: %s" % table)
    # settings within 1% of the fastest are equal within the timing noise;
    # among them prefer the XCD-local cell orders, whose neighbour re-reads
    # stay in each XCD's L2 (far less traffic beyond it), then the fastest
    fastest = min(t["ms"] for t in ok)
    near = [t for t in ok if t["ms"] <= 1.01 * fastest]
    order_rank = {2: 0, 1: 1, 0: 2}
    best = min(near, key=lambda t: (order_rank.get(t["params"].get("cell_order", 0), 3), t["ms"]))
    out = {"best": best["params"], "best_ms": best["ms"], "table": table}
    if cache:
        save(d, out, cache)
    return out


def _main() -> int:
    import argparse
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads

    ap = argparse.ArgumentParser(description="tune the cell parameters for a synthetic workload")
    ap.add_argument("--workload", default="sedov")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    d = workloads.make(args.workload)
    res = autotune(d, 0, progress=True)
    save(d, res, args.out)
    print(json.dumps({"workload": args.workload, "best": res["best"], "best_ms": res["best_ms"]}))
    return 0


if __name__ == "__main__":
    raise SystemExit(_main())
