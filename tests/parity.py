"""Shared helpers of the GPU parity tests: error measures against the oracle,
with the tolerances of the FP32 and FP64 forms."""

import math

import numpy as np
from scipy.spatial import cKDTree

import oracle

# FP32 path: h, rho, f and the weighted count to 1e-5 relative; acceleration
# and du/dt to 1e-4 of the kernel-scale magnitude of particle i: the sum of its
# pair terms with w'(q) replaced by the kernel's largest slope (2). The plain
# gross sum sum_j |m_j G_ij| is ill-conditioned as a scale: where one pair at
# the edge of a kernel dominates it, w'(q) ~ (1 - q)^2 turns a relative error
# of 1e-7 in h (below FP32 resolution) into 4e-4 of that sum on the Sedov set,
# while the kernel-scale error stays at 0.6 times the h error. The gross
# measure is still reported and held at its 99.9th percentile.
TOL32 = {"h": 1e-5, "rho": 1e-5, "f": 1e-5, "nw": 1e-5, "acc": 1e-4, "dudt": 1e-4,
         "acc_gross_p999": 1e-4, "dudt_gross_p999": 1e-4}
TOL64 = {k: 1e-10 for k in TOL32}


def _ratio(num, den):
    """num / den, with 0 where both vanish and inf where only den does."""
    den = np.asarray(den, dtype=np.float64)
    safe = np.where(den > 0, den, 1.0)
    return np.where(den > 0, num / safe, np.where(num > 0, np.inf, 0.0))


def errors(g: dict, r: dict, idx=None) -> dict:
    """Max errors of GPU outputs g against oracle outputs r over idx."""
    if idx is None:
        idx = np.arange(len(r["h"]))
    e = {}
    for k in ("h", "rho", "f", "nw"):
        e[k] = float(np.max(np.abs(g[k][idx] - r[k][idx]) / np.abs(r[k][idx])))
    da = np.linalg.norm(g["acc"][idx] - r["acc"][idx], axis=1)
    du = np.abs(g["dudt"][idx] - r["dudt"][idx])
    e["acc"] = float(np.max(_ratio(da, r["scale_a"][idx])))
    e["dudt"] = float(np.max(_ratio(du, r["scale_u"][idx])))
    e["acc_gross_p999"] = float(np.percentile(_ratio(da, r["gross_a"][idx]), 99.9))
    e["dudt_gross_p999"] = float(np.percentile(_ratio(du, r["gross_u"][idx]), 99.9))
    e["acc_gross_max"] = float(np.max(_ratio(da, r["gross_a"][idx])))
    return e


def assert_within(e: dict, tol: dict, label: str = ""):
    bad = {k: (e[k], tol[k]) for k in tol if not (e[k] <= tol[k])}
    assert not bad, "%s exceeds tolerance: %s" % (label, bad)


def h_upper_bound(pos, L: float, n_ngb: float = 48.0, chunk: int = 1 << 20):
    """An upper bound on every particle's smoothing length from the positions
    alone. w(q) >= w(1/2) = 1/4 for q <= 1/2, so K other particles within a
    radius rho give S0(2 rho) >= 1 + K/4; with K = ceil((3 n_ngb / 32 - 1) * 4)
    (14 for 48 neighbours) that reaches the target, and since S0 grows with h
    the root h_i is at most twice the distance to i's K-th nearest neighbour
    (scipy's cKDTree, periodic)."""
    K = int(math.ceil((3.0 * n_ngb / 32.0 - 1.0) * 4.0 - 1e-9))
    tree = cKDTree(pos, boxsize=L)
    out = np.empty(pos.shape[0])
    for a in range(0, pos.shape[0], chunk):
        dk, _ = tree.query(pos[a:a + chunk], k=K + 1, workers=-1)  # K + 1: the particle itself included
        out[a:a + chunk] = 2.0 * dk[:, K]
    return out * (1.0 + 1e-9), tree


# bounds of the positions already seen (a 2^24-particle set takes tens of
# seconds), keyed by the position array, which the entry keeps alive
_BOUNDS = {}


def oracle_sample_exact(d: dict, targets, box: int = 0) -> dict:
    """Oracle values at `targets` of one box, solving h only where needed:
    the targets, and every particle that can pair with one. Nothing here
    comes from the GPU. A partner j of target i has r_ij < max(h_i, h_j):
    either it lies inside the target's oracle h_i, or inside its own h_j,
    which h_upper_bound caps from the positions alone; the sample takes
    every particle within its bound of some target. The oracle force then
    refuses (rather than skips) any neighbour inside h_i left unsolved.
    Suits sets whose h spans decades, where one radius would either miss
    neighbours or take most of the box."""
    s, e = int(d["box_first"][box]), int(d["box_first"][box + 1])
    L = float(d["box_len"][box])
    pos = np.mod(d["pos"][s:e], L)
    mass = d["mass"][s:e]
    targets = np.asarray(targets, dtype=np.int64)
    key = (id(d["pos"]), box)
    if key not in _BOUNDS or _BOUNDS[key][0] is not d["pos"]:
        _BOUNDS[key] = (d["pos"],) + h_upper_bound(pos, L)
    _, hb, tree = _BOUNDS[key]
    rt = oracle.density(pos, mass, L, targets=targets, h_start=d["h0"][s:e])
    # j within the target's own h
    near = tree.query_ball_point(pos[targets], rt["h"][targets] * (1.0 + 1e-9))
    # j whose bound on h_j reaches some target (scipy takes one radius per query point)
    hits = cKDTree(pos[targets], boxsize=L).query_ball_point(pos, hb, return_length=True)
    need = np.unique(np.concatenate([targets, np.nonzero(hits)[0]] + [np.asarray(x, dtype=np.int64) for x in near]))
    r = oracle.density(pos, mass, L, targets=need, h_start=d["h0"][s:e])
    fo = oracle.force(pos, d["vel"][s:e], mass, d["u"][s:e], r["h"], r["rho"], r["f"], L,
                      targets=targets)
    r.update(fo)
    r["n_sample"] = len(need)
    return r
