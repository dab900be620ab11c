"""Shared helpers of the GPU parity tests: error measures against the oracle,
with the tolerances of the FP32 and FP64 forms."""

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


def oracle_sample(d: dict, targets, radius: float, box: int = 0) -> dict:
    """Oracle values at `targets` of one box: h, rho, f of the targets and of
    every particle within `radius` of them (so the force of each target sees
    every neighbour's h), then the force of the targets. Arrays are full
    length with NaN away from the sample."""
    s, e = int(d["box_first"][box]), int(d["box_first"][box + 1])
    pos = d["pos"][s:e]
    L = float(d["box_len"][box])
    tree = cKDTree(np.mod(pos, L), boxsize=L)
    near = tree.query_ball_point(np.mod(pos[targets], L), radius)
    need = np.unique(np.concatenate([np.asarray(targets)] + [np.asarray(x, dtype=np.int64) for x in near]))
    r = oracle.density(pos, d["mass"][s:e], L, targets=need, h_start=d["h0"][s:e])
    fo = oracle.force(pos, d["vel"][s:e], d["mass"][s:e], d["u"][s:e], r["h"], r["rho"], r["f"], L,
                      targets=np.asarray(targets, dtype=np.int64))
    r.update(fo)
    return r


def oracle_sample_exact(d: dict, targets, h_near, box: int = 0) -> dict:
    """Like oracle_sample, but the sample is every particle j that pairs with a
    target i (r_ij < max(h_i, h_j), with 2% slack), found from the smoothing
    lengths h_near (any close estimate, e.g. the GPU's; they only choose the
    sample, the oracle solves its own h). Suits sets whose h spans decades,
    where one radius would either miss neighbours or take most of the box."""
    s, e = int(d["box_first"][box]), int(d["box_first"][box + 1])
    L = float(d["box_len"][box])
    pos = np.mod(d["pos"][s:e], L)
    hn = np.asarray(h_near[s:e], dtype=np.float64) * 1.02
    targets = np.asarray(targets, dtype=np.int64)
    # j within its own h of some target (scipy takes one radius per query point)
    hits = cKDTree(pos[targets], boxsize=L).query_ball_point(pos, hn, return_length=True)
    # j within the target's h
    near = cKDTree(pos, boxsize=L).query_ball_point(pos[targets], hn[targets])
    need = np.unique(np.concatenate([targets, np.nonzero(hits)[0]] + [np.asarray(x, dtype=np.int64) for x in near]))
    r = oracle.density(pos, d["mass"][s:e], L, targets=need, h_start=d["h0"][s:e])
    fo = oracle.force(pos, d["vel"][s:e], d["mass"][s:e], d["u"][s:e], r["h"], r["rho"], r["f"], L,
                      targets=targets)
    r.update(fo)
    r["n_sample"] = len(need)
    return r
