"""FP64 kick-drift-kick leapfrog and Courant time step (test infrastructure).

Only the test suite may import this module; it never imports the GPU
library. It follows section 2 of the Swift paper (particles are marched
forward in time, positions with their velocities and velocities with their
accelerations) with the readings the paper leaves open, taken from the
Gadget-2 scheme whose force the paper says Swift uses:

  kick       v <- v + a dt/2,  u <- u + du/dt dt/2
  drift      x <- x + v dt (wrapped into the periodic box)
  predict    the force at the end of the step sees v + a dt/2 and
             u + du/dt dt/2 (the state at the drift's end time, extrapolated
             with the old rates: the viscosity and the pressure need both)
  kick       v <- v + a_new dt/2,  u <- u + du/dt_new dt/2
  time step  dt = C min_i h_i / v_sig,i  (Courant condition on the signal
             velocity the force loop reports)

Every quantity is FP64 here; the inputs may be FP32 arrays.
"""

from __future__ import annotations

import numpy as np

from . import ALPHA, GAMMA, N_NGB, run


def timestep(h, vsig, courant: float) -> float:
    """Courant step courant * min(h / v_sig) over the particles with v_sig > 0
    (inf when there is none)."""
    h = np.asarray(h, dtype=np.float64)
    v = np.asarray(vsig, dtype=np.float64)
    ok = v > 0
    if not ok.any():
        return float("inf")
    return float(courant * np.min(h[ok] / v[ok]))


def kick(vel, u, acc, dudt, dt: float):
    """Velocities and internal energies after a kick of length dt."""
    v = np.asarray(vel, dtype=np.float64).reshape(-1, 3) + np.asarray(acc, dtype=np.float64).reshape(-1, 3) * dt
    uu = np.asarray(u, dtype=np.float64) + np.asarray(dudt, dtype=np.float64) * dt
    return v, uu


def drift(pos, vel, dt: float, L: float):
    """Positions after a drift of length dt, wrapped into [0, L)."""
    x = np.asarray(pos, dtype=np.float64).reshape(-1, 3) + np.asarray(vel, dtype=np.float64).reshape(-1, 3) * dt
    x = x - L * np.floor(x / L)
    x[x < 0.0] += L  # x / L rounded up to an integer
    x[x >= L] = 0.0  # rounded up to L
    return x


def kdk_step(d: dict, acc, dudt, dt: float, h_start=None, n_ngb: float = N_NGB, gamma: float = GAMMA,
             alpha: float = ALPHA) -> dict:
    """One step of length dt from the state of workload dict d (positions,
    velocities, masses, u; one or more boxes) with the rates acc, dudt at its
    start. Returns the new state (pos, vel, u), the rates at the end of the
    step (acc, dudt), the density outputs and signal velocities there, and
    the predicted v and u the force saw."""
    v_half, u_half = kick(d["vel"], d["u"], acc, dudt, 0.5 * dt)
    pos1 = np.empty_like(np.asarray(d["pos"], dtype=np.float64))
    for b in range(len(d["box_len"])):
        s, e = int(d["box_first"][b]), int(d["box_first"][b + 1])
        pos1[s:e] = drift(d["pos"][s:e], v_half[s:e], dt, float(d["box_len"][b]))
    v_pred, u_pred = kick(v_half, u_half, acc, dudt, 0.5 * dt)
    d1 = dict(d)
    d1["pos"] = pos1
    d1["vel"] = v_pred
    d1["u"] = u_pred
    d1["h0"] = d["h0"] if h_start is None else h_start
    r = run(d1, n_ngb, gamma, alpha)
    v1, u1 = kick(v_half, u_half, r["acc"], r["dudt"], 0.5 * dt)
    return {"pos": pos1, "vel": v1, "u": u1, "acc": r["acc"], "dudt": r["dudt"], "h": r["h"],
            "rho": r["rho"], "f": r["f"], "vsig": r["vsig"], "scale_a": r["scale_a"],
            "scale_u": r["scale_u"], "v_pred": v_pred, "u_pred": u_pred}


def energy(mass, vel, u) -> float:
    """Total energy sum m (|v|^2 / 2 + u), FP64."""
    m = np.asarray(mass, dtype=np.float64)
    v = np.asarray(vel, dtype=np.float64).reshape(-1, 3)
    return float((m * (0.5 * (v * v).sum(axis=1) + np.asarray(u, dtype=np.float64))).sum())
