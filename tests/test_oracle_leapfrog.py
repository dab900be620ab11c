"""Pins of the oracle's signal velocity and kick-drift-kick step against facts
it does not compute itself: closed-form signal velocities of hand-placed
pairs, the symmetries of a lattice (at rest it stays at rest; moving
uniformly it translates exactly), the second-order convergence of the
leapfrog (a slip in the predicted state or in a kick makes it first order)
and conservation of the total energy."""

import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import leapfrog

GAMMA = oracle.GAMMA


def _sound(u):
    return math.sqrt(GAMMA * (GAMMA - 1.0) * u)


@pytest.mark.parametrize("v0", [0.7, -0.7, 0.0])
def test_signal_velocity_of_a_pair(v0):
    # i at x = 0.4, j at x = 0.45 (r = 0.05 < h); i moves with v0 along +x
    # (towards j when v0 > 0); a third particle k sits far from both with a
    # small h. v_ij . rhat = -v0, so w = min(-v0, 0).
    pos = np.array([[0.40, 0.5, 0.5], [0.45, 0.5, 0.5], [0.90, 0.1, 0.1]])
    vel = np.array([[v0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.3, -0.2, 0.1]])
    mass = np.ones(3)
    u = np.array([2.0, 0.5, 1.3])
    h = np.array([0.1, 0.1, 0.01])
    rho = np.ones(3)
    f = np.ones(3)
    fo = oracle.force(pos, vel, mass, u, h, rho, f)
    w = min(-v0, 0.0)
    ci, cj, ck = _sound(2.0), _sound(0.5), _sound(1.3)
    expect_ij = ci + cj - 3.0 * w
    assert abs(fo["vsig"][0] - max(ci, expect_ij)) < 1e-13
    assert abs(fo["vsig"][1] - max(cj, expect_ij)) < 1e-13
    assert fo["vsig"][2] == pytest.approx(ck, abs=1e-15)


def test_timestep_is_courant_over_signal_speed():
    h = np.array([0.1, 0.02, 0.05])
    vs = np.array([1.0, 4.0, 0.0])  # the last one has no signal speed
    assert leapfrog.timestep(h, vs, 0.3) == pytest.approx(0.3 * 0.005, rel=1e-15)
    assert leapfrog.timestep(h, np.zeros(3), 0.3) == float("inf")


def _lattice(n_side, vel=(0.0, 0.0, 0.0)):
    d = workloads.lattice_box(n_side, [1508, 950], jitter=0.0, u=1.0)
    d["vel"] = np.tile(np.asarray(vel, dtype=np.float32), (d["pos"].shape[0], 1))
    return d


def test_lattice_at_rest_stays_at_rest():
    d = _lattice(10)
    r0 = oracle.run(d)
    s = leapfrog.kdk_step(d, r0["acc"], r0["dudt"], 1e-3)
    assert np.max(np.abs(r0["acc"])) < 1e-9
    dx = s["pos"] - d["pos"]
    dx -= np.round(dx)
    assert np.max(np.abs(dx)) < 1e-15
    assert np.max(np.abs(s["vel"])) < 1e-11
    assert np.max(np.abs(s["u"] - d["u"])) < 1e-12


def test_uniform_motion_translates_the_lattice():
    d = _lattice(10, (0.3, -0.2, 0.45))
    v0 = d["vel"][0].astype(np.float64)  # the velocities are stored in FP32
    r0 = oracle.run(d)
    dt = 2e-3
    s = leapfrog.kdk_step(d, r0["acc"], r0["dudt"], dt)
    # no relative motion: no pressure gradient, no viscosity, no heating
    dx = s["pos"] - (d["pos"] + v0 * dt)
    dx -= np.round(dx)
    assert np.max(np.abs(dx)) < 1e-13
    assert np.max(np.abs(s["vel"] - v0)) < 1e-10
    assert np.max(np.abs(s["u"] - 1.0)) < 1e-10


def _smooth_flow(n_side=12):
    # jittered lattice, a smooth velocity field with compression (so du/dt
    # is not small) and a smooth pressure bump: pressure forces and heating
    # without shocks
    d = workloads.lattice_box(n_side, [1508, 951], jitter=0.1, u=1.0)
    x = d["pos"]
    v = np.stack([0.2 * np.sin(2 * np.pi * x[:, 0]) + 0.1 * np.sin(2 * np.pi * x[:, 1]),
                  0.2 * np.sin(2 * np.pi * x[:, 2]), 0.2 * np.sin(2 * np.pi * x[:, 0])], axis=1)
    d["vel"] = v.astype(np.float32)
    d["u"] = (1.0 + 0.3 * np.cos(2 * np.pi * x[:, 0])).astype(np.float32)
    return d


def _run(d, dt, steps, alpha):
    s = dict(d)
    r = oracle.run(s, alpha=alpha)
    acc, dudt, h = r["acc"], r["dudt"], r["h"]
    for _ in range(steps):
        st = leapfrog.kdk_step(s, acc, dudt, dt, h_start=h, alpha=alpha)
        s = dict(s)
        s["pos"], s["vel"], s["u"] = st["pos"], st["vel"], st["u"]
        acc, dudt, h = st["acc"], st["dudt"], st["h"]
    return s


def test_leapfrog_is_second_order():
    d = _smooth_flow()
    r = oracle.run(d, alpha=0.0)
    T = 4 * leapfrog.timestep(r["h"], r["vsig"], 0.2)
    runs = [_run(d, T / k, k, 0.0) for k in (2, 4, 8)]

    def diff(a, b):
        dx = a["pos"] - b["pos"]
        dx -= np.round(dx)
        return max(np.max(np.abs(dx)), T * np.max(np.abs(a["vel"] - b["vel"])), T * np.max(np.abs(a["u"] - b["u"])))

    e1, e2 = diff(runs[0], runs[1]), diff(runs[1], runs[2])
    # halving dt shrinks the change by 4 for a second-order scheme, 2 for a first-order one
    assert 3.0 < e1 / e2 < 5.5, (e1, e2)


def test_energy_error_is_second_order_and_small():
    # the pairwise force conserves sum m (|v|^2/2 + u) exactly in continuous
    # time; the leapfrog loses a part that is second order in dt. A wrong sign
    # or rate in a kick of u or v instead leaves an error of the order of the
    # kinetic-thermal exchange itself, or one that halves with dt.
    d = _smooth_flow(10)
    e0 = leapfrog.energy(d["mass"], d["vel"], d["u"])
    kin0 = 0.5 * float((d["mass"][:, None] * d["vel"].astype(np.float64) ** 2).sum())
    r = oracle.run(d)
    dt = leapfrog.timestep(r["h"], r["vsig"], 0.2)
    err, exch = [], []
    for k in (1, 2):
        s = _run(d, dt / k, 6 * k, oracle.ALPHA)
        err.append(leapfrog.energy(s["mass"], s["vel"], s["u"]) - e0)
        exch.append(0.5 * float((s["mass"][:, None] * np.asarray(s["vel"]) ** 2).sum()) - kin0)
    assert abs(err[0]) < 0.02 * abs(exch[0]), (err, exch)
    assert abs(err[0] / err[1]) > 3.0, err


def test_drift_wraps_into_the_box():
    # crossings of both faces, several box lengths, and values within rounding
    # of a multiple of L all land in [0, L) at the periodic image of x + v dt
    L = 0.8
    x = np.array([[0.79, 0.01, 0.4], [0.0, 0.7999999999999999, 0.4], [0.3, 0.3, 0.3]])
    v = np.array([[1.0, -1.0, 0.0], [-1e-17, 1e-16, 0.0], [25.0, -33.0, 8.0]])
    dt = 0.05
    y = leapfrog.drift(x, v, dt, L)
    assert np.all(y >= 0.0) and np.all(y < L)
    d = (y - (x + v * dt)) / L
    assert np.max(np.abs(d - np.round(d))) < 1e-12
