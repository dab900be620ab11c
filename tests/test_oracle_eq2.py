"""Pins of the oracle's second force form, the paper's illustrative pressure
sum (its Eq. 2): a hand-computed pair, its independence from the grad-h
factor, its agreement with the grad-h form where every h is equal and
f = 1, and a lattice at rest under uniform pressure feeling no force."""

import math

import numpy as np
import pytest

import oracle
import workloads

GAMMA = oracle.GAMMA


def test_pair_closed_form():
    # i at x = 0.40, j at x = 0.43 (r = 0.03), h_i = 0.1 (q = 0.3), h_j = 0.05
    # (q = 0.6); both at rest, so no viscosity; a third particle far away.
    pos = np.array([[0.40, 0.5, 0.5], [0.43, 0.5, 0.5], [0.90, 0.1, 0.1]])
    vel = np.zeros((3, 3))
    mass = np.array([1.0, 2.0, 1.0])
    u = np.array([2.0, 0.5, 1.0])
    h = np.array([0.1, 0.05, 0.01])
    rho = np.array([1.5, 2.0, 1.0])
    f = np.array([0.7, 1.3, 1.0])
    fo = oracle.force(pos, vel, mass, u, h, rho, f, form=1)
    Pi_, Pj = (GAMMA - 1) * 1.5 * 2.0, (GAMMA - 1) * 2.0 * 0.5
    dwi = -12 * 0.3 + 18 * 0.09                      # w'(0.3) = -1.98
    Di = 8.0 / (math.pi * 0.1 ** 4) * dwi
    dwj = -6 * (1 - 0.6) ** 2                         # w'(0.6) = -0.96, j's own kernel
    G_i = (Pi_ / 1.5 ** 2 + Pj / 2.0 ** 2) * Di       # on i: both terms with h_i; rhat = -x
    assert fo["acc"][0, 0] == pytest.approx(-2.0 * G_i * -1.0, rel=1e-13)
    assert abs(fo["acc"][0, 1]) < 1e-12 and abs(fo["acc"][0, 2]) < 1e-12
    # on j the kernel is j's: q = 0.6 with h_j = 0.05
    Dj = 8.0 / (math.pi * 0.05 ** 4) * dwj
    G_j = (Pj / 2.0 ** 2 + Pi_ / 1.5 ** 2) * Dj
    assert fo["acc"][1, 0] == pytest.approx(-1.0 * G_j * 1.0, rel=1e-13)
    assert np.all(fo["dudt"][:2] == 0.0)
    # f plays no part in this form, but does in the grad-h one
    fo2 = oracle.force(pos, vel, mass, u, h, rho, np.ones(3), form=1)
    assert np.array_equal(fo["acc"], fo2["acc"])
    g0 = oracle.force(pos, vel, mass, u, h, rho, f)
    g1 = oracle.force(pos, vel, mass, u, h, rho, np.ones(3))
    assert not np.allclose(g0["acc"][:2], g1["acc"][:2])


def test_equal_h_and_unit_f_reduce_to_the_grad_h_form():
    d = workloads.lattice_box(8, [1508, 970], jitter=0.0, u=1.0, vel_sigma=0.4)
    pos = np.asarray(d["pos"], dtype=np.float64)
    n = pos.shape[0]
    mass = np.asarray(d["mass"], dtype=np.float64)
    de = oracle.density(pos, mass)
    assert np.ptp(de["h"]) < 1e-12 * de["h"].mean()
    rng = np.random.default_rng([1508, 971])
    u = rng.uniform(0.5, 2.0, n)
    rho = rng.uniform(0.8, 1.2, n)
    args = (pos, d["vel"], mass, u, de["h"], rho, np.ones(n))
    a0 = oracle.force(*args)
    a1 = oracle.force(*args, form=1)
    assert np.allclose(a1["acc"], a0["acc"], rtol=0, atol=1e-12 * a0["scale_a"].max())
    assert np.allclose(a1["dudt"], a0["dudt"], rtol=0, atol=1e-12 * a0["scale_u"].max())
    # with varied h the two forms differ
    h2 = de["h"] * rng.uniform(0.9, 1.1, n)
    b0 = oracle.force(pos, d["vel"], mass, u, h2, rho, np.ones(n))
    b1 = oracle.force(pos, d["vel"], mass, u, h2, rho, np.ones(n), form=1)
    assert np.max(np.linalg.norm(b1["acc"] - b0["acc"], axis=1) / b0["scale_a"]) > 1e-3


def test_lattice_at_rest_feels_no_force():
    d = workloads.lattice_box(10, [1508, 972], jitter=0.0, u=1.0)
    r = oracle.run(d, form=1)
    assert np.max(np.linalg.norm(r["acc"], axis=1) / r["scale_a"]) < 1e-12
    assert np.all(np.abs(r["dudt"]) <= 1e-12 * r["scale_u"] + 1e-300)
