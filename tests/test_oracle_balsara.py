"""Pins of the oracle's velocity divergence and curl and of its Balsara
switch against facts it does not compute itself. On a cubic lattice the
neighbour set of a particle has cubic symmetry, so the second moment
sum_j g(r) rhat rhat^T is a multiple of the identity; for a linear velocity
field v = A x the SPH estimates are then exactly div = kappa tr(A) and
curl = kappa (the curl of A x), with one lattice constant kappa (close to 1,
its continuum value). Hence: an expansion has no curl, a rotation no
divergence, a shear both in the ratio the calculus gives, and the expansion
and the rotation measure the same kappa. The switch scales each pair's
viscosity by the mean of the two factors: on a hand-placed pair the
viscous part of the force scales by exactly that mean."""

import numpy as np
import pytest

import oracle
import workloads

N_SIDE = 16


def _interior_field(A):
    d = workloads.lattice_box(N_SIDE, [1508, 951], jitter=0.0, u=1.0)
    pos = np.asarray(d["pos"], dtype=np.float64)
    mass = np.asarray(d["mass"], dtype=np.float64)
    de = oracle.density(pos, mass)
    c = np.full(3, 0.5)
    vel = (pos - c) @ np.asarray(A, dtype=np.float64).T
    # particles whose whole h-sphere lies inside the box see the linear field
    # without the jump at the periodic wrap
    inner = np.all(np.abs(pos - c) < 0.5 - 1.01 * de["h"][:, None], axis=1)
    assert inner.sum() >= 100
    dc = oracle.divcurl(pos, vel, mass, de["h"], de["rho"])
    return dc, inner, de


def test_expansion_has_divergence_and_no_curl():
    a = 0.7
    dc, inner, _ = _interior_field(a * np.eye(3))
    g = dc["scale"][inner]
    kappa = dc["div"][inner] / (3 * a)
    assert np.all(np.abs(np.linalg.norm(dc["curl"][inner], axis=1)) < 1e-12 * g)
    assert np.ptp(kappa) < 1e-12
    assert 0.9 < kappa[0] < 1.1
    # a compression has the opposite sign
    dc2, _, _ = _interior_field(-a * np.eye(3))
    assert np.allclose(dc2["div"][inner], -dc["div"][inner], rtol=1e-13, atol=0)


def test_rotation_has_curl_along_its_axis_and_no_divergence():
    om = np.array([0.3, -0.5, 0.2])
    A = np.array([[0, -om[2], om[1]], [om[2], 0, -om[0]], [-om[1], om[0], 0]])  # A x = om x x
    dc, inner, _ = _interior_field(A)
    g = dc["scale"][inner]
    assert np.all(np.abs(dc["div"][inner]) < 1e-12 * g)
    dce, _, _ = _interior_field(np.eye(3))
    kappa = dce["div"][inner][0] / 3.0
    # curl (om x x) = 2 om, measured with the same lattice constant
    assert np.allclose(dc["curl"][inner], 2 * kappa * om[None, :], rtol=1e-12, atol=1e-12 * g.max())


def test_shear_splits_into_its_divergence_and_curl():
    s = 0.4
    A = np.zeros((3, 3))
    A[0, 1] = s  # v = (s y, 0, 0): div 0, curl (0, 0, -s)
    dc, inner, _ = _interior_field(A)
    dce, _, _ = _interior_field(np.eye(3))
    kappa = dce["div"][inner][0] / 3.0
    g = dc["scale"][inner]
    assert np.all(np.abs(dc["div"][inner]) < 1e-12 * g)
    assert np.allclose(dc["curl"][inner], kappa * np.array([0.0, 0.0, -s])[None, :], rtol=1e-12,
                       atol=1e-12 * g.max())


def test_uniform_motion_changes_nothing():
    d = workloads.lattice_box(10, [1508, 952], jitter=0.2, u=1.0, vel_sigma=0.5)
    pos = np.asarray(d["pos"], dtype=np.float64)
    vel = np.asarray(d["vel"], dtype=np.float64)
    mass = np.asarray(d["mass"], dtype=np.float64)
    de = oracle.density(pos, mass)
    a = oracle.divcurl(pos, vel, mass, de["h"], de["rho"])
    b = oracle.divcurl(pos, vel + np.array([3.0, -1.0, 2.0]), mass, de["h"], de["rho"])
    c = oracle.divcurl(pos, -vel, mass, de["h"], de["rho"])
    assert np.max(np.abs(a["div"] - b["div"]) / a["scale"]) < 1e-11
    assert np.max(np.abs(a["curl"] - b["curl"]) / a["scale"][:, None]) < 1e-11
    assert np.allclose(c["div"], -a["div"], rtol=0, atol=0)
    assert np.allclose(c["curl"], -a["curl"], rtol=0, atol=0)
    # random motion has both, and the factor lies in [0, 1]
    B = oracle.balsara_factor(a["div"], a["curl"], d["u"], de["h"])
    assert np.all((B >= 0) & (B <= 1)) and 0.2 < B.mean() < 0.8


def test_factor_of_pure_compression_and_pure_rotation():
    h = np.array([0.1])
    u = np.array([1.0])
    c = np.sqrt(oracle.GAMMA * (oracle.GAMMA - 1.0))
    assert oracle.balsara_factor([-2.0], [[0, 0, 0]], u, h)[0] == pytest.approx(2.0 / (2.0 + 1e-4 * c / 0.1), rel=1e-15)
    assert oracle.balsara_factor([0.0], [[0, 3.0, 0]], u, h)[0] == 0.0
    assert oracle.balsara_factor([1.0], [[0, 0, -1.0]], u, h)[0] == pytest.approx(1.0 / (2.0 + 1e-4 * c / 0.1), rel=1e-15)
    assert oracle.balsara_factor([0.0], [[0, 0, 0]], [0.0], h)[0] == 0.0  # at rest and cold


@pytest.mark.parametrize("b", [(0.0, 0.0), (1.0, 1.0), (0.25, 0.9), (1.0, 0.0)])
def test_switch_scales_the_viscosity_of_a_pair_by_the_mean_factor(b):
    # i approaches j (w < 0), so the pair has viscosity; a third particle is far
    pos = np.array([[0.40, 0.5, 0.5], [0.45, 0.51, 0.5], [0.90, 0.1, 0.1]])
    vel = np.array([[0.8, 0.1, 0.0], [-0.2, 0.0, 0.3], [0.0, 0.0, 0.0]])
    mass = np.array([1.0, 1.5, 1.0])
    u = np.array([2.0, 0.5, 1.3])
    h = np.array([0.1, 0.08, 0.01])
    rho = np.array([1.0, 1.3, 1.0])
    f = np.array([0.9, 1.1, 1.0])
    full = oracle.force(pos, vel, mass, u, h, rho, f)
    none = oracle.force(pos, vel, mass, u, h, rho, f, alpha=0.0)
    sw = oracle.force(pos, vel, mass, u, h, rho, f, balsara=np.array([b[0], b[1], 0.5]))
    mean = 0.5 * (b[0] + b[1])
    visc = full["acc"][:2] - none["acc"][:2]
    assert np.abs(visc).max() > 1e-3 * np.abs(none["acc"][:2]).max()
    assert np.allclose(sw["acc"][:2] - none["acc"][:2], mean * visc, rtol=1e-12, atol=1e-14)
    assert np.allclose(sw["dudt"][:2] - none["dudt"][:2], mean * (full["dudt"][:2] - none["dudt"][:2]),
                       rtol=1e-12, atol=1e-14)


def test_divergence_is_the_density_rate_of_the_flow():
    # at fixed h_i, d rho_i / dt = sum_j m_j grad_i W_ij(h_i) . (v_i - v_j)
    # = -rho_i div v_i: a central difference of the O(N^2) density sum (the
    # brute-force module, no shared code) along the flow pins the divergence
    # sum, its sign and its use of h_i, on a jittered set with mixed h
    from oracle import brute
    d = workloads.lattice_box(6, [1508, 953], jitter=0.35, u=1.0, vel_sigma=0.5)
    pos = np.asarray(d["pos"], dtype=np.float64)
    vel = np.asarray(d["vel"], dtype=np.float64)
    mass = np.asarray(d["mass"], dtype=np.float64)
    de = oracle.density(pos, mass)
    h = de["h"]
    assert np.ptp(h) > 0.05 * h.mean()

    def rho_at(x):
        r = np.linalg.norm(brute.separations(x % 1.0), axis=2)
        return (mass[None, :] * 8.0 / (np.pi * h[:, None] ** 3) * brute._w(r / h[:, None])).sum(axis=1)

    eps = 1e-6
    rate = (rho_at(pos + eps * vel) - rho_at(pos - eps * vel)) / (2 * eps)
    dc = oracle.divcurl(pos, vel, mass, h, de["rho"])
    assert np.allclose(-rate / de["rho"], dc["div"], rtol=0, atol=1e-7 * dc["scale"].max())
