"""Pins of the FP64 near-field gravity oracle (oracle/gravity.py), on the CPU.

The definition (section 2 Eq. 3 of the Swift paper, restricted to pairs
closer than r_cut, softened, with the window S(x) = (1 - x^2)^2) is pinned by
what it must satisfy rather than by retyping it:
- the force is the gradient of a pair potential computed by numerical
  quadrature of the radial profile (a wrong power, a dropped window or a
  sign error fails it);
- close pairs follow the inverse-square law;
- the dense row sums conserve momentum and agree with the tree-searched
  pair sums, across the periodic boundary;
- a particle of a perfect lattice feels no pull;
- the window's closed-form values.
"""

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.spatial import cKDTree

from oracle import gravity as og


def test_window_values():
    assert og.window(0.0) == 1.0
    assert og.window(0.5) == pytest.approx(0.5625, abs=1e-15)
    assert og.window(1.0) == 0.0 and og.window(1.5) == 0.0
    # zero slope at the cutoff: the sum is continuous in the positions
    eps = 1e-6
    assert abs((og.window(1.0) - og.window(1.0 - eps)) / eps) < 1e-5


def test_inverse_square_for_close_pairs():
    """Unsoftened, far inside the cutoff: |g| r^2 / (G m) = S(r / r_cut) -> 1."""
    G, m, rc = 1.5, 3.0, 0.2
    for r in (1e-3, 2e-3, 4e-3):
        pos = np.array([[0.5, 0.5, 0.5], [0.5 + r, 0.5, 0.5]])
        g = og.p2p(pos, np.array([2.0, m]), G, 0.0, rc)["acc"]
        assert g[0, 0] > 0 and g[1, 0] < 0  # each pulled towards the other
        assert g[0, 0] * r * r / (G * m) == pytest.approx(1.0 - 2 * (r / rc) ** 2, rel=1e-6)


def _potential(pos, mass, G, eps, rc, L=1.0):
    """U = -G sum_{i<j} m_i m_j phi(r_ij), phi(r) = integral from r to r_cut of
    s (s^2 + eps^2)^(-3/2) S(s / r_cut) ds, by adaptive quadrature."""
    def prof(s):
        return s * (s * s + eps * eps) ** -1.5 * float(og.window(s / rc))
    U = 0.0
    n = len(mass)
    for i in range(n):
        for j in range(i + 1, n):
            d = pos[i] - pos[j]
            d -= L * np.rint(d / L)
            r = float(np.sqrt(d @ d))
            if r < rc:
                phi, _ = quad(prof, r, rc, epsabs=1e-14, epsrel=1e-12, limit=200)
                U -= G * mass[i] * mass[j] * phi
    return U


def test_force_is_minus_gradient_of_the_pair_potential():
    rng = np.random.default_rng([1508, 71])
    n = 10
    pos = 0.5 + 0.05 * rng.standard_normal((n, 3))
    mass = rng.uniform(0.5, 2.0, n)
    G, eps, rc = 1.3, 0.01, 0.12
    g = og.p2p(pos, mass, G, eps, rc)["acc"]
    step = 1e-6
    for i in (0, 3, 7):
        for a in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, a] += step
            p2[i, a] -= step
            dU = (_potential(p1, mass, G, eps, rc) - _potential(p2, mass, G, eps, rc)) / (2 * step)
            assert mass[i] * g[i, a] == pytest.approx(-dU, rel=1e-6, abs=1e-8 * np.abs(mass[i] * g[i]).max())


@pytest.mark.parametrize("seed", [72, 73, 74])
def test_dense_rows_match_tree_pairs_and_conserve_momentum(seed):
    rng = np.random.default_rng([1508, seed])
    n = 300
    pos = rng.random((n, 3))
    pos[:40] = np.mod(0.02 * rng.standard_normal((40, 3)), 1.0)  # a clump across the periodic corner
    mass = rng.uniform(0.5, 2.0, n)
    G, eps, rc = 1.0, 0.003, 0.15
    t = og.p2p(pos, mass, G, eps, rc)
    dn = og.p2p_dense(pos, mass, G, eps, rc)
    scale = t["gross"].max()
    np.testing.assert_allclose(dn, t["acc"], rtol=0, atol=1e-12 * scale)
    mom = np.sum(mass[:, None] * dn, axis=0)
    assert np.all(np.abs(mom) <= 1e-13 * np.sum(mass * t["gross"]))
    assert t["npair"] % 2 == 0 and t["npair"] > 0
    # gross scale: at least the magnitude of the sum
    assert np.all(np.linalg.norm(t["acc"], axis=1) <= t["gross"] * (1 + 1e-12))


def test_rows_match_tree_pairs():
    """The row-sampled form against the tree pairs, rows spread over the set
    (a clump across the periodic corner included)."""
    rng = np.random.default_rng([1508, 75])
    n = 400
    pos = rng.random((n, 3))
    pos[:50] = np.mod(0.03 * rng.standard_normal((50, 3)), 1.0)
    mass = rng.uniform(0.5, 2.0, n)
    G, eps, rc = 0.7, 0.002, 0.12
    t = og.p2p(pos, mass, G, eps, rc)
    rows = np.concatenate([np.arange(0, 50, 7), rng.choice(n, 70, replace=False)])
    w = og.p2p_rows(pos, mass, G, eps, rc, rows)
    np.testing.assert_allclose(w["acc"], t["acc"][rows], rtol=0, atol=1e-12 * t["gross"].max())
    np.testing.assert_allclose(w["gross"], t["gross"][rows], rtol=1e-12)
    # pairs of each row from a periodic ball query (itself excluded; no two
    # particles coincide and none sits at r_cut)
    tree = cKDTree(pos, boxsize=1.0)
    ball = tree.query_ball_point(pos[rows], rc, return_length=True) - 1
    assert np.array_equal(w["npair"], ball)


def test_lattice_feels_no_pull():
    m = 8
    g1 = (np.arange(m) + 0.5) / m
    pos = np.stack(np.meshgrid(g1, g1, g1, indexing="ij"), axis=-1).reshape(-1, 3)
    mass = np.full(len(pos), 1.0 / len(pos))
    t = og.p2p(pos, mass, 1.0, 0.01, 0.3)
    assert np.abs(t["acc"]).max() <= 1e-12 * t["gross"].max()


def test_cutoff_beyond_half_box_is_refused():
    with pytest.raises(ValueError):
        og.p2p(np.zeros((2, 3)), np.ones(2), 1.0, 0.0, 0.5)
