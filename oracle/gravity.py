"""FP64 near-field gravity (particle-particle), test infrastructure.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the GPU library never does.

The paper's gravity (section 2, Eq. 3) is the direct sum of Newton's
attraction over the other particles; its tree code (section 3.2) evaluates
the pairs of nearby cells directly (P2P) and the far ones through multipole
expansions. This module computes the near part alone, with the reading used
throughout this repository: for particles in a periodic box of side L,

    g_i = -G sum_{j != i} m_j  r_ij (|r_ij|^2 + eps^2)^(-3/2)  S(|r_ij| / r_cut),

r_ij the minimum image of x_i - x_j, eps the Plummer softening, and the
window S(x) = (1 - x^2)^2 for x < 1, 0 beyond. S is 1 at r = 0 and falls to
zero with zero slope at the cutoff, so the sum is continuous in the
positions (the part 1 - S would come from the multipoles, not computed
here). Pairs at r = 0 add nothing (no direction).

Two code paths, sharing no arithmetic: ``p2p`` finds the pairs with scipy's
cKDTree and adds every pair to both of its particles; ``p2p_dense`` takes
dense minimum-image separation matrices and sums each row on its own
(``p2p_rows``: the same for chosen rows only, for sampled checks of sets too
large for the tree path).
"""

from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def window(x):
    """S(x) = (1 - x^2)^2 for 0 <= x < 1, else 0."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x < 1.0, (1.0 - x * x) ** 2, 0.0)


def pair_force(r, m_j, G, eps, r_cut):
    """Magnitude of the pull on i towards j per unit of r_ij: the factor F
    with g_i = -F r_ij, F = G m_j (r^2 + eps^2)^(-3/2) S(r / r_cut)."""
    r = np.asarray(r, dtype=np.float64)
    return G * m_j * (r * r + eps * eps) ** -1.5 * window(r / r_cut)


def p2p(pos, mass, G: float, eps: float, r_cut: float, L: float = 1.0) -> dict:
    """Near-field acceleration of every particle (module docstring), with
    the gross scale G sum_j m_j |r_ij| (r^2 + eps^2)^(-3/2) S (the sum of
    the magnitudes of the terms) and the number of ordered pairs with
    0 < r_ij < r_cut."""
    pos = np.mod(np.asarray(pos, dtype=np.float64), L)
    mass = np.asarray(mass, dtype=np.float64)
    n = pos.shape[0]
    if not (0.0 < r_cut < 0.5 * L):
        raise ValueError("r_cut must lie in (0, L/2)")
    tree = cKDTree(pos, boxsize=L)
    pairs = tree.query_pairs(r_cut, output_type="ndarray")
    acc = np.zeros((n, 3))
    gross = np.zeros(n)
    npair = 0
    if len(pairs):
        i, j = pairs[:, 0], pairs[:, 1]
        d = pos[i] - pos[j]
        d -= L * np.rint(d / L)
        r = np.sqrt(np.sum(d * d, axis=1))
        keep = (r > 0.0) & (r < r_cut)
        i, j, d, r = i[keep], j[keep], d[keep], r[keep]
        fi = pair_force(r, mass[j], G, eps, r_cut)  # pull on i
        fj = pair_force(r, mass[i], G, eps, r_cut)  # pull on j
        np.add.at(acc, i, -fi[:, None] * d)
        np.add.at(acc, j, fj[:, None] * d)
        np.add.at(gross, i, fi * r)
        np.add.at(gross, j, fj * r)
        npair = 2 * len(i)
    return {"acc": acc, "gross": gross, "npair": npair}


def p2p_dense(pos, mass, G: float, eps: float, r_cut: float, L: float = 1.0) -> np.ndarray:
    """The same acceleration from dense N x N separation matrices, each
    particle's row summed on its own (tiny inputs)."""
    pos = np.mod(np.asarray(pos, dtype=np.float64), L)
    mass = np.asarray(mass, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.rint(d / L)
    r = np.sqrt(np.sum(d * d, axis=2))
    inside = (r > 0.0) & (r < r_cut)
    x = np.where(inside, r / r_cut, 1.0)
    f = np.where(inside, G * mass[None, :] * (1.0 - x * x) ** 2 / (r * r + eps * eps) ** 1.5, 0.0)
    return -np.einsum("ij,ijk->ik", f, d)


def p2p_rows(pos, mass, G: float, eps: float, r_cut: float, rows, L: float = 1.0) -> dict:
    """Acceleration, gross scale and pair count of the particles ``rows``
    only, each row summed over every particle of the set (dense, one row
    block at a time)."""
    pos = np.mod(np.asarray(pos, dtype=np.float64), L)
    mass = np.asarray(mass, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    if not (0.0 < r_cut < 0.5 * L):
        raise ValueError("r_cut must lie in (0, L/2)")
    acc = np.zeros((len(rows), 3))
    gross = np.zeros(len(rows))
    npair = np.zeros(len(rows), dtype=np.int64)
    for a in range(0, len(rows), 64):
        rb = rows[a:a + 64]
        d = pos[rb][:, None, :] - pos[None, :, :]
        d -= L * np.rint(d / L)
        r = np.sqrt(np.sum(d * d, axis=2))
        inside = (r > 0.0) & (r < r_cut)
        f = np.where(inside, pair_force(np.where(inside, r, 0.0), mass[None, :], G, eps, r_cut), 0.0)
        acc[a:a + 64] = -np.sum(f[:, :, None] * d, axis=1)
        gross[a:a + 64] = np.sum(f * r, axis=1)
        npair[a:a + 64] = np.sum(inside, axis=1)
    return {"acc": acc, "gross": gross, "npair": npair}
