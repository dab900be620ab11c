"""O(N^2) numpy FP64 version of the oracle's definitions, for tiny inputs.

Test infrastructure only. It checks the grid-searched C oracle against an
independent code path: dense minimum-image distance matrices instead of the
bucket search, and plain bisection on every particle at once instead of the
per-particle bracketed Newton iteration. The formulas are those of section 2
of the Swift paper (Eq. 1 and the Gadget-2 grad-h force it cites), stated in
the header of ``sph_oracle.c``.
"""

from __future__ import annotations

import math

import numpy as np


def _w(q):
    q = np.asarray(q, dtype=np.float64)
    inner = 1.0 - 6.0 * q ** 2 + 6.0 * q ** 3
    outer = 2.0 * (1.0 - q) ** 3
    return np.where(q < 0.5, inner, np.where(q < 1.0, outer, 0.0))


def _dw(q):
    q = np.asarray(q, dtype=np.float64)
    inner = -12.0 * q + 18.0 * q ** 2
    outer = -6.0 * (1.0 - q) ** 2
    return np.where(q < 0.5, inner, np.where(q < 1.0, outer, 0.0))


def separations(pos, L=1.0):
    """Minimum-image r_i - r_j for every ordered pair, shape (N, N, 3)."""
    pos = np.asarray(pos, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.rint(d / L)
    return d


def density(pos, mass, L=1.0, n_ngb=48.0, iters=64, keep=256):
    """Bisection on every particle at once over its ``keep`` nearest
    distances (all N^2 distances are formed; the truncation is checked to
    hold every particle inside the root)."""
    d = separations(pos, L)
    r_all = np.sqrt((d ** 2).sum(axis=-1))
    m_all = np.asarray(mass, dtype=np.float64)
    n = r_all.shape[0]
    k = min(keep, n)
    part = np.argpartition(r_all, k - 1, axis=1)[:, :k]
    r = np.take_along_axis(r_all, part, axis=1)
    m = m_all[part]
    target = 3.0 * n_ngb / 32.0
    lo = np.zeros(n)
    hi = np.full(n, 0.5 * L)
    if np.any(_w(r / hi[:, None]).sum(axis=1) < target):
        raise ValueError("root beyond L/2")
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        s0 = _w(r / mid[:, None]).sum(axis=1)
        below = s0 < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    h = 0.5 * (lo + hi)
    if k < n:
        assert np.all(r.max(axis=1) > h), "truncated list does not cover h"
    q = r / h[:, None]
    w = _w(q)
    dw = _dw(q)
    M0 = (w * m).sum(axis=1)
    M1 = (q * dw * m).sum(axis=1)
    S0 = w.sum(axis=1)
    off = ~np.eye(n, dtype=bool)
    return {
        "h": h,
        "rho": 8.0 / (math.pi * h ** 3) * M0,
        "f": -3.0 * M0 / M1,
        "nw": 32.0 / 3.0 * S0,
        "nngb": ((r_all < h[:, None]) & off).sum(axis=1),
    }


def force(pos, vel, mass, u, h, rho, f, L=1.0, gamma=5.0 / 3.0, alpha=0.8):
    d = separations(pos, L)
    r = np.sqrt((d ** 2).sum(axis=-1))
    n = r.shape[0]
    m = np.asarray(mass, dtype=np.float64)
    v = np.asarray(vel, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    P = (gamma - 1.0) * rho * np.asarray(u, dtype=np.float64)
    c = np.sqrt(gamma * (gamma - 1.0) * np.asarray(u, dtype=np.float64))
    Phi = f * P / rho ** 2
    off = ~np.eye(n, dtype=bool)
    inside = off & ((r < h[:, None]) | (r < h[None, :])) & (r > 0)
    rs = np.where(inside, r, 1.0)
    e = d / rs[..., None]
    Di = 8.0 / (math.pi * h[:, None] ** 4) * _dw(r / h[:, None])
    Dj = 8.0 / (math.pi * h[None, :] ** 4) * _dw(r / h[None, :])
    vij = v[:, None, :] - v[None, :, :]
    vr = (vij * e).sum(axis=-1)
    wv = np.minimum(vr, 0.0)
    Pv = -alpha * (c[:, None] + c[None, :] - 3.0 * wv) * wv / (rho[:, None] + rho[None, :])
    Dbar = 0.5 * (Di + Dj)
    G = Phi[:, None] * Di + Phi[None, :] * Dj + Pv * Dbar
    G = np.where(inside, G, 0.0)
    acc = -(m[None, :, None] * G[..., None] * e).sum(axis=1)
    term = np.where(inside, m[None, :] * (Phi[:, None] * Di + 0.5 * Pv * Dbar) * vr, 0.0)
    # the kernel's steepest slope, max |w'(q)| = |w'(1/3)| = 2, inside each h
    # (found here by sampling w' densely, not assumed)
    qs = np.linspace(0.0, 1.0, 30001)
    slope_max = float(np.max(np.abs(_dw(qs))))
    Dmi = np.where(r < h[:, None], slope_max * 8.0 / (math.pi * h[:, None] ** 4), 0.0)
    Dmj = np.where(r < h[None, :], slope_max * 8.0 / (math.pi * h[None, :] ** 4), 0.0)
    sa = m[None, :] * (np.abs(Phi)[:, None] * Dmi + np.abs(Phi)[None, :] * Dmj + np.abs(Pv) * 0.5 * (Dmi + Dmj))
    su = m[None, :] * (np.abs(Phi)[:, None] * Dmi + 0.25 * np.abs(Pv) * (Dmi + Dmj)) * np.abs(vr)
    return {
        "acc": acc,
        "dudt": term.sum(axis=1),
        "gross_a": np.abs(m[None, :] * G).sum(axis=1),
        "gross_u": np.abs(term).sum(axis=1),
        "scale_a": np.where(inside, sa, 0.0).sum(axis=1),
        "scale_u": np.where(inside, su, 0.0).sum(axis=1),
        "npair": inside.sum(axis=1),
    }


def divcurl(pos, vel, mass, h, rho, L=1.0):
    """Velocity divergence and curl of every particle over its neighbours
    0 < r < h_i, and their error scale sum_j m_j |v_ij| max|D_i| / rho_i."""
    d = separations(pos, L)
    r = np.sqrt((d ** 2).sum(axis=-1))
    n = r.shape[0]
    m = np.asarray(mass, dtype=np.float64)
    v = np.asarray(vel, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    off = ~np.eye(n, dtype=bool)
    inside = off & (r < h[:, None]) & (r > 0)
    rs = np.where(inside, r, 1.0)
    e = d / rs[..., None]
    Di = np.where(inside, 8.0 / (math.pi * h[:, None] ** 4) * _dw(r / h[:, None]), 0.0)
    vij = v[:, None, :] - v[None, :, :]
    mD = m[None, :] * Di
    div = -(mD * (vij * e).sum(axis=-1)).sum(axis=1) / rho
    curl = (mD[..., None] * np.cross(vij, e)).sum(axis=1) / rho[:, None]
    qs = np.linspace(0.0, 1.0, 30001)
    slope_max = float(np.max(np.abs(_dw(qs))))
    Dm = slope_max * 8.0 / (math.pi * h ** 4)
    scale = (np.where(inside, m[None, :] * np.linalg.norm(vij, axis=-1), 0.0).sum(axis=1) * Dm / rho)
    return {"div": div, "curl": curl, "scale": scale}
