"""Seeded synthetic particle sets shaped like the paper's SPH workloads.

This module only draws inputs. It holds none of the SPH arithmetic (no
kernel, no density, no force): both the FP64 oracle and the GPU library
consume its arrays unchanged, so neither side can bias the other.

Every generator returns a dict of numpy arrays:

    pos        (N, 3) float64   positions, wrapped into [0, L) of their box
    vel        (N, 3) float32   velocities
    mass       (N,)   float32   particle masses (1 / N_box: mean density 1)
    u          (N,)   float32   specific internal energy
    h0         (N,)   float32   initial smoothing-length guess
    box_first  (B+1,) int64     particle range [box_first[b], box_first[b+1]) of box b
    box_len    (B,)   float64   side length of periodic box b

Velocities, masses, u and h0 are rounded to float32 before they are
returned, so an FP64 consumer and an FP32 consumer see identical values.
Positions stay float64.

The paper measures on snapshots of a cosmological volume (51M and 10M
particles) that are not available; the clustered and log-normal sets stand
in for their clustered structure and wide range of smoothing lengths.

Random streams: ``numpy.random.default_rng([1508, k])`` for set k, and
``[1508, 3, b]`` for box b of the batched set.
"""

from __future__ import annotations

import math

import numpy as np

N_NGB = 48.0  # target weighted neighbour number of every set


def _mean_density_h(mass: float, rho: np.ndarray | float) -> np.ndarray:
    """Initial guess for h from a density estimate: the radius of a sphere
    holding N_NGB particles of mass ``mass`` at density ``rho``. Only a
    starting point; the converged h does not depend on it."""
    return np.cbrt(3.0 * N_NGB * mass / (4.0 * math.pi * np.asarray(rho, dtype=np.float64)))


def _pack(pos, vel, mass, u, h0, box_first, box_len) -> dict:
    return {
        "pos": np.ascontiguousarray(pos, dtype=np.float64),
        "vel": np.ascontiguousarray(vel, dtype=np.float32),
        "mass": np.ascontiguousarray(mass, dtype=np.float32),
        "u": np.ascontiguousarray(u, dtype=np.float32),
        "h0": np.ascontiguousarray(h0, dtype=np.float32),
        "box_first": np.ascontiguousarray(box_first, dtype=np.int64),
        "box_len": np.ascontiguousarray(box_len, dtype=np.float64),
    }


def jittered_lattice(n_side: int, rng: np.random.Generator | None, jitter: float = 0.1,
                     L: float = 1.0) -> np.ndarray:
    """n_side^3 points at (i + 1/2) a, a = L / n_side, each coordinate moved by
    U(-jitter a, +jitter a) (no move when ``rng`` is None), wrapped into [0, L)."""
    a = L / n_side
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * a
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    if rng is not None and jitter > 0.0:
        pos = pos + rng.uniform(-jitter * a, jitter * a, size=pos.shape)
    return np.mod(pos, L)


def lattice_box(n_side: int, seed, jitter: float = 0.1, u: float = 1.0,
                vel_sigma: float = 0.0) -> dict:
    """One periodic unit box holding a (jittered) cubic lattice of equal masses."""
    rng = np.random.default_rng(seed)
    n = n_side ** 3
    pos = jittered_lattice(n_side, rng if jitter > 0 else None, jitter)
    m = 1.0 / n
    if vel_sigma > 0.0:
        vel = rng.normal(0.0, vel_sigma, size=(n, 3))
    else:
        vel = np.zeros((n, 3))
    h0 = np.full(n, _mean_density_h(m, 1.0))
    return _pack(pos, vel, np.full(n, m), np.full(n, u), h0,
                 [0, n], [1.0])


def small(n_side: int = 16) -> dict:
    """16^3 jittered lattice, u = 1, v = 0 (the small FP64 case)."""
    return lattice_box(n_side, [1508, 0], jitter=0.1, u=1.0)


def sedov(n_side: int = 64, n_hot: int = 32) -> dict:
    """Sedov-like blast: jittered lattice, u = 1e-5 except total energy 1
    deposited in the ``n_hot`` particles nearest the box centre (their u is
    replaced by 1 / (n_hot m)); ties are broken by particle index."""
    d = lattice_box(n_side, [1508, 1], jitter=0.1, u=1e-5)
    n = n_side ** 3
    m = 1.0 / n
    dx = d["pos"] - 0.5
    r2 = np.einsum("ij,ij->i", dx, dx)
    hot = np.lexsort((np.arange(n), r2))[:n_hot]
    u = d["u"].astype(np.float64)
    u[hot] = 1.0 / (n_hot * m)
    d["u"] = u.astype(np.float32)
    return d


def _plummer_radii(rng, a: float, count: int, r_max: float) -> np.ndarray:
    """Radii of a Plummer sphere of scale radius ``a`` by inverting its
    cumulative mass profile, redrawing any radius beyond ``r_max``."""
    out = np.empty(count)
    todo = np.arange(count)
    while todo.size:
        x = rng.uniform(0.0, 1.0, size=todo.size)
        x = np.clip(x, 1e-300, 1.0)
        r = a / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
        ok = r <= r_max
        out[todo[ok]] = r[ok]
        todo = todo[~ok]
    return out


def _isotropic(rng, count: int) -> np.ndarray:
    v = rng.normal(size=(count, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def clustered(n_uniform: int = 1 << 19, n_spheres: int = 64, per_sphere: int = 8192,
              a_range=(0.005, 0.05)) -> dict:
    """Half uniform random, half drawn from Plummer spheres with random centres
    and log-uniform scale radii, in a periodic unit box; u = 1, v = 0.

    h0 comes from the density of the generating mixture at each particle (the
    uniform background plus every sphere's Plummer profile), so the guess
    follows the clustering; the converged h does not depend on it."""
    rng = np.random.default_rng([1508, 2])
    n = n_uniform + n_spheres * per_sphere
    m = 1.0 / n
    parts = [rng.uniform(0.0, 1.0, size=(n_uniform, 3))]
    centres = rng.uniform(0.0, 1.0, size=(n_spheres, 3))
    scales = np.exp(rng.uniform(math.log(a_range[0]), math.log(a_range[1]), size=n_spheres))
    for k in range(n_spheres):
        r = _plummer_radii(rng, scales[k], per_sphere, 0.5)
        parts.append(centres[k] + r[:, None] * _isotropic(rng, per_sphere))
    pos = np.mod(np.concatenate(parts, axis=0), 1.0)
    # generating density (mass per unit volume) for the h guess
    rho = np.full(n, n_uniform * m)
    for k in range(n_spheres):
        d = pos - centres[k]
        d -= np.rint(d)
        r2 = np.einsum("ij,ij->i", d, d)
        mk = per_sphere * m
        a2 = scales[k] ** 2
        rho += mk * 3.0 / (4.0 * math.pi * scales[k] ** 3) * (1.0 + r2 / a2) ** -2.5
    h0 = _mean_density_h(m, rho)
    return _pack(pos, np.zeros((n, 3)), np.full(n, m), np.ones(n), h0, [0, n], [1.0])


def batched(n_boxes: int = 256, n_min: int = 8192, n_max: int = 65536,
            side_min: int = 20, side_max: int = 40, vel_sigma: float = 0.1) -> dict:
    """Independent periodic unit boxes, each a jittered lattice of n_b^3
    particles with n_b = clamp(round(N_b^(1/3))) for N_b log-uniform in
    [n_min, n_max]; Gaussian velocities (sigma per component); u = 1."""
    rng = np.random.default_rng([1508, 3])
    nb = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_boxes))
    sides = np.clip(np.rint(np.cbrt(nb)).astype(np.int64), side_min, side_max)
    boxes = [lattice_box(int(s), [1508, 3, b], jitter=0.1, u=1.0, vel_sigma=vel_sigma)
             for b, s in enumerate(sides)]
    counts = np.array([bx["pos"].shape[0] for bx in boxes], dtype=np.int64)
    first = np.concatenate([[0], np.cumsum(counts)])
    cat = lambda k: np.concatenate([bx[k] for bx in boxes], axis=0)
    return _pack(cat("pos"), cat("vel"), cat("mass"), cat("u"), cat("h0"),
                 first, np.ones(n_boxes))


def lognormal(n_mesh: int = 256, n_part: int | None = None, sigma_ln: float = 1.5,
              vel_rms: float = 0.1, slope: float = -2.0) -> dict:
    """Particles sampled from a log-normal density field in a periodic unit box.

    A white-noise field on an n_mesh^3 grid is filtered to power spectrum
    P(k) ~ k^slope (the k = 0 mode removed), scaled to standard deviation
    ``sigma_ln`` and exponentiated; particle counts per mesh cell are a
    multinomial draw of n_part over the normalised cell densities and
    positions are uniform inside each cell. Velocities follow the linear
    displacement field of the same Gaussian field, normalised to ``vel_rms``
    per component and assigned from each particle's cell; u = 1. h0 comes
    from the cell density."""
    rng = np.random.default_rng([1508, 4])
    if n_part is None:
        n_part = n_mesh ** 3
    noise = rng.normal(size=(n_mesh,) * 3)
    dk = np.fft.rfftn(noise)
    kx = np.fft.fftfreq(n_mesh) * n_mesh
    kz = np.fft.rfftfreq(n_mesh) * n_mesh
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    k2[0, 0, 0] = 1.0
    dk *= k2 ** (slope / 4.0)
    dk[0, 0, 0] = 0.0
    delta = np.fft.irfftn(dk, s=(n_mesh,) * 3)
    delta *= sigma_ln / delta.std()
    rho_c = np.exp(delta)
    rho_c /= rho_c.mean()
    p = (rho_c / rho_c.sum()).ravel()
    counts = rng.multinomial(n_part, p)
    cell = np.repeat(np.arange(p.size, dtype=np.int64), counts)
    ci = np.stack(np.unravel_index(cell, (n_mesh,) * 3), axis=1).astype(np.float64)
    pos = (ci + rng.uniform(0.0, 1.0, size=(n_part, 3))) / n_mesh
    vel = np.empty((n_part, 3))
    kvec = (kx[:, None, None], kx[None, :, None], kz[None, None, :])
    for ax in range(3):
        vk = 1j * kvec[ax] * dk / k2
        vk[0, 0, 0] = 0.0
        vfield = np.fft.irfftn(vk, s=(n_mesh,) * 3)
        vfield *= vel_rms / vfield.std()
        vel[:, ax] = vfield.ravel()[cell]
    m = 1.0 / n_part
    h0 = _mean_density_h(m, rho_c.ravel()[cell])
    pos = np.mod(pos, 1.0)
    return _pack(pos, vel, np.full(n_part, m), np.ones(n_part), h0, [0, n_part], [1.0])


CONFIGS = {
    "small": small,
    "sedov": sedov,
    "clustered": clustered,
    "batched": batched,
    "large": lognormal,
}


def make(name: str, **kw) -> dict:
    """Build one of the named workloads (optionally resized through ``kw``)."""
    return CONFIGS[name](**kw)


def box_slice(d: dict, b: int) -> dict:
    """The arrays of box ``b`` of a multi-box set, as a one-box set."""
    s, e = int(d["box_first"][b]), int(d["box_first"][b + 1])
    out = {k: d[k][s:e] for k in ("pos", "vel", "mass", "u", "h0")}
    out["box_first"] = np.array([0, e - s], dtype=np.int64)
    out["box_len"] = d["box_len"][b:b + 1].copy()
    return out
