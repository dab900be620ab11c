"""FP64 CPU oracle for the SPH density and force sums (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package. The GPU library never does, and this
package never imports the GPU library: the two share nothing but the seeded
input arrays.

``sph_oracle.c`` holds the grid-searched FP64 implementation (built with gcc
and OpenMP on first use); ``brute.py`` holds an O(N^2) numpy version for tiny
inputs. Both follow the same definitions: section 2 of the Swift paper (Eq. 1
and the text that follows Eq. 2) with the grad-h Gadget-2 force in the
internal-energy variable (see the header of ``sph_oracle.c``).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "libsph_oracle.so")

GAMMA = 5.0 / 3.0
ALPHA = 0.8
N_NGB = 48.0

_ERR = {1: "bad argument", 2: "out of memory", 3: "smoothing length reaches L/2",
        4: "root finder did not converge",
        5: "a neighbour inside the target's h has no smoothing length (sample not closed)"}

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle (gcc -O2 -fopenmp, strict IEEE FP64)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.orc_density.argtypes = [I64, P, P, D, D, I64, P, P, P, P, P, P, P, ctypes.c_int, P]
        lib.orc_density.restype = ctypes.c_int
        lib.orc_force.argtypes = [I64, P, P, P, P, P, P, P, D, D, D, I64, P,
                                  P, P, P, P, P, P, P, P, P, ctypes.c_int, ctypes.c_int, P]
        lib.orc_force.restype = ctypes.c_int
        lib.orc_divcurl.argtypes = [I64, P, P, P, P, P, D, I64, P, P, P, P, ctypes.c_int, P]
        lib.orc_divcurl.restype = ctypes.c_int
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def max_threads() -> int:
    return int(_load().orc_max_threads())


def density(pos, mass, L: float = 1.0, n_ngb: float = N_NGB, targets=None, h_start=None,
            threads: int = 0) -> dict:
    """h, rho, f (grad-h factor), weighted count nw and integer neighbour
    count of the targets (every particle when ``targets`` is None). Entries of
    particles that are not targets are NaN (or -1 for counts)."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    n = pos.shape[0]
    mass = _f64(mass)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    hs = None if h_start is None else _f64(h_start)
    out = {k: np.full(n, np.nan) for k in ("h", "rho", "f", "nw")}
    out["nngb"] = np.full(n, -1, dtype=np.int64)
    bad = ctypes.c_int64(-1)
    rc = lib.orc_density(n, _ptr(pos), _ptr(mass), float(L), float(n_ngb),
                         0 if tg is None else tg.size, _ptr(tg), _ptr(hs),
                         _ptr(out["h"]), _ptr(out["rho"]), _ptr(out["f"]), _ptr(out["nw"]),
                         _ptr(out["nngb"]), int(threads), ctypes.byref(bad))
    if rc:
        raise RuntimeError("oracle density: %s (particle %d)" % (_ERR.get(rc, rc), bad.value))
    return out


def force(pos, vel, mass, u, h, rho, f, L: float = 1.0, gamma: float = GAMMA,
          alpha: float = ALPHA, targets=None, threads: int = 0, balsara=None, form: int = 0) -> dict:
    """Acceleration, du/dt, their gross scales (sum of |pair term|), their
    kernel scales (pair terms at full kernel slope), the ordered pair count
    #{j != i: 0 < r < max(h_i, h_j)} and the signal velocity
    max(c_i, max_j (c_i + c_j - 3 min(v_ij . rhat, 0))) of the targets (all
    when None). ``balsara``: per-particle Balsara factors that scale the
    viscosity of each pair by their mean (None: no switch). ``form`` 1: the
    paper's Eq. 2 pressure sum in place of the grad-h terms (f unused)."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    n = pos.shape[0]
    vel = _f64(vel, (-1, 3))
    arrs = [_f64(a) for a in (mass, u, h, rho, f)]
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    acc = np.full((n, 3), np.nan)
    out = {k: np.full(n, np.nan) for k in ("dudt", "gross_a", "gross_u", "scale_a", "scale_u", "vsig")}
    npair = np.full(n, -1, dtype=np.int64)
    bad = ctypes.c_int64(-1)
    rc = lib.orc_force(n, _ptr(pos), _ptr(vel), *[_ptr(a) for a in arrs], float(L), float(gamma),
                       float(alpha), 0 if tg is None else tg.size, _ptr(tg), _ptr(acc),
                       _ptr(out["dudt"]), _ptr(out["gross_a"]), _ptr(out["gross_u"]),
                       _ptr(out["scale_a"]), _ptr(out["scale_u"]), _ptr(npair), _ptr(out["vsig"]),
                       _ptr(None if balsara is None else _f64(balsara)), int(form), int(threads),
                       ctypes.byref(bad))
    if rc:
        raise RuntimeError("oracle force: %s (particle %d)" % (_ERR.get(rc, rc), bad.value))
    out["acc"] = acc
    out["npair"] = npair
    return out


def divcurl(pos, vel, mass, h, rho, L: float = 1.0, targets=None, threads: int = 0) -> dict:
    """Velocity divergence ``div``, curl ``curl`` (n, 3) and their error scale
    ``scale`` (sum of m_j |v_ij| / rho_i times the kernel's largest slope) of
    the targets (all when None), as in the Balsara paragraph of the header of
    ``sph_oracle.c``."""
    lib = _load()
    pos = _f64(pos, (-1, 3))
    n = pos.shape[0]
    vel = _f64(vel, (-1, 3))
    mass, h, rho = _f64(mass), _f64(h), _f64(rho)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    out = {"div": np.full(n, np.nan), "curl": np.full((n, 3), np.nan), "scale": np.full(n, np.nan)}
    bad = ctypes.c_int64(-1)
    rc = lib.orc_divcurl(n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(h), _ptr(rho), float(L),
                         0 if tg is None else tg.size, _ptr(tg), _ptr(out["div"]), _ptr(out["curl"]),
                         _ptr(out["scale"]), int(threads), ctypes.byref(bad))
    if rc:
        raise RuntimeError("oracle divcurl: %s (particle %d)" % (_ERR.get(rc, rc), bad.value))
    return out


def balsara_factor(div, curl, u, h, gamma: float = GAMMA):
    """B = |div v| / (|div v| + |curl v| + 1e-4 c / h), c the sound speed of
    the ideal gas at u (the Gadget-2 form of the Balsara switch); 0 where the
    denominator is 0 (no motion and no sound speed: nothing to damp)."""
    a = np.abs(np.asarray(div, dtype=np.float64))
    w = np.linalg.norm(np.asarray(curl, dtype=np.float64).reshape(-1, 3), axis=1)
    c = np.sqrt(gamma * (gamma - 1.0) * np.asarray(u, dtype=np.float64))
    den = a + w + 1e-4 * c / np.asarray(h, dtype=np.float64)
    return np.where(den > 0, a / np.where(den > 0, den, 1.0), 0.0)


def run_box(pos, vel, mass, u, L: float = 1.0, n_ngb: float = N_NGB, gamma: float = GAMMA,
            alpha: float = ALPHA, h_start=None, threads: int = 0, balsara: bool = False,
            form: int = 0) -> dict:
    """Density then force for every particle of one periodic box, with the
    conservation sums of the box and the wall time of the two phases. With
    ``balsara`` the force applies the Balsara switch; the factors are
    returned as ``balsara``, div v and curl v as ``div`` and ``curl`` (their
    error scale as ``scale_dc``)."""
    t0 = time.perf_counter()
    d = density(pos, mass, L, n_ngb, h_start=h_start, threads=threads)
    t1 = time.perf_counter()
    B = None
    if balsara:
        dc = divcurl(pos, vel, mass, d["h"], d["rho"], L, threads=threads)
        B = balsara_factor(dc["div"], dc["curl"], u, d["h"], gamma)
        d.update(div=dc["div"], curl=dc["curl"], scale_dc=dc["scale"], balsara=B)
    fo = force(pos, vel, mass, u, d["h"], d["rho"], d["f"], L, gamma, alpha, threads=threads, balsara=B,
               form=form)
    t2 = time.perf_counter()
    d.update(fo)
    d.update(conservation(mass, vel, fo["acc"], fo["dudt"]))
    d["t_density"] = t1 - t0
    d["t_force"] = t2 - t1
    return d


def conservation(mass, vel, acc, dudt) -> dict:
    """Total momentum rate sum m a and energy rate sum m (v.a + du/dt), in
    FP64, with the gross scales they are judged against."""
    m = np.asarray(mass, dtype=np.float64)
    v = np.asarray(vel, dtype=np.float64).reshape(-1, 3)
    a = np.asarray(acc, dtype=np.float64).reshape(-1, 3)
    du = np.asarray(dudt, dtype=np.float64)
    va = np.einsum("ij,ij->i", v, a)
    return {
        "mom": (m[:, None] * a).sum(axis=0),
        "mom_scale": float((m[:, None] * np.abs(a)).sum()),
        "energy": float((m * (va + du)).sum()),
        "energy_scale": float((m * (np.abs(va) + np.abs(du))).sum()),
    }


def run(d: dict, n_ngb: float = N_NGB, gamma: float = GAMMA, alpha: float = ALPHA,
        threads: int = 0, balsara: bool = False, form: int = 0) -> dict:
    """Oracle over every box of a workload dict (see the ``workloads``
    package); per-particle outputs are concatenated in input order."""
    keys = ("h", "rho", "f", "nw", "nngb", "acc", "dudt", "gross_a", "gross_u", "scale_a", "scale_u",
            "npair", "vsig") + (("div", "curl", "scale_dc", "balsara") if balsara else ())
    parts = {k: [] for k in keys}
    cons = []
    t_d = t_f = 0.0
    nb = len(d["box_len"])
    for b in range(nb):
        s, e = int(d["box_first"][b]), int(d["box_first"][b + 1])
        if e == s:
            for k in keys:
                parts[k].append(np.zeros((0, 3) if k in ("acc", "curl") else (0,),
                                         dtype=np.int64 if k in ("nngb", "npair") else np.float64))
            cons.append((np.zeros(3), 0.0, 0.0, 0.0))
            continue
        r = run_box(d["pos"][s:e], d["vel"][s:e], d["mass"][s:e], d["u"][s:e],
                    float(d["box_len"][b]), n_ngb, gamma, alpha, h_start=d["h0"][s:e],
                    threads=threads, balsara=balsara, form=form)
        for k in keys:
            parts[k].append(r[k])
        cons.append((r["mom"], r["energy"], r["mom_scale"], r["energy_scale"]))
        t_d += r["t_density"]
        t_f += r["t_force"]
    out = {k: np.concatenate(v, axis=0) for k, v in parts.items()}
    out["cons"] = cons
    out["t_density"] = t_d
    out["t_force"] = t_f
    return out
