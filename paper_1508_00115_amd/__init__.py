"""Python binding of the MI355X SPH neighbour-interaction library.

The functions mirror the C ABI of ``include/sph.h`` one to one (same names,
same arguments); ``Context`` wraps them for torch tensors. Everything here is
argument marshalling: every step of the computation runs in the HIP kernels
of ``libsph.so``. Importing the package does not load the library; the first
call does, and fails loudly if the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsph.so")

SPH_OK = 0
SPH_E_ARG = 1
SPH_E_HIP = 2
SPH_E_NOMEM = 3
SPH_E_H_TOO_LARGE = 4
SPH_E_NOT_CONVERGED = 5
SPH_E_STATE = 6

EXPORTS = ("sph_create", "sph_destroy", "sph_build_cells", "sph_density", "sph_force",
           "sph_density_f64", "sph_force_f64", "sph_get_timings", "sph_status_string",
           "sph_last_error", "sph_version", "sph_struct_size", "sph_pass", "sph_get_build_info",
           "sph_kick", "sph_drift", "sph_timestep", "sph_get_balsara", "sph_timestep_noalloc",
           "sph_predict_h", "sph_gravity_p2p")


class sph_params(ctypes.Structure):
    _fields_ = [("n_ngb", ctypes.c_double), ("gamma", ctypes.c_double),
                ("alpha_visc", ctypes.c_double), ("n_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("h_margin", ctypes.c_double),
                ("cell_ratio", ctypes.c_double), ("leaf_target", ctypes.c_int32),
                ("workspace_limit", ctypes.c_int64), ("timing", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("queue_batch", ctypes.c_int32),
                ("tile_cap", ctypes.c_int32), ("cell_order", ctypes.c_int32),
                ("signal_velocity", ctypes.c_int32), ("balsara", ctypes.c_int32),
                ("force_form", ctypes.c_int32)]


class sph_stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("rebuilds", ctypes.c_int32),
                ("unconverged", ctypes.c_int64), ("interactions_density", ctypes.c_int64),
                ("interactions_force", ctypes.c_int64), ("candidates_density", ctypes.c_int64),
                ("candidates_force", ctypes.c_int64), ("n_cells", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("sweep_interactions_density", ctypes.c_int64),
                ("rescanned_density", ctypes.c_int64), ("tests_density", ctypes.c_int64),
                ("listed_density", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class sph_build_info(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("max_cell_particles", ctypes.c_int64),
                ("max_neighbour_cells", ctypes.c_int64), ("max_candidates", ctypes.c_int64),
                ("candidate_pairs", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class sph_timings(ctypes.Structure):
    _fields_ = [("density_kernel_ms", ctypes.c_double), ("density_call_ms", ctypes.c_double),
                ("force_kernel_ms", ctypes.c_double), ("force_call_ms", ctypes.c_double),
                ("build_ms", ctypes.c_double), ("density_launches", ctypes.c_int32),
                ("density_rescan_ms", ctypes.c_double), ("pass_call_ms", ctypes.c_double),
                ("builds", ctypes.c_int64), ("gravity_kernel_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class SphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (status_string(code), msg))
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``libsph.so``; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsph.so is not built (run __graft_entry__.build() or "
                           "python paper_1508_00115_amd/build.py); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    S = ctypes.c_int
    lib.sph_create.argtypes = [ctypes.POINTER(sph_params), ctypes.c_int, ctypes.POINTER(P)]
    lib.sph_create.restype = S
    lib.sph_destroy.argtypes = [P]
    lib.sph_destroy.restype = None
    lib.sph_build_cells.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int64, P, P, P]
    lib.sph_build_cells.restype = S
    lib.sph_density.argtypes = [P, P, P, P, P, P, ctypes.POINTER(sph_stats), P]
    lib.sph_density.restype = S
    lib.sph_force.argtypes = [P, P, P, P, P, P, ctypes.POINTER(sph_stats), P]
    lib.sph_force.restype = S
    lib.sph_pass.argtypes = [P] * 11 + [ctypes.POINTER(sph_stats), P]
    lib.sph_pass.restype = S
    lib.sph_density_f64.argtypes = [P, P, P, P, P, P, ctypes.POINTER(sph_stats), P]
    lib.sph_density_f64.restype = S
    lib.sph_force_f64.argtypes = [P, P, P, P, P, P, ctypes.POINTER(sph_stats), P]
    lib.sph_force_f64.restype = S
    lib.sph_get_timings.argtypes = [P, ctypes.POINTER(sph_timings)]
    lib.sph_get_timings.restype = S
    lib.sph_get_build_info.argtypes = [P, ctypes.POINTER(sph_build_info)]
    lib.sph_get_build_info.restype = S
    lib.sph_status_string.argtypes = [S]
    lib.sph_status_string.restype = ctypes.c_char_p
    lib.sph_last_error.argtypes = [P]
    lib.sph_last_error.restype = ctypes.c_char_p
    lib.sph_version.argtypes = []
    lib.sph_version.restype = ctypes.c_char_p
    lib.sph_kick.argtypes = [P, ctypes.c_double, P, P, P, P, P, P, P]
    lib.sph_kick.restype = ctypes.c_int
    lib.sph_drift.argtypes = [P, ctypes.c_double, P, P, P]
    lib.sph_drift.restype = ctypes.c_int
    lib.sph_timestep.argtypes = [P, ctypes.c_double, ctypes.POINTER(ctypes.c_double), P]
    lib.sph_timestep.restype = ctypes.c_int
    lib.sph_timestep_noalloc.argtypes = [P, ctypes.c_double, ctypes.POINTER(ctypes.c_double), P]
    lib.sph_timestep_noalloc.restype = ctypes.c_int
    lib.sph_predict_h.argtypes = [P, ctypes.c_double, P, P]
    lib.sph_predict_h.restype = ctypes.c_int
    lib.sph_get_balsara.argtypes = [P, P, P]
    lib.sph_get_balsara.restype = ctypes.c_int
    lib.sph_gravity_p2p.argtypes = [P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P, P]
    lib.sph_gravity_p2p.restype = ctypes.c_int
    lib.sph_struct_size.argtypes = [ctypes.c_int32]
    lib.sph_struct_size.restype = ctypes.c_int32
    _lib = lib
    return lib


# ---- one-to-one wrappers of the C ABI -------------------------------------------


def status_string(code: int) -> str:
    return load_library().sph_status_string(int(code)).decode()


def sph_last_error(ctx) -> str:
    return load_library().sph_last_error(ctx).decode()


def sph_version() -> str:
    return load_library().sph_version().decode()


def _check(code: int, ctx) -> None:
    if code != SPH_OK:
        raise SphError(code, sph_last_error(ctx))


def sph_create(params: sph_params | None = None, hip_device: int = 0):
    lib = load_library()
    out = ctypes.c_void_p()
    rc = lib.sph_create(ctypes.byref(params) if params is not None else None, int(hip_device),
                        ctypes.byref(out))
    _check(rc, None)
    return out


def sph_destroy(ctx) -> None:
    load_library().sph_destroy(ctx)


def sph_build_cells(ctx, n_boxes, box_first_ptr, box_len_ptr, n, pos_ptr, h_guess_ptr, stream) -> int:
    return load_library().sph_build_cells(ctx, n_boxes, box_first_ptr, box_len_ptr, n, pos_ptr,
                                          h_guess_ptr, stream)


def sph_density(ctx, mass, h, rho, f, nw, stats, stream) -> int:
    return load_library().sph_density(ctx, mass, h, rho, f, nw, stats, stream)


def sph_force(ctx, vel, u, acc, dudt, cons, stats, stream) -> int:
    return load_library().sph_force(ctx, vel, u, acc, dudt, cons, stats, stream)


def sph_pass(ctx, mass, h, rho, f, nw, vel, u, acc, dudt, cons, stats, stream) -> int:
    return load_library().sph_pass(ctx, mass, h, rho, f, nw, vel, u, acc, dudt, cons, stats, stream)


def sph_density_f64(ctx, mass, h, rho, f, nw, stats, stream) -> int:
    return load_library().sph_density_f64(ctx, mass, h, rho, f, nw, stats, stream)


def sph_force_f64(ctx, vel, u, acc, dudt, cons, stats, stream) -> int:
    return load_library().sph_force_f64(ctx, vel, u, acc, dudt, cons, stats, stream)


def sph_kick(ctx, dt, acc, dudt, vel_in, u_in, vel_out, u_out, stream) -> int:
    return load_library().sph_kick(ctx, dt, acc, dudt, vel_in, u_in, vel_out, u_out, stream)


def sph_drift(ctx, dt, vel, pos, stream) -> int:
    return load_library().sph_drift(ctx, dt, vel, pos, stream)


def sph_timestep(ctx, courant, dt_out, stream) -> int:
    return load_library().sph_timestep(ctx, courant, dt_out, stream)


def sph_predict_h(ctx, dt, h, stream) -> int:
    return load_library().sph_predict_h(ctx, dt, h, stream)


def sph_timestep_noalloc(ctx, courant, dt_out, stream) -> int:
    return load_library().sph_timestep_noalloc(ctx, courant, dt_out, stream)


def sph_get_balsara(ctx, balsara, stream) -> int:
    return load_library().sph_get_balsara(ctx, balsara, stream)


def sph_gravity_p2p(ctx, mass, G, eps, r_cut, acc, counts_out, stream) -> int:
    return load_library().sph_gravity_p2p(ctx, mass, G, eps, r_cut, acc, counts_out, stream)


def sph_get_timings(ctx, out) -> int:
    return load_library().sph_get_timings(ctx, out)


def sph_get_build_info(ctx, out) -> int:
    return load_library().sph_get_build_info(ctx, out)


# ---- torch convenience ---------------------------------------------------------------


def _dev(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """One library context on one GPU, driven with torch tensors."""

    def __init__(self, device: int = 0, **params):
        p = sph_params()
        for k, v in params.items():
            setattr(p, k, v)
        self.device = device
        self.signal_velocity = bool(params.get("signal_velocity", 0))
        self.ctx = sph_create(p, device)
        self.n = 0
        self.n_boxes = 0

    def close(self):
        if self.ctx:
            sph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timings(self) -> dict:
        t = sph_timings()
        _check(sph_get_timings(self.ctx, ctypes.byref(t)), self.ctx)
        return t.as_dict()

    def build_info(self) -> dict:
        b = sph_build_info()
        _check(sph_get_build_info(self.ctx, ctypes.byref(b)), self.ctx)
        return b.as_dict()

    def build_cells(self, pos, h_guess, box_first=None, box_len=None, stream=None):
        import torch
        n = pos.shape[0]
        if box_first is None:
            box_first = np.array([0, n], dtype=np.int64)
        if box_len is None:
            box_len = np.ones(len(box_first) - 1)
        bf = np.ascontiguousarray(box_first, dtype=np.int64)
        bl = np.ascontiguousarray(box_len, dtype=np.float64)
        rc = sph_build_cells(self.ctx, len(bl), bf.ctypes.data_as(ctypes.c_void_p),
                             bl.ctypes.data_as(ctypes.c_void_p), n,
                             _dev(pos, torch.float64, (n, 3), "pos"),
                             _dev(h_guess, torch.float32, (n,), "h_guess"), _stream(stream))
        _check(rc, self.ctx)
        self.n = n
        self.n_boxes = len(bl)

    def density(self, mass, h, rho=None, f=None, nw=None, stream=None) -> dict:
        """h is updated in place; returns the output tensors and the stats."""
        import torch
        n = self.n or mass.shape[0]
        rho = torch.empty(n, dtype=torch.float32, device=h.device) if rho is None else rho
        f = torch.empty(n, dtype=torch.float32, device=h.device) if f is None else f
        st = sph_stats()
        rc = sph_density(self.ctx, _dev(mass, torch.float32, (n,), "mass"),
                         _dev(h, torch.float32, (n,), "h"), _dev(rho, torch.float32, (n,), "rho"),
                         _dev(f, torch.float32, (n,), "f"),
                         None if nw is None else _dev(nw, torch.float32, (n,), "nw"),
                         ctypes.byref(st), _stream(stream))
        _check(rc, self.ctx)
        return {"h": h, "rho": rho, "f": f, "nw": nw, "stats": st.as_dict()}

    def force(self, vel, u, acc=None, dudt=None, cons=True, stream=None) -> dict:
        import torch
        n = self.n or u.shape[0]
        acc = torch.empty((n, 3), dtype=torch.float32, device=u.device) if acc is None else acc
        dudt = torch.empty(n, dtype=torch.float32, device=u.device) if dudt is None else dudt
        cb = np.zeros((self.n_boxes, 4)) if cons else None
        st = sph_stats()
        rc = sph_force(self.ctx, _dev(vel, torch.float32, (n, 3), "vel"), _dev(u, torch.float32, (n,), "u"),
                       _dev(acc, torch.float32, (n, 3), "acc"), _dev(dudt, torch.float32, (n,), "dudt"),
                       None if cb is None else cb.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st),
                       _stream(stream))
        _check(rc, self.ctx)
        return {"acc": acc, "dudt": dudt, "cons": cb, "stats": st.as_dict()}

    def pass_(self, mass, h, vel, u, rho=None, f=None, acc=None, dudt=None, nw=None, cons=False,
              stream=None) -> dict:
        """sph_pass: density then force in one launch sequence; h is updated in place."""
        import torch
        n = self.n or mass.shape[0]
        rho = torch.empty(n, dtype=torch.float32, device=h.device) if rho is None else rho
        f = torch.empty(n, dtype=torch.float32, device=h.device) if f is None else f
        acc = torch.empty((n, 3), dtype=torch.float32, device=h.device) if acc is None else acc
        dudt = torch.empty(n, dtype=torch.float32, device=h.device) if dudt is None else dudt
        cb = np.zeros((self.n_boxes, 4)) if cons else None
        st = sph_stats()
        rc = sph_pass(self.ctx, _dev(mass, torch.float32, (n,), "mass"), _dev(h, torch.float32, (n,), "h"),
                      _dev(rho, torch.float32, (n,), "rho"), _dev(f, torch.float32, (n,), "f"),
                      None if nw is None else _dev(nw, torch.float32, (n,), "nw"),
                      _dev(vel, torch.float32, (n, 3), "vel"), _dev(u, torch.float32, (n,), "u"),
                      _dev(acc, torch.float32, (n, 3), "acc"), _dev(dudt, torch.float32, (n,), "dudt"),
                      None if cb is None else cb.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st),
                      _stream(stream))
        _check(rc, self.ctx)
        return {"h": h, "rho": rho, "f": f, "nw": nw, "acc": acc, "dudt": dudt, "cons": cb,
                "stats": st.as_dict()}

    # ---- time integration (kick-drift-kick leapfrog) ------------------------------------

    def kick(self, dt, acc, dudt, vel, u, vel_out=None, u_out=None, stream=None):
        """sph_kick: vel_out = vel + acc dt, u_out = u + dudt dt (in place by default)."""
        import torch
        n = self.n
        vel_out = vel if vel_out is None else vel_out
        u_out = u if u_out is None else u_out
        rc = sph_kick(self.ctx, float(dt), _dev(acc, torch.float32, (n, 3), "acc"),
                      _dev(dudt, torch.float32, (n,), "dudt"), _dev(vel, torch.float32, (n, 3), "vel"),
                      _dev(u, torch.float32, (n,), "u"), _dev(vel_out, torch.float32, (n, 3), "vel_out"),
                      _dev(u_out, torch.float32, (n,), "u_out"), _stream(stream))
        _check(rc, self.ctx)
        return vel_out, u_out

    def drift(self, dt, vel, pos, stream=None):
        """sph_drift: pos += vel dt, wrapped into the boxes (the cells are kept)."""
        import torch
        n = self.n
        rc = sph_drift(self.ctx, float(dt), _dev(vel, torch.float32, (n, 3), "vel"),
                       _dev(pos, torch.float64, (n, 3), "pos"), _stream(stream))
        _check(rc, self.ctx)
        return pos

    def timestep(self, courant, stream=None) -> float:
        """sph_timestep: courant * min h / v_sig after the last force pass."""
        out = ctypes.c_double()
        rc = sph_timestep(self.ctx, float(courant), ctypes.byref(out), _stream(stream))
        _check(rc, self.ctx)
        return out.value

    def predict_h(self, dt, h, stream=None):
        """sph_predict_h: h *= exp(dt div v / 3) from the last force pass."""
        import torch
        rc = sph_predict_h(self.ctx, float(dt), _dev(h, torch.float32, (self.n,), "h"), _stream(stream))
        _check(rc, self.ctx)
        return h

    def timestep_noalloc(self, courant, stream=None) -> float:
        """sph_timestep_noalloc: sph_timestep with its scratch in the
        library's static device array (no allocation)."""
        out = ctypes.c_double()
        rc = sph_timestep_noalloc(self.ctx, float(courant), ctypes.byref(out), _stream(stream))
        _check(rc, self.ctx)
        return out.value

    def balsara(self, out=None, stream=None):
        """sph_get_balsara: the Balsara factors of the last force pass, in
        input order (float32, (n,), on the context's device)."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float32, device=self.device)
        rc = sph_get_balsara(self.ctx, _dev(out, torch.float32, (self.n,), "balsara"), _stream(stream))
        _check(rc, self.ctx)
        return out

    def gravity_p2p(self, mass, G, eps, r_cut, acc=None, stream=None, candidates=False):
        """sph_gravity_p2p: the near-field gravity of every particle over the
        pairs closer than r_cut (float32, (n, 3), input order) and the number
        of ordered pairs (and of the candidate pairs tested, with
        candidates=True)."""
        import torch
        n = self.n
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float32, device=self.device)
        counts = (ctypes.c_int64 * 2)()
        rc = sph_gravity_p2p(self.ctx, _dev(mass, torch.float32, (n,), "mass"), float(G), float(eps), float(r_cut),
                             _dev(acc, torch.float32, (n, 3), "acc"), counts, _stream(stream))
        _check(rc, self.ctx)
        return (acc, counts[0], counts[1]) if candidates else (acc, counts[0])

    def step(self, dt, pos, mass, h, vel, u, acc, dudt, rho=None, f=None, stream=None,
             predict_h=True) -> dict:
        """One kick-drift-kick step of length dt (every array in place): acc
        and dudt hold the rates at the start and hold those at the end on
        return. The sequence of sph.h (half kick, drift, prediction, pass,
        half kick; the library keeps or rebuilds the cells). With signal
        velocities on (and predict_h), h is advanced after the drift by the
        velocity divergence of the last pass (sph_predict_h), a better
        starting guess for the solve; the result does not depend on it. The predicted v
        and u, and rho and f when not given, live in
        scratch tensors that the next step reuses (copy them to keep them):
        with the same arrays every step, a step that keeps the cells replays
        the captured pass instead of capturing it again."""
        import torch
        key = (vel.shape, vel.dtype, vel.device, u.shape, u.dtype)
        sc = getattr(self, "_step_scratch", None)
        if sc is None or sc["key"] != key:
            sc = {"key": key, "vel_p": torch.empty_like(vel), "u_p": torch.empty_like(u),
                  "rho": torch.empty_like(u), "f": torch.empty_like(u)}
            self._step_scratch = sc
        vel_p, u_p = sc["vel_p"], sc["u_p"]
        rho = sc["rho"] if rho is None else rho
        f = sc["f"] if f is None else f
        self.kick(0.5 * dt, acc, dudt, vel, u, stream=stream)
        self.drift(dt, vel, pos, stream=stream)
        if predict_h and self.signal_velocity:
            # the starting guesses of the next solve, from the velocity
            # divergence the last force pass recorded
            self.predict_h(dt, h, stream=stream)
        self.kick(0.5 * dt, acc, dudt, vel, u, vel_p, u_p, stream=stream)
        r = self.pass_(mass, h, vel_p, u_p, rho=rho, f=f, acc=acc, dudt=dudt, stream=stream)
        self.kick(0.5 * dt, acc, dudt, vel, u, stream=stream)
        return r

    def density_f64(self, mass, h, rho=None, f=None, nw=None, stream=None) -> dict:
        import torch
        n = self.n
        rho = torch.empty(n, dtype=torch.float64, device=h.device) if rho is None else rho
        f = torch.empty(n, dtype=torch.float64, device=h.device) if f is None else f
        st = sph_stats()
        rc = sph_density_f64(self.ctx, _dev(mass, torch.float64, (n,), "mass"),
                             _dev(h, torch.float64, (n,), "h"), _dev(rho, torch.float64, (n,), "rho"),
                             _dev(f, torch.float64, (n,), "f"),
                             None if nw is None else _dev(nw, torch.float64, (n,), "nw"),
                             ctypes.byref(st), _stream(stream))
        _check(rc, self.ctx)
        return {"h": h, "rho": rho, "f": f, "nw": nw, "stats": st.as_dict()}

    def force_f64(self, vel, u, acc=None, dudt=None, cons=True, stream=None) -> dict:
        import torch
        n = self.n
        acc = torch.empty((n, 3), dtype=torch.float64, device=u.device) if acc is None else acc
        dudt = torch.empty(n, dtype=torch.float64, device=u.device) if dudt is None else dudt
        cb = np.zeros((self.n_boxes, 4)) if cons else None
        st = sph_stats()
        rc = sph_force_f64(self.ctx, _dev(vel, torch.float64, (n, 3), "vel"),
                           _dev(u, torch.float64, (n,), "u"), _dev(acc, torch.float64, (n, 3), "acc"),
                           _dev(dudt, torch.float64, (n,), "dudt"),
                           None if cb is None else cb.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st),
                           _stream(stream))
        _check(rc, self.ctx)
        return {"acc": acc, "dudt": dudt, "cons": cb, "stats": st.as_dict()}


def run_workload(ctx: Context, d: dict, device="cuda:0", fp64: bool = False) -> dict:
    """Upload a workload dict (see the ``workloads`` package) and run build,
    density and force; returns host numpy copies of every output."""
    import torch
    pos = torch.from_numpy(d["pos"]).to(device)
    h0 = torch.from_numpy(d["h0"]).to(device)
    ctx.build_cells(pos, h0, d["box_first"], d["box_len"])
    ft = torch.float64 if fp64 else torch.float32
    mass = torch.from_numpy(d["mass"]).to(device=device, dtype=ft)
    h = torch.from_numpy(d["h0"]).to(device=device, dtype=ft)
    vel = torch.from_numpy(d["vel"]).to(device=device, dtype=ft)
    u = torch.from_numpy(d["u"]).to(device=device, dtype=ft)
    nw = torch.empty_like(h)
    if fp64:
        dr = ctx.density_f64(mass, h, nw=nw)
        fr = ctx.force_f64(vel, u)
    else:
        dr = ctx.density(mass, h, nw=nw)
        fr = ctx.force(vel, u)
    torch.cuda.synchronize()
    out = {k: dr[k].double().cpu().numpy() for k in ("h", "rho", "f", "nw")}
    out["acc"] = fr["acc"].double().cpu().numpy()
    out["dudt"] = fr["dudt"].double().cpu().numpy()
    out["cons"] = fr["cons"]
    out["stats_density"] = dr["stats"]
    out["stats_force"] = fr["stats"]
    return out
