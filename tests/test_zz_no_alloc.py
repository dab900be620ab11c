"""sph_timestep_noalloc (the entry point that allocates nothing; its scratch
is the library's static device array) against sph_timestep through the C
ABI: the same dt bit for bit, on two calls in a row, the second with a
smaller input, and again on the first context afterwards (the shared array
keeps the last call's contents, which must not leak into the next)."""

import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _ctx(sph, n_side, seed):
    import torch
    d = workloads.lattice_box(n_side, [1508, seed], jitter=0.3, u=1.0, vel_sigma=0.3)
    t = {k: torch.from_numpy(d[k]).cuda() for k in ("pos", "h0", "mass", "vel", "u")}
    ctx = sph.Context(0, signal_velocity=1)
    ctx.build_cells(t["pos"], t["h0"])
    ctx.pass_(t["mass"], t["h0"].clone(), t["vel"], t["u"])
    return ctx, d["pos"].shape[0]


def _both(sph, ctx):
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ref, na = ctypes.c_double(), ctypes.c_double()
    assert sph.sph_timestep(ctx.ctx, 0.3, ctypes.byref(ref), s) == sph.SPH_OK
    assert sph.sph_timestep_noalloc(ctx.ctx, 0.3, ctypes.byref(na), s) == sph.SPH_OK
    return ref.value, na.value


def test_noalloc_timestep_matches(gpu_lib):
    sph = gpu_lib
    # 104^3 particles: more workgroups' worth than the static array has
    # slots, so the workgroups stride over the particles
    big, n_big = _ctx(sph, 104, 920)
    small, n_small = _ctx(sph, 12, 921)
    assert n_big > 4096 * 256 > n_small
    try:
        r1, a1 = _both(sph, big)
        r2, a2 = _both(sph, small)
        r3, a3 = _both(sph, big)
        print("dt", r1, a1, r2, a2, r3, a3, flush=True)
        assert np.isfinite(r1) and r1 > 0 and r2 > 0
        assert a1 == r1 and a2 == r2 and a3 == r3
        assert r1 != r2
    finally:
        big.close()
        small.close()


def test_noalloc_timestep_errors(gpu_lib):
    import torch
    sph = gpu_lib
    d = workloads.lattice_box(12, [1508, 922], jitter=0.3, u=1.0, vel_sigma=0.3)
    t = {k: torch.from_numpy(d[k]).cuda() for k in ("pos", "h0", "mass", "vel", "u")}
    ctx = sph.Context(0, signal_velocity=1)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = ctypes.c_double()
    try:
        ctx.build_cells(t["pos"], t["h0"])
        assert sph.sph_timestep_noalloc(ctx.ctx, 0.3, ctypes.byref(out), s) == sph.SPH_E_STATE
        ctx.pass_(t["mass"], t["h0"].clone(), t["vel"], t["u"])
        assert sph.sph_timestep_noalloc(ctx.ctx, -1.0, ctypes.byref(out), s) == sph.SPH_E_ARG
        assert sph.sph_timestep_noalloc(ctx.ctx, 0.3, None, s) == sph.SPH_E_ARG
        assert sph.sph_timestep_noalloc(None, 0.3, ctypes.byref(out), s) == sph.SPH_E_ARG
        assert ctx.timestep_noalloc(0.3) == ctx.timestep(0.3)
    finally:
        ctx.close()
