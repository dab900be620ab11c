"""Time integration on the GPU (sph_kick, sph_drift, sph_timestep with the
force loop's signal velocities) against the oracle's leapfrog.

One step is checked three ways: the kick and drift arithmetic against the
step's own inputs (FP32 rounding only); the force at the end of the step
against the oracle evaluated on the GPU's own predicted state (the FP32
tolerances of the pass); and the whole step against the oracle's step from
the same start, within the bounds the rate tolerances imply. A Sedov blast
run checks the physics the step sequence produces: the shock radius of the
Sedov-Taylor similarity solution and energy conservation."""

import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import leapfrog
from parity import TOL32, TOL64, assert_within, errors

pytestmark = pytest.mark.gpu


def _tensors(d):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(d[k])).cuda() for k in ("pos", "h0", "mass", "vel", "u")}


def _np(t):
    return t.double().cpu().numpy()


def _case():
    return workloads.lattice_box(20, [1508, 960], jitter=0.3, u=1.0, vel_sigma=0.3)


def test_timestep_matches_oracle(gpu_lib):
    d = _case()
    t = _tensors(d)
    ctx = gpu_lib.Context(0, signal_velocity=1)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        h = t["h0"].clone()
        ctx.pass_(t["mass"], h, t["vel"], t["u"])
        dt = ctx.timestep(0.3)
    finally:
        ctx.close()
    r = oracle.run(d)
    dt_o = leapfrog.timestep(r["h"], r["vsig"], 0.3)
    print("dt", dt, dt_o, flush=True)
    # h to 1e-5 (the density tolerance); v_sig from FP32 sound speeds and velocities
    assert abs(dt / dt_o - 1.0) < 2e-5


def test_timestep_needs_signal_velocities(gpu_lib):
    d = _case()
    t = _tensors(d)
    ctx = gpu_lib.Context(0)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        h = t["h0"].clone()
        ctx.pass_(t["mass"], h, t["vel"], t["u"])
        with pytest.raises(gpu_lib.SphError) as e:
            ctx.timestep(0.3)
        assert e.value.code == gpu_lib.SPH_E_STATE
    finally:
        ctx.close()


def _drifted(d, x):
    e = dict(d)
    e["pos"] = x
    return e


def _boxes8():
    # eight boxes of different particle counts, scaled to sides 0.8 .. 1.5
    d = workloads.batched(n_boxes=8, n_min=1000, n_max=8000, side_min=10, side_max=20)
    pos, h0 = d["pos"].copy(), d["h0"].astype(np.float64)
    L = 0.8 + 0.1 * np.arange(8)
    for b in range(8):
        s, e = int(d["box_first"][b]), int(d["box_first"][b + 1])
        pos[s:e] *= L[b]
        h0[s:e] *= L[b]
    d["pos"], d["h0"], d["box_len"] = pos, h0.astype(np.float32), L
    return d


def _clustered_vel():
    # Plummer spheres in a uniform background (cells of several sizes, so the
    # density culls against the particle boxes refreshed after each drift)
    d = workloads.clustered(n_uniform=6000, n_spheres=4, per_sphere=1500, a_range=(0.02, 0.08))
    rng = np.random.default_rng([1508, 961])
    d["vel"] = rng.normal(0.0, 0.3, size=d["pos"].shape).astype(np.float32)
    return d


@pytest.mark.parametrize("case", ["lattice", "batched8", "clustered"])
def test_drift_keeps_the_cells(gpu_lib, case):
    """After drifts the pass runs on the kept cells (search radius reduced by
    twice the drift bound) and, once the bound eats the margin, on rebuilt
    ones; both against the oracle at the drifted positions (one box, eight
    boxes of different sides and counts, each wrapped on its own, and a
    clustered set whose cells have several sizes)."""
    import torch
    d = {"lattice": _case, "batched8": _boxes8, "clustered": _clustered_vel}[case]()
    t = _tensors(d)
    ctx = gpu_lib.Context(0, signal_velocity=1)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        h = t["h0"].clone()
        r = ctx.pass_(t["mass"], h, t["vel"], t["u"])
        vmax = float(np.abs(d["vel"]).max())
        # the rebuild threshold: 2 delta > (1 - 1/h_margin) h_margin min(h_guess), h_margin 1.26
        budget = (1.0 - 1.0 / 1.26) * 1.26 * float(d["h0"].min())
        dt = 0.2 * budget / (2.0 * math.sqrt(3.0) * vmax)  # delta well inside the budget
        ctx.drift(dt, t["vel"], t["pos"])
        for call in (lambda: ctx.timestep(0.3), lambda: ctx.force(t["vel"], t["u"])):
            with pytest.raises(gpu_lib.SphError) as e:
                call()
            assert e.value.code == gpu_lib.SPH_E_STATE
        with pytest.raises(gpu_lib.SphError) as e:
            ctx.kick(float("nan"), r["acc"], r["dudt"], t["vel"], t["u"])
        assert e.value.code == gpu_lib.SPH_E_ARG
        for regime, n_drift, step in (("kept cells", 1, dt), ("rebuilt cells", 8, 20.0 * dt)):
            if regime == "rebuilt cells":
                for _ in range(n_drift):
                    ctx.drift(step, t["vel"], t["pos"])
                delta = math.sqrt(3.0) * vmax * (dt + n_drift * step)
                assert 2.0 * delta > budget  # this regime must rebuild
            ro = oracle.run(_drifted(d, _np(t["pos"])))
            # the plain FP64 form first (its own check of the drift, and a
            # rebuild from the last guesses in the second regime), then FP32
            h64 = t["h0"].double().clone()
            r64 = ctx.density_f64(t["mass"].double(), h64)
            f64 = ctx.force_f64(t["vel"].double(), t["u"].double(), cons=False)
            torch.cuda.synchronize()
            g64 = {"h": _np(h64), "rho": _np(r64["rho"]), "f": _np(r64["f"]), "nw": _np(h64) * 0 + 1,
                   "acc": _np(f64["acc"]), "dudt": _np(f64["dudt"])}
            e64 = errors(g64, ro)
            e64["nw"] = 0.0
            print(regime, "fp64", e64, flush=True)
            assert_within(e64, TOL64, regime + " fp64")
            r = ctx.pass_(t["mass"], h, t["vel"], t["u"])
            torch.cuda.synchronize()
            g = {"h": _np(h), "rho": _np(r["rho"]), "f": _np(r["f"]), "nw": _np(h) * 0 + 1,
                 "acc": _np(r["acc"]), "dudt": _np(r["dudt"])}
            e = errors(g, ro)
            e["nw"] = 0.0
            print(regime, e, flush=True)
            assert_within(e, TOL32, regime)
            assert ctx.timestep(0.3) > 0
    finally:
        ctx.close()


def test_one_step_matches_oracle(gpu_lib):
    import torch
    d = _case()
    t = _tensors(d)
    ctx = gpu_lib.Context(0, signal_velocity=1)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        h = t["h0"].clone()
        r0 = ctx.pass_(t["mass"], h, t["vel"], t["u"])
        dt = ctx.timestep(0.25)
        a0, du0 = r0["acc"].clone(), r0["dudt"].clone()
        x0, v0, u0 = _np(t["pos"]), _np(t["vel"]), _np(t["u"])
        # the step of sph.h, with the intermediate arrays kept
        vel, u, pos = t["vel"].clone(), t["u"].clone(), t["pos"].clone()
        ctx.kick(0.5 * dt, a0, du0, vel, u)
        v_half, u_half = _np(vel), _np(u)
        ctx.drift(dt, vel, pos)
        vel_p, u_p = torch.empty_like(vel), torch.empty_like(u)
        ctx.kick(0.5 * dt, a0, du0, vel, u, vel_p, u_p)
        r1 = ctx.pass_(t["mass"], h, vel_p, u_p)  # on the kept cells
        ctx.kick(0.5 * dt, r1["acc"], r1["dudt"], vel, u)
        torch.cuda.synchronize()
        x1, vp, up, v1, u1 = _np(pos), _np(vel_p), _np(u_p), _np(vel), _np(u)
        a0n, du0n, a1n, du1n = _np(a0), _np(du0), _np(r1["acc"]), _np(r1["dudt"])
        g1 = {"h": _np(h), "rho": _np(r1["rho"]), "f": _np(r1["f"]), "nw": _np(h) * 0 + 1, "acc": a1n,
              "dudt": du1n}
    finally:
        ctx.close()
    print("dt", dt, flush=True)

    # (1) arithmetic of kick and drift on the step's own inputs: FP64 sums
    # rounded once to FP32 (1 ulp for a possible fused multiply-add)
    def f32(x):
        return np.float32(x).astype(np.float64)

    def ulp(x):
        return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)

    assert np.all(np.abs(v_half - f32(v0 + a0n * 0.5 * dt)) <= ulp(v_half))
    assert np.all(np.abs(u_half - f32(u0 + du0n * 0.5 * dt)) <= ulp(u_half))
    assert np.all(np.abs(vp - f32(v_half + a0n * 0.5 * dt)) <= ulp(vp))
    assert np.all(np.abs(up - f32(u_half + du0n * 0.5 * dt)) <= ulp(up))
    assert np.all(np.abs(v1 - f32(v_half + a1n * 0.5 * dt)) <= ulp(v1))
    assert np.all(np.abs(u1 - f32(u_half + du1n * 0.5 * dt)) <= ulp(u1))
    x_ref = leapfrog.drift(x0, v_half, dt, 1.0)
    dx = x1 - x_ref
    dx -= np.round(dx)
    assert np.max(np.abs(dx)) < 1e-15

    # (2) the force at the end of the step, on the GPU's own predicted state
    d1 = dict(d)
    d1["pos"], d1["vel"], d1["u"] = x1, vp, up
    ro = oracle.run(d1)
    e = errors(g1, ro)
    e["nw"] = 0.0  # not requested from the pass
    print("end-of-step force", e, flush=True)
    assert_within(e, TOL32, "end of step")

    # (3) the whole step against the oracle's step from the same start: the
    # rates differ within 1e-4 of their kernel scales, which bounds the state
    ra = oracle.run(d)
    so = leapfrog.kdk_step(d, ra["acc"], ra["dudt"], dt, h_start=ra["h"])
    sa = np.maximum(ra["scale_a"], so["scale_a"])
    su = np.maximum(ra["scale_u"], so["scale_u"])
    tol_v = 2.0 * (dt * 1e-4 * sa + 4e-7 * np.linalg.norm(v1, axis=1))
    tol_u = 2.0 * (dt * 1e-4 * su + 4e-7 * np.abs(u1))
    tol_x = 2.0 * (0.5 * dt * dt * 1e-4 * ra["scale_a"] + dt * 4e-7 * np.linalg.norm(v_half, axis=1)) + 1e-15
    dxo = x1 - so["pos"]
    dxo -= np.round(dxo)
    ev = np.linalg.norm(v1 - so["vel"], axis=1) / tol_v
    eu = np.abs(u1 - so["u"]) / tol_u
    ex = np.linalg.norm(dxo, axis=1) / tol_x
    print("step vs oracle (fraction of bound): v %.3f u %.3f x %.3f" % (ev.max(), eu.max(), ex.max()), flush=True)
    assert ev.max() <= 1.0 and eu.max() <= 1.0 and ex.max() <= 1.0


@pytest.mark.parametrize("balsara", [0, 1])
def test_sedov_taylor_blast(gpu_lib, balsara):
    """The Sedov 64^3 blast evolved to t = 0.025 with Courant factor 0.3 (with
    and without the Balsara switch, which leaves a radial shock's viscosity
    on). The
    shock of the similarity solution sits at R = xi (E t^2 / rho)^(1/5), xi =
    1.1517 for gamma = 5/3 in three dimensions; the SPH density peak spreads
    over the kernel, so it is held to within two post-shock smoothing lengths
    (h at four times the mean density) of R. The total energy sum m (v^2/2 +
    u) is held to 1%, the shock's density peak to at least twice the mean."""
    import time

    import torch
    d = workloads.sedov()
    t = _tensors(d)
    n = d["pos"].shape[0]
    m = d["mass"].astype(np.float64)
    E0 = float((m * d["u"].astype(np.float64)).sum())
    ctx = gpu_lib.Context(0, signal_velocity=1, balsara=balsara)
    try:
        pos, vel, u, h = t["pos"].clone(), t["vel"].clone(), t["u"].clone(), t["h0"].clone()
        ctx.build_cells(pos, h, d["box_first"], d["box_len"])
        r = ctx.pass_(t["mass"], h, vel, u)
        acc, dudt, rho = r["acc"], r["dudt"], r["rho"]
        t_now, t_end, steps = 0.0, 0.025, 0
        t0 = time.time()
        while t_now < t_end and steps < 20000:
            dt = min(ctx.timestep(0.3), t_end - t_now)
            r = ctx.step(dt, pos, t["mass"], h, vel, u, acc, dudt, rho=rho)
            t_now += dt
            steps += 1
            if steps % 200 == 0:
                print("sedov step", steps, "t %.5f dt %.2e" % (t_now, dt), flush=True)
        torch.cuda.synchronize()
        wall = time.time() - t0
        x, v, uu, rh = _np(pos), _np(vel), _np(u), _np(rho)
    finally:
        ctx.close()
    E1 = float((m * (0.5 * (v * v).sum(axis=1) + uu)).sum())
    rr = np.linalg.norm(x - 0.5, axis=1)
    bins = np.arange(0.0, 0.45, 0.01)
    idx = np.digitize(rr, bins)
    prof = np.array([rh[idx == k].mean() if np.any(idx == k) else 0.0 for k in range(1, len(bins))])
    r_peak = 0.5 * (bins[np.argmax(prof)] + bins[np.argmax(prof) + 1])
    R = 1.1517 * (E0 * t_now ** 2 / 1.0) ** 0.2
    h_post = 2.2545 * n ** (-1.0 / 3.0) * 4.0 ** (-1.0 / 3.0)
    print("balsara", balsara, flush=True)
    print("sedov: %d steps in %.1f s, t %.4f, R_peak %.3f, R_ST %.3f, peak rho %.2f, E %.6f -> %.6f"
          % (steps, wall, t_now, r_peak, R, prof.max(), E0, E1), flush=True)
    assert t_now >= t_end * (1 - 1e-12)
    assert abs(r_peak - R) <= 2.0 * h_post
    assert prof.max() >= 2.0
    assert abs(E1 / E0 - 1.0) < 1e-2


def test_flags_after_a_replayed_pass(gpu_lib):
    """sph_pass replays its captured graph when the cells and every array are
    unchanged, as after a short drift: the signal velocities and Balsara
    factors that the replay leaves must still serve sph_timestep and
    sph_get_balsara (a replay runs no host code of the force call)."""
    import torch
    d = workloads.lattice_box(16, [1508, 980], jitter=0.3, u=1.0, vel_sigma=0.3)
    t = _tensors(d)
    ctx = gpu_lib.Context(0, signal_velocity=1, balsara=1, h_margin=1.3)
    try:
        pos, vel, u, h = t["pos"].clone(), t["vel"].clone(), t["u"].clone(), t["h0"].clone()
        ctx.build_cells(pos, h, d["box_first"], d["box_len"])
        rho, f, nw, dudt = (torch.empty_like(h) for _ in range(4))
        acc = torch.empty_like(vel)
        kw = dict(rho=rho, f=f, nw=nw, acc=acc, dudt=dudt)
        ctx.pass_(t["mass"], h, vel, u, **kw)
        dt0 = ctx.timestep(0.3)
        B0 = ctx.balsara().clone()
        cells = ctx.build_info()["n_cells"]
        for k in range(3):
            print("replay", k, flush=True)
            ctx.drift(1e-3 * dt0, vel, pos)  # far inside the drift budget: the cells stay
            with pytest.raises(gpu_lib.SphError):
                ctx.timestep(0.3)
            ctx.pass_(t["mass"], h, vel, u, **kw)
            assert ctx.timestep(0.3) == pytest.approx(dt0, rel=1e-2)
            assert torch.allclose(ctx.balsara(), B0, atol=1e-2)
        assert ctx.build_info()["n_cells"] == cells
    finally:
        ctx.close()


def test_predict_h_follows_the_divergence(gpu_lib):
    """sph_predict_h advances h by exp(dt div v / 3), with the divergence the
    force pass recorded: recovered from the prediction, div v matches the
    oracle's (over the pairs inside h_i) to 1e-4 of its error scale."""
    d = _case()
    t = _tensors(d)
    ctx = gpu_lib.Context(0, signal_velocity=1)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        h = t["h0"].clone()
        ctx.pass_(t["mass"], h, t["vel"], t["u"])
        h_before = _np(h)
        r = oracle.run(d)
        dc = oracle.divcurl(d["pos"], d["vel"], d["mass"], r["h"], r["rho"])
        # a step long enough that exp(dt div / 3) moves h well above FP32 resolution
        dt = 0.15 / float(np.median(dc["scale"]))
        ctx.predict_h(dt, h)
        h_after = _np(h)
    finally:
        ctx.close()
    div_gpu = 3.0 * np.log(h_after / h_before) / dt
    err = np.abs(div_gpu - dc["div"]) / dc["scale"]
    print("div v from the prediction: max err %.2e of the scale, dt %.3g" % (err.max(), dt), flush=True)
    assert err.max() < 1e-4


def test_predict_h_needs_a_force_pass(gpu_lib):
    d = _case()
    t = _tensors(d)
    for sv in (0, 1):
        ctx = gpu_lib.Context(0, signal_velocity=sv)
        try:
            ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
            h = t["h0"].clone()
            with pytest.raises(gpu_lib.SphError) as ei:
                ctx.predict_h(1e-3, h)
            assert ei.value.code == gpu_lib.SPH_E_STATE
            ctx.pass_(t["mass"], h, t["vel"], t["u"])
            if sv:
                ctx.predict_h(1e-3, h)
                # kept across a drift (the particles keep their order)
                ctx.drift(1e-4, t["vel"], t["pos"].clone())
                ctx.predict_h(1e-3, h)
            else:
                with pytest.raises(gpu_lib.SphError) as ei:
                    ctx.predict_h(1e-3, h)
                assert ei.value.code == gpu_lib.SPH_E_STATE
        finally:
            ctx.close()


def test_predicted_h_saves_sweeps(gpu_lib):
    """Leapfrog steps of a lattice with a random velocity field, with and
    without the h prediction: the same results within the pass tolerance,
    fewer Newton evaluations per particle with the prediction."""
    import torch
    d = _case()
    out = {}
    for pred in (False, True):
        t = _tensors(d)
        ctx = gpu_lib.Context(0, signal_velocity=1)
        try:
            pos, vel, u, h = t["pos"].clone(), t["vel"].clone(), t["u"].clone(), t["h0"].clone()
            ctx.build_cells(pos, h, d["box_first"], d["box_len"])
            r = ctx.pass_(t["mass"], h, vel, u)
            acc, dudt, rho = r["acc"], r["dudt"], r["rho"]
            evals, inter = 0, 0
            for _ in range(6):
                dt = ctx.timestep(0.3)
                r = ctx.step(dt, pos, t["mass"], h, vel, u, acc, dudt, rho=rho, predict_h=pred)
                evals += r["stats"]["sweep_interactions_density"]
                inter += r["stats"]["interactions_density"]
            torch.cuda.synchronize()
            out[pred] = (evals / inter, _np(h), _np(rho))
        finally:
            ctx.close()
    print("evaluations per particle: without %.3f, with the prediction %.3f" % (out[False][0], out[True][0]),
          flush=True)
    assert out[True][0] < out[False][0]
    assert np.max(np.abs(out[True][1] / out[False][1] - 1)) < 2e-5
    assert np.max(np.abs(out[True][2] / out[False][2] - 1)) < 2e-5
