"""Parity of the Balsara switch (sph_params.balsara) with the FP64 oracle:
the factors B (through sph_get_balsara) and the force with the switch, on
the direct calls and on the captured pass, with both cell schedules.

B error bound: div v and curl v are FP32 sums of about 50 terms, each at
most m_j |v_ij| Dm_i / rho_i (Dm_i the kernel's largest slope); their errors
stay below 5e-5 of the sum of those bounds (the oracle's ``scale_dc``), and
B = |div| / den moves by at most twice that over den."""

import numpy as np
import pytest

import oracle
import workloads
from parity import TOL32, assert_within, errors

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "lattice_vel":
        return workloads.lattice_box(20, [1508, 901], jitter=0.3, u=1.0, vel_sigma=0.3)
    if name == "batched8":
        return workloads.batched(n_boxes=8, n_min=1000, n_max=8000, side_min=10, side_max=20)
    if name == "clustered_vel":
        d = workloads.clustered(n_uniform=1 << 14, n_spheres=4, per_sphere=4096)
        n = d["pos"].shape[0]
        d["vel"] = np.random.default_rng([1508, 960]).normal(0.0, 0.3, size=(n, 3)).astype(np.float32)
        return d
    if name == "sedov32":
        return workloads.sedov(n_side=32, n_hot=32)
    raise KeyError(name)


def _b_errors(gB, r):
    den = np.abs(r["div"]) + np.linalg.norm(r["curl"], axis=1) + 1e-4 * np.sqrt(
        oracle.GAMMA * (oracle.GAMMA - 1.0) * r["u"]) / r["h"]
    bound = 2 * 5e-5 * r["scale_dc"] / den + 1e-7
    return float(np.max(np.abs(gB - r["balsara"]) / bound))


@pytest.mark.parametrize("name,params", [("lattice_vel", {}), ("lattice_vel", {"schedule": 1}),
                                         ("batched8", {}), ("clustered_vel", {}), ("sedov32", {})])
def test_balsara_matches_oracle(gpu_lib, name, params):
    import torch
    d = _case(name)
    print("case", name, params, "N", d["pos"].shape[0], flush=True)
    ctx = gpu_lib.Context(0, balsara=1, **params)
    try:
        g = gpu_lib.run_workload(ctx, d)
        gB = ctx.balsara().double().cpu().numpy()
        # the captured pass gives the same factors and force
        dev = "cuda:0"
        mass = torch.from_numpy(d["mass"]).to(dev)
        h = torch.from_numpy(d["h0"]).to(dev)
        vel = torch.from_numpy(d["vel"]).to(dev)
        u = torch.from_numpy(d["u"]).to(dev)
        rp = ctx.pass_(mass, h, vel, u)
        torch.cuda.synchronize()
        gB2 = ctx.balsara().double().cpu().numpy()
        acc2 = rp["acc"].double().cpu().numpy()
    finally:
        ctx.close()
    r = oracle.run(d, balsara=True)
    r["u"] = np.asarray(d["u"], dtype=np.float64)
    eb = _b_errors(gB, r)
    e = errors(g, r)
    print(name, "B err / bound", eb, e, flush=True)
    assert eb <= 1.0
    assert_within(e, TOL32, name)
    assert _b_errors(gB2, r) <= 1.0
    da = np.linalg.norm(acc2 - r["acc"], axis=1)
    assert np.all(da <= TOL32["acc"] * r["scale_a"] + 1e-30)
    if name == "sedov32":
        assert np.all(gB == 0.0)  # at rest: no divergence, no curl
    else:
        assert 0.1 < gB.mean() < 0.9
    for b, (mom, en, mscale, escale) in enumerate(r["cons"]):
        cg = g["cons"][b]
        assert np.all(np.abs(cg[:3]) <= 1e-5 * mscale + 1e-300)
        assert abs(cg[3]) <= 1e-5 * escale + 1e-300


def test_switch_changes_the_viscous_force_only(gpu_lib):
    # same cells, with and without the switch: the difference is the oracle's
    d = _case("lattice_vel")
    c0 = gpu_lib.Context(0)
    g0 = gpu_lib.run_workload(c0, d)
    c0.close()
    ctx = gpu_lib.Context(0, balsara=1)
    g1 = gpu_lib.run_workload(ctx, d)
    ctx.close()
    r0 = oracle.run(d)
    r1 = oracle.run(d, balsara=True)
    diff_o = r1["acc"] - r0["acc"]
    diff_g = g1["acc"] - g0["acc"]
    assert np.max(np.linalg.norm(diff_o, axis=1) / r0["scale_a"]) > 1e-2  # the switch matters here
    assert np.all(np.linalg.norm(diff_g - diff_o, axis=1) <= 2 * TOL32["acc"] * r0["scale_a"])


def test_balsara_error_paths(gpu_lib):
    import torch
    d = _case("lattice_vel")
    ctx = gpu_lib.Context(0, balsara=1)
    try:
        pos = torch.from_numpy(d["pos"]).to("cuda:0")
        ctx.build_cells(pos, torch.from_numpy(d["h0"]).to("cuda:0"), d["box_first"], d["box_len"])
        with pytest.raises(gpu_lib.SphError, match="sph_get_balsara"):
            ctx.balsara()
        mass = torch.from_numpy(d["mass"]).to("cuda:0", torch.float64)
        h = torch.from_numpy(d["h0"]).to("cuda:0", torch.float64)
        ctx.density_f64(mass, h)
        with pytest.raises(gpu_lib.SphError, match="Balsara"):
            ctx.force_f64(torch.from_numpy(d["vel"]).to("cuda:0", torch.float64),
                          torch.from_numpy(d["u"]).to("cuda:0", torch.float64))
    finally:
        ctx.close()
