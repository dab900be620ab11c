"""sph_pass (density + force as one launch sequence, captured into a HIP
graph) against separate sph_density + sph_force calls: the same kernels in
the same order, so the outputs must agree bit for bit, on every replay of the
graph, after recapture for new buffers, in the uncaptured timing mode and
through the rebuild fallback. One case is also held against the oracle."""

import numpy as np
import pytest

import oracle
import workloads
from parity import TOL32, assert_within, errors

pytestmark = pytest.mark.gpu

KEYS = ("h", "rho", "f", "acc", "dudt")


def _inputs(d):
    import torch
    t = {k: torch.from_numpy(d[k]).cuda() for k in ("pos", "h0", "mass", "vel", "u")}
    return t


def _separate(sph, d, **params):
    """Reference: sph_density then sph_force on a fresh context."""
    t = _inputs(d)
    ctx = sph.Context(0, **params)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        h = t["h0"].clone()
        dr = ctx.density(t["mass"], h)
        fr = ctx.force(t["vel"], t["u"])
        out = {"h": h, "rho": dr["rho"], "f": dr["f"], "acc": fr["acc"], "dudt": fr["dudt"]}
        out = {k: v.cpu().numpy() for k, v in out.items()}
        out["cons"] = fr["cons"]
        out["stats"] = {**dr["stats"], **{k: fr["stats"][k] for k in ("interactions_force", "candidates_force")}}
        return out
    finally:
        ctx.close()


def _pass(ctx, t, d, bufs=None):
    import torch
    n = t["pos"].shape[0]
    if bufs is None:
        bufs = {"h": t["h0"].clone(), "rho": torch.empty(n, device="cuda"), "f": torch.empty(n, device="cuda"),
                "acc": torch.empty((n, 3), device="cuda"), "dudt": torch.empty(n, device="cuda")}
    bufs["h"].copy_(t["h0"])
    r = ctx.pass_(t["mass"], bufs["h"], t["vel"], t["u"], rho=bufs["rho"], f=bufs["f"], acc=bufs["acc"],
                  dudt=bufs["dudt"], cons=True)
    torch.cuda.synchronize()
    out = {k: bufs[k].cpu().numpy() for k in KEYS}
    out["cons"] = r["cons"]
    out["stats"] = r["stats"]
    return out, bufs


def _same(a, b, label, d=None):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (label, k, np.max(np.abs(a[k] - b[k])))
    # the conservation sums are FP64 atomic sums whose order varies; they
    # cancel to ~0, so compare them on the scale of their terms
    if d is not None:
        m = d["mass"].astype(np.float64)
        acc, dudt, vel = b["acc"].astype(np.float64), b["dudt"].astype(np.float64), d["vel"].astype(np.float64)
        for box in range(len(d["box_len"])):
            sl = slice(int(d["box_first"][box]), int(d["box_first"][box + 1]))
            s_mom = np.sum(m[sl] * np.abs(acc[sl]).sum(axis=1))
            s_en = np.sum(m[sl] * (np.abs(np.einsum("ij,ij->i", vel[sl], acc[sl])) + np.abs(dudt[sl])))
            assert np.all(np.abs(a["cons"][box, :3] - b["cons"][box, :3]) <= 1e-12 * s_mom + 1e-300), label
            assert abs(a["cons"][box, 3] - b["cons"][box, 3]) <= 1e-12 * s_en + 1e-300, label
    for k in ("interactions_density", "interactions_force", "candidates_density", "candidates_force",
              "sweeps", "rescanned_density"):
        assert a["stats"][k] == b["stats"][k], (label, k, a["stats"][k], b["stats"][k])


def test_detail_counters(gpu_lib):
    """sph_params.timing = 2 counts the density loop's list-building tests and
    the candidates they list. Every particle lists each particle inside its
    search radius H_i = h_margin h_guess_i (itself included) once, so the
    listed count is sum_i #{j : r_ij < H_i} (scipy's cKDTree, periodic), up to
    pairs within FP32 rounding of H_i; the tests count at least those. Without
    it nothing is counted, and the outputs are the same bits either way."""
    from scipy.spatial import cKDTree
    d = workloads.small()
    t = _inputs(d)
    out = {}
    for timing in (0, 2):
        ctx = gpu_lib.Context(0, timing=timing, h_margin=1.26)
        try:
            ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
            out[timing], _ = _pass(ctx, t, d)
        finally:
            ctx.close()
    _same(out[0], out[2], "timing 2")
    st0, st = out[0]["stats"], out[2]["stats"]
    assert st0["tests_density"] == 0 and st0["listed_density"] == 0
    H = (np.float32(1.26) * d["h0"].astype(np.float32)).astype(np.float64)  # the FP32 radius of the build
    pos = np.mod(d["pos"], 1.0)
    tree = cKDTree(pos, boxsize=1.0)
    lo = int(tree.query_ball_point(pos, H * (1.0 - 1e-5), return_length=True).sum())
    hi = int(tree.query_ball_point(pos, H * (1.0 + 1e-5), return_length=True).sum())
    print("listed %d (expected %d..%d), tests %d" % (st["listed_density"], lo, hi, st["tests_density"]), flush=True)
    assert st["rescanned_density"] == 0
    assert lo <= st["listed_density"] <= hi
    assert st["tests_density"] >= st["listed_density"]


@pytest.mark.parametrize("name", ["small", "sedov32", "batched8", "mixed_mass"])
def test_pass_equals_density_then_force(gpu_lib, name):
    import torch
    if name == "small":
        d = workloads.small()
    elif name == "sedov32":
        d = workloads.sedov(n_side=32, n_hot=32)
    elif name == "batched8":
        d = workloads.batched(n_boxes=8, n_min=1000, n_max=8000, side_min=10, side_max=20)
    else:
        d = workloads.lattice_box(16, [1508, 906], jitter=0.3, u=1.0, vel_sigma=0.2)
        d["mass"] = (d["mass"] * np.random.default_rng([1508, 906, 1]).uniform(0.5, 1.5, d["mass"].shape[0])
                     ).astype(np.float32)
    print("case", name, flush=True)
    ref = _separate(gpu_lib, d)
    t = _inputs(d)
    ctx = gpu_lib.Context(0)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        bufs = None
        for rep in range(3):  # capture, then replays with eager work in between
            got, bufs = _pass(ctx, t, d, bufs)
            _same(got, ref, "%s replay %d" % (name, rep), d)
            scratch = torch.randn(4096, device="cuda")
            (scratch * 2).sum().item()
        # new output buffers: the pass is captured again
        got, _ = _pass(ctx, t, d)
        _same(got, ref, name + " recaptured", d)
    finally:
        ctx.close()


def test_pass_timing_mode_uncaptured(gpu_lib):
    """Timing mode launches the same kernels uncaptured with HIP events: the
    same bits, and durations from every call."""
    d = workloads.sedov(n_side=24, n_hot=16)
    ref = _separate(gpu_lib, d)
    t = _inputs(d)
    ctx = gpu_lib.Context(0, timing=1)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        bufs = None
        for rep in range(3):
            got, bufs = _pass(ctx, t, d, bufs)
            _same(got, ref, "timing mode replay %d" % rep, d)
            tm = ctx.timings()
            assert 0 < tm["density_kernel_ms"] < tm["pass_call_ms"], tm
            assert 0 < tm["force_kernel_ms"] < tm["pass_call_ms"], tm
            assert 0 <= tm["density_rescan_ms"] < tm["density_kernel_ms"], tm
    finally:
        ctx.close()


def test_pass_rebuild_fallback_matches_oracle(gpu_lib):
    """Guesses 0.3x too small: every h outgrows its cell, the pass falls back
    to the rebuild loop and repeats the force."""
    d = workloads.lattice_box(18, [1508, 903], jitter=0.2, u=1.0, vel_sigma=0.1)
    d["h0"] = (d["h0"] * 0.3).astype(np.float32)
    t = _inputs(d)
    ctx = gpu_lib.Context(0)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        got, _ = _pass(ctx, t, d)
    finally:
        ctx.close()
    assert got["stats"]["rebuilds"] >= 1
    g = {k: got[k].astype(np.float64) for k in KEYS}
    g["nw"] = None
    r = oracle.run(d)
    e = errors({**g, "nw": r["nw"]}, r)  # nw is not returned by this call
    assert_within(e, TOL32, "pass with rebuild")
    n_f = int(r["npair"].sum())
    assert abs(got["stats"]["interactions_force"] - n_f) <= 1e-5 * n_f + 2


def test_conservation_sums_reproducible(gpu_lib):
    """The per-box sums are each cell's share added per box in a fixed order:
    bit-identical over repeated calls, over the graph-captured pass, and over
    work schedules and cell orders that change only which wavefront takes
    which cell (several boxes, so the per-box leaf ranges are exercised)."""
    import torch
    d = workloads.batched(n_boxes=8, n_min=1000, n_max=8000, side_min=10, side_max=20)
    print("case batched8 cons", flush=True)
    ref = _separate(gpu_lib, d)
    for params in (dict(), dict(schedule=1), dict(cell_order=1), dict(cell_order=2, schedule=1)):
        got = _separate(gpu_lib, d, **params)
        assert np.array_equal(got["cons"], ref["cons"]), params
    t = _inputs(d)
    ctx = gpu_lib.Context(0)
    try:
        ctx.build_cells(t["pos"], t["h0"], d["box_first"], d["box_len"])
        bufs = None
        for rep in range(2):
            got, bufs = _pass(ctx, t, d, bufs)
            assert np.array_equal(got["cons"], ref["cons"]), rep
    finally:
        ctx.close()
    # and the sums are those of the outputs (momentum and energy rates per
    # box), up to the order of FP64 additions
    m = d["mass"].astype(np.float64)
    acc, dudt, vel = ref["acc"].astype(np.float64), ref["dudt"].astype(np.float64), d["vel"].astype(np.float64)
    for b in range(len(d["box_len"])):
        sl = slice(int(d["box_first"][b]), int(d["box_first"][b + 1]))
        mom = (m[sl, None] * acc[sl]).sum(axis=0)
        en = np.sum(m[sl] * (np.einsum("ij,ij->i", vel[sl], acc[sl]) + dudt[sl]))
        s_mom = np.sum(m[sl] * np.abs(acc[sl]).sum(axis=1))
        s_en = np.sum(m[sl] * (np.abs(vel[sl] * acc[sl]).sum(axis=1) + np.abs(dudt[sl])))
        assert np.all(np.abs(ref["cons"][b, :3] - mom) <= 1e-12 * s_mom), b
        assert abs(ref["cons"][b, 3] - en) <= 1e-12 * s_en, b
