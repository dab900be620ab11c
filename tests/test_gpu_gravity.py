"""Near-field gravity on the GPU (sph_gravity_p2p) against the FP64 oracle
(oracle/gravity.py: the pair sum of section 2 Eq. 3 restricted to pairs inside
r_cut, Plummer-softened, with the window S(x) = (1 - x^2)^2).

Error measure: |g_gpu - g_oracle| over the window-free scale
W_i = G sum_j m_j r_ij (r_ij^2 + eps^2)^(-3/2) (the pairs inside r_cut, the
window replaced by its largest value 1). The plain gross sum of the windowed
terms is no scale near the cutoff: there S = (1 - x^2)^2 is a difference of
nearly equal numbers, and FP32 rounding of r^2 / r_cut^2 (a few 1e-7) is a
relative error of ~1e-7 / (1 - x^2) of the term, 6e-4 of a particle whose
only pair sits at x = 0.9993, while the absolute error stays ~1e-7 of the
window-free term. The kernel's positions are FP32 in the cell frame, so a term
also carries ~3 u X / r_ij (u = 6e-8, X the frame scale, up to ~100 r_ij for
the closest pairs of a clump): the error is held at 5e-5 of W_i at worst and
5e-6 at the 99th percentile. A particle without pairs gets exactly 0.
The pair count is decided in FP32 on the GPU and in FP64 in the oracle: the
two may differ only by pairs whose separation lies within a relative 1e-5 of
r_cut, and such a pair moves the sum by (1 - x^2)^2 ~ 4e-10 of its window-free
term (the window's zero slope)."""

import ctypes

import numpy as np
import pytest
from scipy.spatial import cKDTree

import workloads
from oracle import gravity as og

pytestmark = pytest.mark.gpu

TOL = 5e-5      # worst particle, on the window-free scale
TOL_P99 = 5e-6  # 99th percentile
H_MARGIN = 1.26  # the library's default search margin (search radius = margin x h guess)


def _f32(x):
    return np.asarray(x, dtype=np.float32)


def _masses(n, seed):
    rng = np.random.default_rng([1508, 880, seed])
    return _f32(rng.uniform(0.5, 2.0, n) / n)


def _band(pos, rc, L=1.0):
    """Ordered pairs whose separation lies within a relative 1e-5 of rc."""
    t = cKDTree(np.mod(pos, L), boxsize=L)
    hi = t.count_neighbors(t, rc * (1 + 1e-5))
    lo = t.count_neighbors(t, rc * (1 - 1e-5))
    return int(hi - lo)


def _window_free(pos, mass, G, eps, rc, L=1.0, rows=None):
    """W_i (module docstring) of every particle, or of `rows`, from periodic
    tree queries."""
    pos = np.mod(pos, L)
    t = cKDTree(pos, boxsize=L)
    if rows is None:
        pr = t.query_pairs(rc, output_type="ndarray")
        i, j = pr[:, 0], pr[:, 1]
        out = np.zeros(len(pos))
    else:
        nb = t.query_ball_point(pos[rows], rc)
        i = np.concatenate([np.full(len(b), k) for k, b in enumerate(nb)]).astype(np.int64)
        j = np.concatenate([np.asarray(b, dtype=np.int64) for b in nb])
        out = np.zeros(len(rows))
    src = i if rows is None else np.asarray(rows)[i]
    dd = pos[src] - pos[j]
    dd -= L * np.rint(dd / L)
    r = np.linalg.norm(dd, axis=1)
    k = r > 0
    i, j, r = i[k], j[k], r[k]
    w = G * r * (r * r + eps * eps) ** -1.5
    np.add.at(out, i, w * mass[j])
    if rows is None:
        np.add.at(out, j, w * mass[i])
    return out


def _assert_close(acc_g, acc_o, scale, label):
    err = np.linalg.norm(acc_g - acc_o, axis=1)
    has = scale > 0
    rel = err[has] / scale[has]
    worst = float(rel.max()) if has.any() else 0.0
    p99 = float(np.percentile(rel, 99)) if has.any() else 0.0
    print(label, "worst", worst, "p99", p99, flush=True)
    assert worst <= TOL and p99 <= TOL_P99, (label, worst, p99)
    assert np.all(acc_g[~has] == 0.0), label


def _gpu(gpu_lib, d, mass, G, eps, rc, ctx=None):
    import torch
    own = ctx is None
    if own:
        ctx = gpu_lib.Context(0, timing=1)
    try:
        if own:
            ctx.build_cells(torch.from_numpy(d["pos"]).cuda(), torch.from_numpy(d["h0"]).cuda(), d["box_first"],
                            d["box_len"])
        acc, npair = ctx.gravity_p2p(torch.from_numpy(mass).cuda(), G, eps, rc)
        torch.cuda.synchronize()
        return acc.double().cpu().numpy(), npair
    finally:
        if own:
            ctx.close()


def _check_box(acc_g, pos, mass, G, eps, rc, L, label):
    m = mass.astype(np.float64)
    r = og.p2p(pos, m, G, eps, rc, L)
    print(label, "n", len(pos), "pairs", r["npair"], flush=True)
    _assert_close(acc_g, r["acc"], _window_free(pos, m, G, eps, rc, L), label)
    return r["npair"]


@pytest.mark.parametrize("case", ["lattice", "clustered", "batched"])
def test_gravity_matches_oracle(gpu_lib, case):
    if case == "lattice":
        d = workloads.lattice_box(20, [1508, 881], jitter=0.3)
    elif case == "clustered":
        d = workloads.clustered(n_uniform=6000, n_spheres=4, per_sphere=1500, a_range=(0.02, 0.08))
    else:
        d = workloads.batched(n_boxes=5, n_min=1000, n_max=6000, side_min=10, side_max=18)
    n = len(d["pos"])
    mass = _masses(n, 1)
    G, eps = 1.3, 1e-3
    rc = 0.95 * float(d["h0"].min())
    print("case", case, "n", n, "r_cut", rc, flush=True)
    acc, npair = _gpu(gpu_lib, d, mass, G, eps, rc)
    tot, band = 0, 0
    for b in range(len(d["box_len"])):
        s, e = int(d["box_first"][b]), int(d["box_first"][b + 1])
        L = float(d["box_len"][b])
        tot += _check_box(acc[s:e], d["pos"][s:e], mass[s:e], G, eps, rc, L, "%s box %d" % (case, b))
        band += _band(d["pos"][s:e], rc, L)
    assert abs(npair - tot) <= band, (npair, tot, band)


def test_gravity_empty_and_lonely_boxes(gpu_lib):
    """A batch with an empty box and a box of side 2 holding one particle:
    the lonely particle has no pair and gets exactly 0; the other boxes
    match the oracle."""
    a = workloads.lattice_box(12, [1508, 886], jitter=0.25)
    b = workloads.lattice_box(9, [1508, 887], jitter=0.25)
    n1, n2 = len(a["pos"]), len(b["pos"])
    d = {k: np.concatenate([a[k], np.array([[1.3, 0.2, 1.7]]) if k == "pos" else a[k][:1], b[k]])
         for k in ("pos", "vel", "mass", "u", "h0")}
    d["box_first"] = np.array([0, n1, n1, n1 + 1, n1 + 1 + n2], dtype=np.int64)
    d["box_len"] = np.array([1.0, 1.0, 2.0, 1.0])
    mass = _masses(len(d["pos"]), 7)
    rc = 0.95 * float(d["h0"].min())
    acc, npair = _gpu(gpu_lib, d, mass, 1.0, 1e-3, rc)
    assert np.all(acc[n1] == 0.0)
    tot = _check_box(acc[:n1], d["pos"][:n1], mass[:n1], 1.0, 1e-3, rc, 1.0, "box 0")
    tot += _check_box(acc[n1 + 1:], d["pos"][n1 + 1:], mass[n1 + 1:], 1.0, 1e-3, rc, 1.0, "box 3")
    band = _band(d["pos"][:n1], rc) + _band(d["pos"][n1 + 1:], rc)
    assert abs(npair - tot) <= band


def test_gravity_unsoftened_and_at_the_search_radius(gpu_lib):
    """eps = 0 and r_cut just inside the smallest search radius (every pair
    the cells' lists can hold)."""
    d = workloads.lattice_box(16, [1508, 882], jitter=0.2)
    mass = _masses(len(d["pos"]), 2)
    rc = 0.999 * H_MARGIN * float(d["h0"].min())
    acc, npair = _gpu(gpu_lib, d, mass, 0.8, 0.0, rc)
    tot = _check_box(acc, d["pos"], mass, 0.8, 0.0, rc, 1.0, "unsoftened")
    assert abs(npair - tot) <= _band(d["pos"], rc)


def test_gravity_after_a_drift(gpu_lib):
    """The cells kept across a drift: pairs within r_cut of the moved
    positions, and r_cut held below the search radius less twice the drift
    bound."""
    import torch
    d = workloads.lattice_box(18, [1508, 883], jitter=0.2, vel_sigma=1.0)
    n = len(d["pos"])
    mass = _masses(n, 3)
    hmin = float(d["h0"].min())
    vmax = float(np.abs(d["vel"]).max())
    dt = 0.01 * hmin / vmax  # moves every particle by at most 0.0173 hmin
    ctx = gpu_lib.Context(0, timing=1)
    try:
        pos = torch.from_numpy(d["pos"]).cuda()
        ctx.build_cells(pos, torch.from_numpy(d["h0"]).cuda())
        ctx.drift(dt, torch.from_numpy(d["vel"]).cuda(), pos)
        rc = 0.9 * hmin
        acc, npair = _gpu(gpu_lib, d, mass, 1.0, 1e-3, rc, ctx=ctx)
        moved = pos.cpu().numpy()
        tot = _check_box(acc, moved, mass, 1.0, 1e-3, rc, 1.0, "drift")
        assert abs(npair - tot) <= _band(moved, rc)
        assert ctx.timings()["builds"] == 1  # the drift stayed within the cells' margin
        # at the build's search radius the drift leaves the lists short: refused
        with pytest.raises(gpu_lib.SphError) as ei:
            ctx.gravity_p2p(torch.from_numpy(mass).cuda(), 1.0, 1e-3, 0.999 * H_MARGIN * hmin)
        assert ei.value.code == gpu_lib.SPH_E_ARG
    finally:
        ctx.close()


def test_gravity_repeats_bit_for_bit(gpu_lib):
    import torch
    d = workloads.clustered(n_uniform=4000, n_spheres=3, per_sphere=1000)
    mass = torch.from_numpy(_masses(len(d["pos"]), 4)).cuda()
    ctx = gpu_lib.Context(0)
    try:
        ctx.build_cells(torch.from_numpy(d["pos"]).cuda(), torch.from_numpy(d["h0"]).cuda())
        rc = 0.9 * float(d["h0"].min())
        a1, n1 = ctx.gravity_p2p(mass, 1.0, 1e-3, rc)
        a2, n2 = ctx.gravity_p2p(mass, 1.0, 1e-3, rc)
        assert n1 == n2 and torch.equal(a1, a2)
    finally:
        ctx.close()


def test_gravity_errors(gpu_lib):
    import torch
    d = workloads.lattice_box(10, [1508, 884], jitter=0.1)
    n = len(d["pos"])
    mass = torch.from_numpy(_masses(n, 5)).cuda()
    acc = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    ctx = gpu_lib.Context(0)
    try:
        # no cells yet
        rc = gpu_lib.sph_gravity_p2p(ctx.ctx, ctypes.c_void_p(mass.data_ptr()), 1.0, 0.0, 0.01,
                                     ctypes.c_void_p(acc.data_ptr()), None,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == gpu_lib.SPH_E_STATE
        ctx.build_cells(torch.from_numpy(d["pos"]).cuda(), torch.from_numpy(d["h0"]).cuda())
        hmin = float(d["h0"].min())
        for G, eps, rcut in ((1.0, -1e-3, 0.5 * hmin), (float("nan"), 0.0, 0.5 * hmin), (1.0, 0.0, 0.0),
                             (1.0, 0.0, 1.01 * H_MARGIN * hmin)):
            with pytest.raises(gpu_lib.SphError) as ei:
                ctx.gravity_p2p(mass, G, eps, rcut)
            assert ei.value.code == gpu_lib.SPH_E_ARG, (G, eps, rcut)
        bad = mass.clone()
        bad[n // 2] = 0.0
        with pytest.raises(gpu_lib.SphError) as ei:
            ctx.gravity_p2p(bad, 1.0, 0.0, 0.5 * hmin)
        assert ei.value.code == gpu_lib.SPH_E_ARG
        # the context still works after the refusals
        a, npair = ctx.gravity_p2p(mass, 1.0, 0.0, 0.5 * hmin)
        assert npair > 0 and bool(torch.isfinite(a).all())
    finally:
        ctx.close()


def test_gravity_full_batched_sampled(gpu_lib):
    """The batched set at full size (256 boxes, 8k to 64k particles each),
    launched as the benchmark launches it; sampled rows of three boxes
    against the oracle's row sums."""
    import torch
    d = workloads.make("batched")
    n = len(d["pos"])
    mass = _masses(n, 6)
    rc = 0.95 * float(d["h0"].min())
    print("batched full n", n, "r_cut", rc, flush=True)
    acc, npair = _gpu(gpu_lib, d, mass, 1.0, 1e-3, rc)
    rng = np.random.default_rng([1508, 885])
    for b in (0, 101, 255):
        s, e = int(d["box_first"][b]), int(d["box_first"][b + 1])
        rows = np.concatenate([[0, e - s - 1], rng.choice(e - s, 150, replace=False)])
        m = mass[s:e].astype(np.float64)
        L = float(d["box_len"][b])
        r = og.p2p_rows(d["pos"][s:e], m, 1.0, 1e-3, rc, rows, L)
        _assert_close(acc[s + rows], r["acc"], _window_free(d["pos"][s:e], m, 1.0, 1e-3, rc, L, rows),
                      "box %d" % b)
    assert npair > 0 and np.isfinite(acc).all()
