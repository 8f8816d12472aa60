"""Pins of the oracle's reflective walls and of its classical (Zhang-Xia-Shu)
decomposition, against what the paper and the mathematics fix: the printed ZXS CFL
numbers (tab:2019), the Fig. 1744 ratio ranges, a hand-derived closed form of the
classical P2 limiter vector u*, positivity (Sec. 4.4), conservation at walls, the
method of images and the rotation-invariance test of Example EulerImp."""

import math
import os

import numpy as np
import pytest

import oracle
from synth import mesh as smesh
from synth import problems, workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_zxs():
    rows = []
    for line in open(os.path.join(GOLD, "tab2019_cfl.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, k, val, nodes, form = line.split()
        if name.endswith("_zxs"):
            rows.append((name[:-4], int(k), float(val), form))
    return rows


def _one_cell(v):
    return smesh.Mesh(xy=np.asarray(v, float), tri=np.array([[0, 1, 2]], np.int32))


def test_zxs_cfl_numbers_of_table_2019():
    """tab:2019, classical rows: C^ZXS_{K,k} on the equilateral and the right isosceles
    cell, from the oracle's per-cell C|K| with decomposition='zxs'."""
    s2 = math.sqrt(2.0)
    cells = {"equilateral": [[0, 0], [1, 0], [0.5, math.sqrt(3) / 2]],
             "right_isosceles": [[0, 0], [s2 / 2, 0], [0, s2 / 2]]}
    rows = _golden_zxs()
    assert len(rows) == 4
    for name, k, val, form in rows:
        o = oracle.Oracle(_one_cell(cells[name]), k, decomposition="zxs")
        a = o.mesh_arrays()
        c = a["ck"][0] / a["area"][0]
        assert abs(c - eval(form, {"sqrt": math.sqrt})) < 1e-15
        assert abs(c - val) < 5e-5
        assert a["minck"] == a["ck"].min()


def test_zxs_over_dcw_ratio_within_fig1744_ranges():
    """Fig. 1744: per cell, C^DCW/C^ZXS lies in [2, 3] (P1) and [3.8038, 4.5] (P2); on a
    Delaunay mesh the ranges are met cell by cell by the oracle's own tables."""
    m, _, _ = workloads.quadrant_delaunay(n_cells=3000, seed=31)
    for k, lo, hi in ((1, 2.0, 3.0), (2, 3.8038, 4.5)):
        d = oracle.Oracle(m, k).mesh_arrays()
        z = oracle.Oracle(m, k, decomposition="zxs").mesh_arrays()
        r = d["ck"] / z["ck"]
        assert r.min() >= lo - 1e-4 and r.max() <= hi + 1e-4, (k, r.min(), r.max())


def test_classical_p2_ustar_closed_form_and_range():
    """Sec. 4.2 weights w_i = 2 w1^GL/3 = 1/9 (L = 3) and the exact edge averages of the
    basis (edges 0, 1, 2 sum to 3, 0, 0, 8/3, 0, 5/3 for Psi_0..5, worked by hand) give
    u* = u_0 - 4/9 u_3 - 5/18 u_5.  u* is the mean of the decomposition's internal node
    values, so it lies within the polynomial's range over the cell."""
    m, _, _ = workloads.quadrant_delaunay(n_cells=300, seed=32)
    o = oracle.Oracle(m, 2, decomposition="zxs")
    rng = np.random.default_rng(5)
    u = rng.normal(size=(4, 6, m.n_cell))
    vals = o.limiter_node_values(u)
    closed = u[:, 0] - 4.0 / 9.0 * u[:, 3] - 5.0 / 18.0 * u[:, 5]     # (4, nc)
    for t in (9, 10):
        assert np.abs(vals[:, t, :].T - closed).max() < 1e-13 * np.abs(u).max()
    # the range over a dense barycentric sampling of the cell
    g = np.linspace(0.0, 1.0, 41)
    X, E = np.meshgrid(g, g)
    keep = X + E <= 1.0
    P = np.array([oracle.basis(x, e)[0] for x, e in zip(X[keep], E[keep])])   # (npts, 6)
    vals_pts = np.einsum("vlc,pl->vcp", u, P)
    assert np.all(closed >= vals_pts.min(axis=2) - 1e-12)
    assert np.all(closed <= vals_pts.max(axis=2) + 1e-12)
    # the optimal decomposition's slots 9, 10 are its two internal nodes instead
    vd = oracle.Oracle(m, 2).limiter_node_values(u)
    assert np.abs(vd[:, 9, :].T - closed).max() > 1e-3


def test_classical_p1_node_set_is_the_edge_points():
    """Classical P1 decomposition: no internal nodes (the edge weights sum to one), so
    the node set is the 6 edge Gauss points (the two trailing slots repeat 0 and 1)."""
    m, _, _ = workloads.quadrant_delaunay(n_cells=200, seed=33)
    rng = np.random.default_rng(6)
    u = rng.normal(size=(4, 3, m.n_cell))
    z = oracle.Oracle(m, 1, decomposition="zxs").limiter_node_values(u)
    d = oracle.Oracle(m, 1).limiter_node_values(u)
    assert np.array_equal(z[:, :6], d[:, :6])
    assert np.array_equal(z[:, 6], z[:, 0]) and np.array_equal(z[:, 7], z[:, 1])


@pytest.mark.parametrize("k", [1, 2])
def test_classical_limiter_positivity(k):
    """Sec. 4.4, classical branch: after the limiter rho >= eps1 and E(u) >= eps2 at the
    edge points and at u* (P2); averages unchanged."""
    m, kind, p = workloads.quadrant_delaunay(n_cells=500, seed=34)
    o = oracle.Oracle(m, k, decomposition="zxs")
    o.init_problem(kind, p)
    u = o.state(0)
    rng = np.random.default_rng(k + 10)
    u[:, 1:, :] += 0.6 * rng.normal(size=u[:, 1:, :].shape) * np.abs(u[:, :1, :])
    assert (o.limiter_node_values(u)[..., 0] < 0).any()
    lim, bad = o.limit(u)
    assert bad == 0 and np.array_equal(lim[:, 0, :], u[:, 0, :])
    v = o.limiter_node_values(lim)
    rho = v[..., 0]
    e = v[..., 3] - 0.5 * (v[..., 1] ** 2 + v[..., 2] ** 2) / rho
    assert rho.min() >= 1e-13 * (1 - 1e-9) - 1e-15
    assert e.min() >= 1e-13 * (1 - 1e-9) - 1e-14


def test_classical_time_step_ratio():
    """Sec. 6: Delta t = C_SSP/alpha min_K C_{K,k}|K| for both decompositions; from the
    same state the two first steps differ exactly by the ratio of the minima."""
    m, kind, p = workloads.quadrant_delaunay(n_cells=800, seed=35)
    for k in (1, 2):
        d = oracle.Oracle(m, k)
        z = oracle.Oracle(m, k, decomposition="zxs")
        d.init_problem(kind, p)
        z.init_problem(kind, p)
        sd, sz = d.scalars(), z.scalars()
        assert sd["alpha"] > 0
        ratio = sd["dt"] / sz["dt"]
        assert abs(ratio - sd["minck"] / sz["minck"]) < 1e-14 * ratio
        assert (2.0 if k == 1 else 3.8) <= ratio <= (3.0 if k == 1 else 4.5)


# ----------------------------------------------------------------------------- walls

def _box_walls(m, lo=0.0, hi=1.0):
    return workloads.wall_tags(m, lambda x, y: (x == lo) | (x == hi) | (y == lo) | (y == hi))


@pytest.mark.parametrize("k", [1, 2])
def test_walls_conserve_mass_and_energy(k):
    """A reflective wall has zero mass and energy flux (the LF flux of the mirrored
    state), so with walls all round the domain totals are conserved to round-off;
    momentum is not (the wall pressure)."""
    m, kind, p = workloads.quadrant_delaunay(n_cells=600, seed=36)
    m.edge_bc = _box_walls(m)
    o = oracle.Oracle(m, k)
    o.init_problem(kind, p)
    area = o.mesh_arrays()["area"]
    tot0 = (o.state(0)[:, 0, :] * area).sum(axis=1)
    for _ in range(5):
        assert o.step() == 0
    tot = (o.state(0)[:, 0, :] * area).sum(axis=1)
    assert abs(tot[0] - tot0[0]) < 1e-14 * abs(tot0[0]) * 20
    assert abs(tot[3] - tot0[3]) < 1e-14 * abs(tot0[3]) * 20
    # the transmissive run of the same data loses mass through the boundary
    m.edge_bc = None
    t = oracle.Oracle(m, k)
    t.init_problem(kind, p)
    for _ in range(5):
        assert t.step() == 0
    tt = (t.state(0)[:, 0, :] * area).sum(axis=1)
    assert abs(tt[0] - tot0[0]) > 1e3 * abs(tot[0] - tot0[0])


def _mirrored(m):
    """The mesh together with its mirror image in y = 0 (vertices on y = 0 shared)."""
    on = m.xy[:, 1] == 0.0
    ids = np.where(~on)[0]
    remap = np.arange(m.n_vert)
    remap[ids] = m.n_vert + np.arange(len(ids))
    xy = np.concatenate([m.xy, m.xy[ids] * np.array([1.0, -1.0])])
    tri = np.concatenate([m.tri, remap[m.tri]]).astype(np.int32)
    return smesh.Mesh(xy=xy, tri=tri)


@pytest.mark.parametrize("k", [1, 2])
def test_wall_is_the_method_of_images(k):
    """Reflective wall on y = 0 versus the mirror-symmetric problem on the doubled
    domain (mirrored mesh, m2 reversed): every step of the scheme without the OE filter
    (whose jump at a wall is zero in the reading both codes take, while the mirror has a jump)
    maps the one onto the other, so the upper halves agree to round-off."""
    half, _, _ = workloads.quadrant_delaunay(n_cells=700, seed=37)
    full = _mirrored(half)
    half.edge_bc = workloads.wall_tags(half, lambda x, y: y == 0.0)
    assert half.edge_bc.sum() > 10
    # piecewise-constant data with flow towards the wall
    qp = problems.quadrant_riemann_params(seed=37)
    src = oracle.Oracle(half, k)
    src.init_problem(problems.PROBLEM_QUADRANT, qp)
    u = src.state(0)
    u[:, 1:, :] = 0.0
    u[2, 0, :] = -np.abs(u[2, 0, :]) - 0.1 * u[0, 0, :]
    mir = u.copy()
    mir[2] = -mir[2]
    uf = np.concatenate([u, mir], axis=2)
    a = oracle.Oracle(half, k, oe=False)
    b = oracle.Oracle(full, k, oe=False)
    a.init_modal(u)
    b.init_modal(uf)
    assert a.scalars()["dt"] == pytest.approx(b.scalars()["dt"], rel=1e-14)
    for _ in range(4):
        assert a.step() == 0 and b.step() == 0
    ua, ub = a.state(0)[:, 0, :], b.state(0)[:, 0, :half.n_cell]
    scale = np.abs(ua).max(axis=1, keepdims=True)
    assert (np.abs(ua - ub) / scale).max() < 1e-12
    # and the lower half is the mirror image of the upper one
    low = b.state(0)[:, 0, half.n_cell:]
    assert np.abs(low[2] + ub[2]).max() < 1e-12 * scale[2, 0]
    assert np.abs(ua[2] - u[2, 0]).max() > 1e-4 * scale[2, 0]     # the wall did act


def test_tags_follow_input_vertex_order():
    """A tag names the edge opposite input vertex i; a clockwise input cell is oriented
    by swapping its vertices 1 and 2, and its tags move with them."""
    m, kind, p = workloads.quadrant_delaunay(n_cells=300, seed=38)
    tags = _box_walls(m)
    flip = m.tri.copy()
    flip[::2] = flip[::2][:, [0, 2, 1]]                      # every other cell clockwise
    ftags = tags.copy()
    ftags[::2] = ftags[::2][:, [0, 2, 1]]
    ma = smesh.Mesh(xy=m.xy, tri=m.tri, edge_bc=tags)
    mb = smesh.Mesh(xy=m.xy, tri=flip, edge_bc=ftags)
    out = []
    for mm in (ma, mb):
        o = oracle.Oracle(mm, 2)
        o.init_problem(kind, p)
        for _ in range(2):
            assert o.step() == 0
        out.append(o.state(0))
    assert np.array_equal(out[0], out[1])


def ri_errors(a, b):
    """Example EulerImp: max-norm differences of the cell averages of rho, v1, v2, p,
    with b's velocity turned back by M^{-1}."""
    c = math.sqrt(2.0) / 2.0
    def prim(u):
        rho, m1, m2, E = u[0, 0], u[1, 0], u[2, 0], u[3, 0]
        v1, v2 = m1 / rho, m2 / rho
        return rho, v1, v2, 0.4 * (E - 0.5 * rho * (v1 * v1 + v2 * v2))
    ra, v1a, v2a, pa = prim(a)
    rb, v1b, v2b, pb = prim(b)
    v1t, v2t = c * v1b - c * v2b, c * v1b + c * v2b
    return np.array([np.abs(ra - rb).max(), np.abs(v1a - v1t).max(), np.abs(v2a - v2t).max(),
                     np.abs(pa - pb).max()])


def test_implosion_rotation_invariance_ri_vs_cw():
    """Example EulerImp: the implosion quadrant with reflective walls and its copy turned
    clockwise by pi/4.  RI-OEDG keeps the two at round-off; the component-wise OE does
    not."""
    m, kind, p = workloads.implosion(n_cells=900, seed=39)
    mr, kindr, pr = workloads.implosion(n_cells=900, seed=39, rotate=True)
    errs = {}
    for mode in (0, 1):
        a = oracle.Oracle(m, 2, oe_mode=mode)
        b = oracle.Oracle(mr, 2, oe_mode=mode)
        a.init_problem(kind, p)
        b.init_problem(kindr, pr)
        for _ in range(8):
            assert a.step() == 0 and b.step() == 0
        errs[mode] = ri_errors(a.state(0), b.state(0))
    assert errs[0].max() < 1e-12, errs
    assert errs[1].max() > 1e3 * max(errs[0].max(), 1e-15), errs
