"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact integrals,
textbook quadrature rules, brute force, printed table values (tests/golden/), the
paper's invariance theorems, conservation and convergence order.
"""

import math
import os

import numpy as np
import pytest

import oracle
from synth import mesh as smesh
from synth import problems, workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")
MONO = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


def ref_moment(a, b):
    """Exact integral of xi^a eta^b over the reference triangle (area 1/2)."""
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


def basis_monomials():
    """Monomial coefficients of the oracle's Psi_0..5, recovered from point values."""
    rng = np.random.default_rng(0)
    pts = rng.random((20, 2)) * 0.5
    V = np.array([[x ** a * y ** b for a, b in MONO] for x, y in pts])
    P = np.array([oracle.basis(x, y)[0] for x, y in pts])
    C, *_ = np.linalg.lstsq(V, P, rcond=None)
    return C.T   # (6 basis, 6 monomials)


def poly_product_integral(c1, c2):
    tot = 0.0
    for i, (a1, b1) in enumerate(MONO):
        for j, (a2, b2) in enumerate(MONO):
            tot += c1[i] * c2[j] * ref_moment(a1 + a2, b1 + b2)
    return tot


# ----------------------------------------------------------------------------- basis, mass

def test_basis_orthogonal_and_mass():
    """Basis of eq. basisfunc is L2-orthogonal; a_K^(l)/|K| = 1, 2/3, 1/2, 16/15, 4/9, 1/3."""
    C = basis_monomials()
    G = np.array([[poly_product_integral(C[i], C[j]) for j in range(6)] for i in range(6)])
    expect = np.array([1, 2 / 3, 1 / 2, 16 / 15, 4 / 9, 1 / 3]) / 2.0   # reference area 1/2
    assert np.allclose(np.diag(G), expect, atol=1e-13)
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-13
    # the oracle's per-cell mass a_K^(l) agrees with |K| times the ratios
    m, _, _ = workloads.periodic_vortex(n=4)
    o = oracle.Oracle(m, 2)
    M = o.mass()
    area = o.mesh_arrays()["area"]
    assert np.allclose(M / area[:, None], expect * 2, rtol=1e-14, atol=0)


def test_basis_gradients_match_difference_quotients():
    for xi, eta in [(0.1, 0.2), (0.3, 0.6), (0.7, 0.05)]:
        p, dx, de = oracle.basis(xi, eta)
        h = 1e-6
        px = (oracle.basis(xi + h, eta)[0] - oracle.basis(xi - h, eta)[0]) / (2 * h)
        pe = (oracle.basis(xi, eta + h)[0] - oracle.basis(xi, eta - h)[0]) / (2 * h)
        assert np.allclose(dx, px, atol=1e-7) and np.allclose(de, pe, atol=1e-7)


# ----------------------------------------------------------------------------- quadrature

@pytest.mark.parametrize("which,deg", [(0, 2), (1, 4), (2, 6)])
def test_triangle_rules_exact(which, deg):
    """App. A rules integrate every monomial up to their degree exactly."""
    B, w = oracle.quadrature(which)
    assert np.all(B > 0) and np.allclose(B.sum(axis=1), 1.0, atol=1e-15)
    tol = 1e-15 if which < 2 else 5e-15   # the 12-point rule is used as printed (15 digits)
    assert abs(w.sum() - 1.0) <= tol
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            q = np.sum(w * B[:, 1] ** a * B[:, 2] ** b)
            assert abs(q - 2.0 * ref_moment(a, b)) < 4 * tol, (a, b)
    # the rule one degree higher is not exact (the degree is sharp)
    errs = [abs(np.sum(w * B[:, 1] ** a * B[:, 2] ** (deg + 1 - a)) - 2 * ref_moment(a, deg + 1 - a))
            for a in range(deg + 2)]
    assert max(errs) > 1e-6


def test_six_point_closed_forms_match_printed_table():
    """The closed forms used for tab:4th reproduce the printed 15-digit values."""
    printed = np.loadtxt(os.path.join(GOLD, "tab4th_quadrature.txt"))
    B, w = oracle.quadrature(1)
    assert np.abs(B - printed[:, :3]).max() < 1e-15
    assert np.abs(w - printed[:, 3]).max() < 2e-15


@pytest.mark.parametrize("which,Q", [(3, 2), (4, 3)])
def test_edge_gauss_exact(which, Q):
    s, w = oracle.quadrature(which)
    assert abs(w.sum() - 1) < 1e-15 and np.all((s > 0) & (s < 1))
    for p in range(2 * Q):
        assert abs(np.sum(w * s ** p) - 1.0 / (p + 1)) < 1e-15


# ----------------------------------------------------------------------------- mesh

def brute_force_neighbours(tri):
    n = len(tri)
    nbr = -np.ones((n, 3), int)
    nbe = -np.ones((n, 3), int)
    for c in range(n):
        for i in range(3):
            e = {tri[c][(i + 1) % 3], tri[c][(i + 2) % 3]}
            for d in range(n):
                if d == c:
                    continue
                for j in range(3):
                    if {tri[d][(j + 1) % 3], tri[d][(j + 2) % 3]} == e:
                        nbr[c, i], nbe[c, i] = d, j
    return nbr, nbe


@pytest.mark.parametrize("kind", ["periodic", "delaunay"])
def test_edge_table_brute_force(kind):
    m = smesh.periodic_jittered_grid(n=5, seed=9) if kind == "periodic" else \
        smesh.poisson_delaunay(150, seed=5)
    o = oracle.Oracle(m, 1)
    a = o.mesh_arrays()
    nbr, nbe = brute_force_neighbours(a["tri"].tolist())
    assert np.array_equal(nbr, a["nbr"]) and np.array_equal(nbe, a["nbe"])
    # reciprocity, closed polygons, Euler characteristic
    for c in range(m.n_cell):
        for i in range(3):
            if a["nbr"][c, i] >= 0:
                assert a["nbr"][a["nbr"][c, i], a["nbe"][c, i]] == c
        s = (a["len"][c][:, None] * a["nrm"][c]).sum(axis=0)
        assert np.abs(s).max() < 1e-14
    n_edges = (3 * m.n_cell + (a["nbr"] < 0).sum()) // 2
    chi = m.n_vert - n_edges + m.n_cell
    assert chi == (0 if kind == "periodic" else 1)
    assert np.all(a["area"] > 0)


# ----------------------------------------------------------------------------- decomposition

def random_triangles(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.random((n, 3, 2))
    det = (v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1]) - (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1])
    v[det < 0] = v[det < 0][:, [0, 2, 1]]
    keep = np.abs(det) > 1e-3
    return v[keep]


def _quad_poly(c, x, y):
    return c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y


@pytest.mark.parametrize("k", [1, 2])
def test_decomposition_exact_and_feasible(k):
    """Def. 980: the decomposition of eq. 1040 (P1) / eq. 1139 (P2) reproduces cell
    averages of every P^k polynomial, with positive weights summing to one and
    internal nodes inside K.  Cell average by the edge-midpoint rule, edge averages
    by Simpson's rule (both exact for quadratics)."""
    rng = np.random.default_rng(k)
    worst = 0.0
    for v in random_triangles(1500, 10 + k):
        w, nodes, nw, cd, perm = oracle.decompose(k, v)
        lens = np.array([np.linalg.norm(v[(i + 2) % 3] - v[(i + 1) % 3]) for i in range(3)])
        assert np.all(np.diff(lens[perm]) <= 0)
        assert np.all(w > 0) and np.all(nw >= 0)
        assert abs(w.sum() + (nw.sum() if k == 2 else nw[0]) - 1.0) < 1e-14
        # internal nodes strictly inside (barycentric coordinates > 0)
        T = np.array([v[1] - v[0], v[2] - v[0]]).T
        for s in range(2 if k == 2 else 1):
            lam = np.linalg.solve(T, nodes[s] - v[0])
            bary = np.array([1 - lam.sum(), lam[0], lam[1]])
            assert np.all(bary > -1e-12)
        for _ in range(3):
            c = rng.normal(size=6)
            if k == 1:
                c[3:] = 0
            mids = [(v[i] + v[(i + 1) % 3]) / 2 for i in range(3)]
            avg = np.mean([_quad_poly(c, *p) for p in mids])
            rhs = 0.0
            for r in range(3):
                e = perm[r]
                a, b = v[(e + 1) % 3], v[(e + 2) % 3]
                eavg = (_quad_poly(c, *a) + 4 * _quad_poly(c, *((a + b) / 2)) + _quad_poly(c, *b)) / 6
                rhs += w[r] * eavg
            if k == 1:
                rhs += nw[0] * _quad_poly(c, *nodes[0])
            else:
                rhs += nw[0] * _quad_poly(c, *nodes[0]) + nw[1] * _quad_poly(c, *nodes[1])
            worst = max(worst, abs(avg - rhs) / (1 + abs(avg)))
        # C_BP = min_i w_i / l_i equals the closed form C^DCW (eq. 1692 / eq. 1713)
        assert abs(np.min(w / lens[perm]) - cd) < 1e-14 * cd * 10
    assert worst < 1e-13


def test_p1_node_on_shortest_edge():
    """The P1 internal node of eq. 1040 lies on e^(3), between v1 and v2 (Sec. 4.4 remark)."""
    for v in random_triangles(300, 3):
        w, nodes, nw, cd, perm = oracle.decompose(1, v)
        v1, v2 = v[perm[0]], v[perm[1]]
        d = nodes[0] - v1
        e = v2 - v1
        cross = d[0] * e[1] - d[1] * e[0]
        t = d @ e / (e @ e)
        assert abs(cross) < 1e-13 and -1e-14 <= t <= 1 + 1e-14


def _golden_tab2019():
    rows = []
    for line in open(os.path.join(GOLD, "tab2019_cfl.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, k, val, nodes, form = line.split()
        rows.append((name, int(k), float(val), int(nodes), form))
    return rows


def test_table_2019_cfl_numbers():
    """tab:2019: optimal BP CFL numbers on the two example cells."""
    s2 = math.sqrt(2.0)
    cells = {"equilateral": np.array([[0, 0], [1, 0], [0.5, math.sqrt(3) / 2]]),
             "right_isosceles": np.array([[0, 0], [s2 / 2, 0], [0, s2 / 2]])}
    for name, k, val, nnodes, form in _golden_tab2019():
        exact = eval(form, {"sqrt": math.sqrt})
        assert abs(exact - val) < 5e-5, name
        if name.endswith("_zxs"):
            continue
        v = cells[name]
        w, nodes, nw, cd, perm = oracle.decompose(k, v)
        assert abs(cd - exact) < 1e-15
        # number of distinct internal nodes with positive weight
        if k == 1:
            n_int = int(nw[0] > 1e-14)
        else:
            n_int = 1 if np.linalg.norm(nodes[0] - nodes[1]) < 1e-12 else 2
        assert n_int == nnodes, (name, k)


def test_fig1744_ratio_ranges():
    """Fig. 1744 caption: ranges of C^DCW/C^ZXS and C^DCW/C^CS over all triangles."""
    rng = np.random.default_rng(7)
    rows = [l.split() for l in open(os.path.join(GOLD, "fig1744_ranges.txt")) if l[0] != "#"]
    # normalised shapes 1 = l1 >= l2 >= l3, l2 + l3 >= 1; bias towards the extremes
    n = 20000
    l2 = np.concatenate([rng.uniform(0.5, 1.0, n), np.full(50, 1.0), np.full(50, 0.5 + 1e-6),
                         rng.uniform(0.999, 1.0, 50)])
    l3 = np.empty_like(l2)
    l3[:n] = rng.uniform(1 - l2[:n], l2[:n])
    l3[n:n + 50] = 1.0
    l3[n + 50:n + 100] = 0.5 + 1e-6
    l3[n + 100:] = 1 - l2[n + 100:] + 1e-9
    ratios = {("dcw_zxs", 1): [], ("dcw_cs", 1): [], ("dcw_zxs", 2): [], ("dcw_cs", 2): []}
    for a, b in zip(l2, l3):
        # triangle with edges l1 = 1 (opposite v0), l2 (opposite v1), l3 (opposite v2)
        x = (b * b + 1 - a * a) / 2
        y = math.sqrt(max(b * b - x * x, 0.0))
        v = np.array([[x, y], [0.0, 0.0], [1.0, 0.0]])
        if y < 1e-9:
            continue
        lbar = (1 + a + b) / 3
        for k in (1, 2):
            cd = oracle.decompose(k, v)[3]
            zxs = 1 / (9 * lbar) if k == 1 else 1 / (27 * lbar)
            ratios[("dcw_zxs", k)].append(cd / zxs)
            ratios[("dcw_cs", k)].append(cd / (1 / 6.0))
    for name, k, lo, hi in rows:
        r = np.array(ratios[(name, int(k))])
        lo, hi = float(lo), float(hi)
        assert r.min() >= lo - 1e-4 and r.max() <= hi + 1e-4, (name, k, r.min(), r.max())
        assert r.min() <= lo + 2e-3 and r.max() >= hi - 2e-3, (name, k, r.min(), r.max())


# ----------------------------------------------------------------------------- residual

def constant_state(nc, nm, rho=1.3, u=0.4, v=-0.7, p=0.9, gamma=1.4):
    s = np.zeros((4, nm, nc))
    s[0, 0] = rho
    s[1, 0] = rho * u
    s[2, 0] = rho * v
    s[3, 0] = p / (gamma - 1) + 0.5 * rho * (u * u + v * v)
    return s


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("kind", ["periodic", "delaunay"])
def test_free_stream(k, kind):
    """A constant state is an exact steady solution: L(u) = 0 (eq. DGSystem:Dis with the
    divergence theorem), and OE/limiter leave it unchanged."""
    m = smesh.periodic_jittered_grid(n=6, seed=3) if kind == "periodic" else \
        smesh.poisson_delaunay(300, seed=6)
    o = oracle.Oracle(m, k)
    u = constant_state(m.n_cell, o.nm)
    L = o.residual(u, 2.0)
    # round-off only: terms of size |F| |grad Psi| l cancel, divided by a_K ~ |K|
    assert np.abs(L).max() < 2e-11
    o.init_modal(u)
    o.step()
    assert np.abs(o.state(0) - u).max() < 1e-13


def test_periodic_conservation():
    """Periodic mesh: OE keeps mode 0 (eq. OE:m0), the limiter keeps averages, and the
    LF fluxes cancel, so sum |K| ubar_K is conserved to round-off."""
    m, kind, p = workloads.periodic_vortex(n=8)
    o = oracle.Oracle(m, 2)
    o.init_problem(kind, p)
    area = o.mesh_arrays()["area"]
    tot0 = (o.state(0)[:, 0, :] * area).sum(axis=1)
    for _ in range(5):
        assert o.step() == 0
    tot = (o.state(0)[:, 0, :] * area).sum(axis=1)
    assert np.abs(tot - tot0).max() < 1e-12 * np.abs(tot0).max()


# ----------------------------------------------------------------------------- OE

def test_oe_keeps_mode0_and_identity_cases():
    m, kind, p = workloads.quadrant_delaunay(n_cells=600, seed=4)
    o = oracle.Oracle(m, 2)
    o.init_problem(kind, p)
    u = o.state(0)
    rng = np.random.default_rng(1)
    u[:, 1:, :] += 0.05 * rng.normal(size=u[:, 1:, :].shape)
    f = o.oe(u, 0.01)
    assert np.array_equal(f[:, 0, :], u[:, 0, :])            # eq. OE:m0, bitwise
    assert np.all(np.abs(f[:, 1:, :]) <= np.abs(u[:, 1:, :]))  # pure damping
    assert np.array_equal(o.oe(u, 0.0), u)                    # tau = 0
    c = constant_state(m.n_cell, 6)
    assert np.array_equal(o.oe(c, 0.5), c)                    # zero-norm branch


@pytest.mark.parametrize("k", [1, 2])
def test_oe_hand_computed_sigma(k):
    """Two cells forming the unit square, rho = 1 | 2, p = 1, v = 0: the only nonzero
    damping coefficient is sigma^0 = beta/h * A^{k,0}/||rho - 1.5|| * |jump| with
    beta = sqrt(1.4) (the larger sound speed), h = 1/sqrt(2), norm 0.5, jump 1."""
    m = smesh.Mesh(xy=np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float),
                   tri=np.array([[0, 1, 2], [0, 2, 3]], np.int32))
    o = oracle.Oracle(m, k)
    nm = o.nm
    u = np.zeros((4, nm, 2))
    u[0, 0] = [1.0, 2.0]
    u[3, 0] = 1.0 / 0.4
    eps = 1e-10
    u[0, 1, 0] = eps          # a tiny observable mode in cell 0
    dt = 0.01
    f = o.oe(u, dt)
    A0 = 1.0 if k == 1 else 1.0 / 3.0
    sigma0 = math.sqrt(1.4) / (1 / math.sqrt(2)) * A0 / 0.5 * 1.0
    fac = f[0, 1, 0] / eps
    assert abs(fac - math.exp(-dt * sigma0)) < 1e-7


def _step_state(m, k, u, nsteps=1, oe_mode=0, bp=True):
    o = oracle.Oracle(m, k, oe_mode=oe_mode, bp=bp)
    o.init_modal(u)
    for _ in range(nsteps):
        assert o.step() == 0
    return o.state(0), o.scalars()


def test_scale_invariance_bitwise():
    """Sec. 2.4: doubling the state doubles every stage exactly (the limiter floors are
    inactive on this smooth problem)."""
    m, kind, p = workloads.periodic_vortex(n=8)
    o = oracle.Oracle(m, 2)
    o.init_problem(kind, p)
    u = o.state(0)
    a, sa = _step_state(m, 2, u, 2)
    b, sb = _step_state(m, 2, 2 * u, 2)
    assert np.array_equal(b, 2 * a) and sa["dt"] == sb["dt"]


def test_evolution_invariance_bitwise():
    """Sec. 2.4: (rho, 2 m, 4 E) moves twice as fast; with Delta t halved every stage
    maps exactly, so the step reproduces (rho, 2 m, 4 E) of the original step."""
    m, kind, p = workloads.periodic_vortex(n=8)
    o = oracle.Oracle(m, 2)
    o.init_problem(kind, p)
    u = o.state(0)
    T = np.array([1.0, 2.0, 2.0, 4.0])[:, None, None]
    a, sa = _step_state(m, 2, u, 2)
    b, sb = _step_state(m, 2, T * u, 2)
    assert np.array_equal(b, T * a)
    assert sb["dt"] * 2 == sa["dt"] and sb["t"] * 2 == sa["t"]


def rotate_mesh(m, phi, centre):
    c, s = math.cos(phi), math.sin(phi)
    R = np.array([[c, -s], [s, c]])
    xy = (m.xy - centre) @ R.T + centre
    cxy = None
    if m.cell_xy is not None:
        cxy = ((m.cell_xy.reshape(-1, 3, 2) - centre) @ R.T + centre).reshape(-1, 6)
    return smesh.Mesh(xy=xy, tri=m.tri.copy(), cell_xy=cxy, periodic=m.periodic), R


def rotate_state(u, R):
    out = u.copy()
    out[1] = R[0, 0] * u[1] + R[0, 1] * u[2]
    out[2] = R[1, 0] * u[1] + R[1, 1] * u[2]
    return out


def ri_error(a, b, R):
    """max-norm of the difference of cell averages after rotating momentum back."""
    back = rotate_state(b, R.T)
    return np.abs(back[:, 0, :] - a[:, 0, :]).max()


def test_rotation_invariance_ri_vs_cw():
    """Sec. 3.3 theorem and Example EulerImp: RI-OEDG results on a mesh rotated by pi/4
    agree to round-off; component-wise OE (the negative control) does not."""
    m, kind, p = workloads.quadrant_delaunay(n_cells=800, seed=8)
    o = oracle.Oracle(m, 2)
    o.init_problem(kind, p)
    u = o.state(0)
    mr, R = rotate_mesh(m, math.pi / 4, np.array([0.5, 0.5]))
    ur = rotate_state(u, R)
    errs = {}
    for mode in (0, 1):
        a, _ = _step_state(m, 2, u, 6, oe_mode=mode)
        b, _ = _step_state(mr, 2, ur, 6, oe_mode=mode)
        errs[mode] = ri_error(a, b, R)
    assert errs[0] < 1e-12, errs
    assert errs[1] > 1e3 * max(errs[0], 1e-15), errs


def test_quarter_turn_rotation():
    m, kind, p = workloads.periodic_vortex(n=8)
    o = oracle.Oracle(m, 1)
    o.init_problem(kind, p)
    u = o.state(0)
    mr, R = rotate_mesh(m, math.pi / 2, np.array([0.0, 0.0]))
    R = np.round(R)
    a, _ = _step_state(m, 1, u, 3)
    b, _ = _step_state(mr, 1, rotate_state(u, R), 3)
    assert ri_error(a, b, R) < 1e-13


# ----------------------------------------------------------------------------- limiter

def test_limiter_positivity_average_and_idempotence():
    """Sec. 4.4: after the limiter, rho >= eps1 and E - |m|^2/(2 rho) >= eps2 at every node
    of the decomposition; cell averages are unchanged; a second pass changes nothing."""
    for k in (1, 2):
        m, kind, p = workloads.quadrant_delaunay(n_cells=500, seed=11)
        o = oracle.Oracle(m, k)
        o.init_problem(kind, p)
        u = o.state(0)
        rng = np.random.default_rng(k)
        u[:, 1:, :] += 0.6 * rng.normal(size=u[:, 1:, :].shape) * np.abs(u[:, :1, :])
        before = o.limiter_node_values(u)
        assert (before[..., 0] < 0).any()                # the perturbation breaks positivity
        lim, bad = o.limit(u)
        assert bad == 0
        assert np.array_equal(lim[:, 0, :], u[:, 0, :])
        vals = o.limiter_node_values(lim)
        rho = vals[..., 0]
        e = vals[..., 3] - 0.5 * (vals[..., 1] ** 2 + vals[..., 2] ** 2) / rho
        assert rho.min() >= 1e-13 * (1 - 1e-9) - 1e-15
        assert e.min() >= 1e-13 * (1 - 1e-9) - 1e-14
        lim2, _ = o.limit(lim)
        assert np.abs(lim2 - lim).max() <= 1e-14 * np.abs(lim).max()


def test_limiter_theta_closed_form():
    """One P1 cell with rho = 1 + a Psi_1: at the node set the minimum of Psi_1 is the
    vertex value -2 (vertex v0), so theta_1 = (1 - eps)/(1 - (1 - 2a))."""
    m = smesh.Mesh(xy=np.array([[0, 0], [1, 0], [0, 1]], float), tri=np.array([[0, 1, 2]], np.int32))
    o = oracle.Oracle(m, 1)
    a = 0.8
    u = np.zeros((4, 3, 1))
    u[0, 0] = 1.0
    u[0, 1] = a
    u[3, 0] = 10.0
    lim, bad = o.limit(u)
    # limiter node set: edge Gauss points and v1, v2 (vertices opposite the two longest
    # edges: the hypotenuse is opposite v0, the legs tie and the stable order keeps v1)
    vals = o.limiter_node_values(u)[0, :, 0]
    rmin = vals.min()
    th = (1 - 1e-13) / (1 - rmin)
    assert abs(lim[0, 1, 0] - a * th) < 1e-15
    # the node set here is {Gauss points, v0, v1}: Psi_1(v0) = -2 gives 1 - 2a
    assert abs(rmin - (1 - 2 * a)) < 1e-15


def test_blast_positivity_and_failure_without_limiter():
    """Near-vacuum blast: with the BP limiter every node stays admissible; without it
    the scheme produces negative pressure (the failure the paper reports)."""
    m, kind, p = workloads.blast_delaunay(n_cells=1500, seed=3)
    o = oracle.Oracle(m, 2)
    assert o.init_problem(kind, p) == 0
    for _ in range(8):
        assert o.step() == 0
        vals = o.limiter_node_values(o.state(0))
        rho = vals[..., 0]
        e = vals[..., 3] - 0.5 * (vals[..., 1] ** 2 + vals[..., 2] ** 2) / rho
        assert rho.min() > 0 and e.min() > 0
    assert o.scalars()["n_limited"] > 0
    o2 = oracle.Oracle(m, 2, bp=False)
    o2.init_problem(kind, p)
    neg = False
    for _ in range(8):
        o2.step()
        vals = o2.limiter_node_values(o2.state(0))
        e = vals[..., 3] - 0.5 * (vals[..., 1] ** 2 + vals[..., 2] ** 2) / vals[..., 0]
        if (e < 0).any() or not np.isfinite(e).all():
            neg = True
            break
    assert neg


def _oversized_blast(**kw):
    """Near-vacuum blast with c_SSP = 4, four times the SSP coefficient the BP time
    step assumes: from the second step on, a stage leaves the admissible set."""
    m, kind, p = workloads.blast_delaunay(n_cells=3000, seed=23)
    o = oracle.Oracle(m, 2, cssp=4.0, **kw)
    assert o.init_problem(kind, p) == 0
    return o, m, kind, p


def test_restart_is_the_step_with_halved_dt():
    """A restarted step equals, bit for bit, a plain step taken with the halved
    Delta t from u^n (u^n is untouched by the discarded attempt)."""
    o, m, kind, p = _oversized_blast()
    assert o.step() == 0 and o.scalars()["n_restarts"] == 0
    s0, u_n = o.scalars(), o.state(0)
    assert o.step() == 0
    r = int(o.scalars()["n_restarts"])
    assert r >= 1
    ref, _, _, _ = _oversized_blast(max_restarts=0)
    assert ref.step() == 0
    assert np.array_equal(ref.state(0), u_n)
    ref.set_time(s0["t"], s0["dt"] / 2 ** r, s0["alpha"], int(s0["step"]))
    assert ref.step() == 0
    assert np.array_equal(ref.state(0), o.state(0))
    assert ref.scalars()["t"] == o.scalars()["t"] == s0["t"] + s0["dt"] / 2 ** r
    u = o.state(0)
    e = u[3, 0] - 0.5 * (u[1, 0] ** 2 + u[2, 0] ** 2) / u[0, 0]
    assert u[0, 0].min() > 0 and e.min() > 0


def test_restart_limit_stops_with_u_n_kept():
    o, m, kind, p = _oversized_blast(max_restarts=0)
    assert o.step() == 0
    u_n = o.state(0)
    assert o.step() == -5
    sc = o.scalars()
    assert sc["active"] == 0 and sc["step"] == 1
    assert np.array_equal(o.state(0), u_n)


# ----------------------------------------------------------------------------- convergence

def exact_cell_averages(m, t, params, period):
    """Cell averages of the exact vortex by the edge-midpoint... 7-point degree-5 rule
    (Radon), independent of the oracle's tables."""
    a = (6 - math.sqrt(15)) / 21
    b = (6 + math.sqrt(15)) / 21
    wa = (155 - math.sqrt(15)) / 1200
    wb = (155 + math.sqrt(15)) / 1200
    B = np.array([[1 / 3, 1 / 3, 1 / 3], [a, a, 1 - 2 * a], [a, 1 - 2 * a, a], [1 - 2 * a, a, a],
                  [b, b, 1 - 2 * b], [b, 1 - 2 * b, b], [1 - 2 * b, b, b]])
    W = np.array([9 / 40, wa, wa, wa, wb, wb, wb])
    V = m.cell_coords()
    X = np.einsum("qi,cid->cqd", B, V)
    rho, uu, vv, pp = problems.vortex_exact_primitive(X[..., 0], X[..., 1], t, params, period=period)
    return (rho * W).sum(axis=1)


@pytest.mark.parametrize("k,ns,lo", [(1, (16, 32, 64), 1.6), (2, (16, 32), 2.4)])
def test_vortex_convergence_order(k, ns, lo):
    """Design order k+1 on the isentropic vortex (the paper's accuracy tests show
    (k+1)-th order); L1 error of density cell averages at t = 0.5."""
    t_end = 0.5
    errs = []
    for n in ns:
        m, kind, p = workloads.periodic_vortex(n=n)
        o = oracle.Oracle(m, k)
        o.init_problem(kind, p)
        r, _ = o.run(t_end)
        assert r == 0 and abs(o.scalars()["t"] - t_end) < 1e-12
        area = o.mesh_arrays()["area"]
        ex = exact_cell_averages(m, t_end, p, 10.0)
        errs.append(np.sum(area * np.abs(o.state(0)[0, 0] - ex)) / area.sum())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > lo, (errs, rates)


# ----------------------------------------------------------------------------- OE, j >= 1, by hand

def _unit_square():
    """Cells A B C (lower right) and A C D (upper left) of the unit square; the
    shared edge is the diagonal AC, of length sqrt(2), with h = 2|K|/l = 1/sqrt(2)."""
    return smesh.Mesh(xy=np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float),
                      tri=np.array([[0, 1, 2], [0, 2, 3]], np.int32))


def _modal(o, m, fields):
    """Modal coefficients (4, nm, 2) of per-cell polynomial fields: fields[c](x, y)
    returns the four conservative variables.  Interpolation at the vertices (and edge
    midpoints for P2) of the reference triangle, through the oriented vertex order the
    oracle built; exact for polynomials of the cell's degree."""
    tri = o.mesh_arrays()["tri"]
    ref = [(0, 0), (1, 0), (0, 1)] + ([(0.5, 0), (0.5, 0.5), (0, 0.5)] if o.k == 2 else [])
    V = np.array([oracle.basis(xi, eta)[0][:o.nm] for xi, eta in ref])
    u = np.zeros((4, o.nm, m.n_cell))
    for c in range(m.n_cell):
        P = m.xy[tri[c]]
        vals = np.array([fields[c](*(P[0] + xi * (P[1] - P[0]) + eta * (P[2] - P[0]))) for xi, eta in ref])
        u[:, :, c] = np.linalg.solve(V, vals).T
    return u


def _damping_factors(o, u, f, var):
    """exp(-dt sum_{j<=m} sigma^j) per degree m (1..k) and cell, read from the modes of
    `var` that are nonzero (None where a degree has no such mode)."""
    out = {}
    for c in range(u.shape[2]):
        for deg, ls in ((1, (1, 2)), (2, (3, 4, 5))):
            if deg > o.k:
                continue
            r = [f[var, l, c] / u[var, l, c] for l in ls if abs(u[var, l, c]) > 1e-9]
            if r:
                assert max(r) - min(r) < 1e-14       # one factor per degree (eq. oe:sys)
                out[(c, deg)] = r[0]
    return out


# volume-point coordinate extremes of the quadrature rules (tab:2th, tab:4th): the
# barycentric coordinates that occur at the 3-point rule's points are 1/6 and 2/3; at
# the 6-point rule's points a, 1 - 2a, b, 1 - 2b
B6 = 0.091576213509770743
A6 = 0.44594849091596488


@pytest.mark.parametrize("k", [1, 2])
def test_oe_hand_computed_sigma1(k):
    """Density 1 + |x - y| (continuous on the diagonal, gradient jump (2, -2) at both
    endpoints), p = 1, v = 0.  With no value jump sigma^0 = 0 and, by eq. OEScalar:Coef2,
    sigma^1 = beta/h * A^{k,1} h / ||rho - rhobar|| * sqrt(1/2 (|j_A|^2 + |j_C|^2))
            = sqrt(1.4) * A^{k,1} * sqrt(8) / ||rho - rhobar||,
    A^{1,1} = 3, A^{2,1} = 1.  rhobar^Omega = 4/3; |x - y| at the volume points is a
    barycentric coordinate of the point, so the norm is 2/3 - 1/3 = 1/3 (3-point rule)
    or 1 - 2 b - 1/3 (6-point rule).  Degree-1 modes decay by exp(-dt sigma^1); for P2
    the degree-2 modes (here zero) would too."""
    m = _unit_square()
    o = oracle.Oracle(m, k)
    E = 1.0 / 0.4
    u = _modal(o, m, [lambda x, y: (1 + (x - y), 0, 0, E), lambda x, y: (1 - (x - y), 0, 0, E)])
    dt = 0.01
    f = o.oe(u, dt)
    nrm = 1.0 / 3.0 if k == 1 else (1 - 2 * B6) - 1.0 / 3.0
    A1 = 3.0 if k == 1 else 1.0
    sigma1 = math.sqrt(1.4) * A1 * math.sqrt(8.0) / nrm
    fac = _damping_factors(o, u, f, 0)
    for c in range(2):
        assert abs(fac[(c, 1)] - math.exp(-dt * sigma1)) < 1e-13, (fac[(c, 1)], math.exp(-dt * sigma1))
    # E is constant: its zero-norm branch leaves it alone; momentum is zero
    assert np.array_equal(f[1:], u[1:])


def test_oe_hand_computed_sigma2():
    """P2, density 1 +- (x - y)^2 / 2 (value and gradient continuous on the diagonal,
    Hessian jump (xx, xy, yy) = (-2, 2, -2)), p = 1 at the edge's ends, v = 0.  Only
    sigma^2 survives: sigma^2 = beta/h * A^{2,2} h^2 / ||.|| * sqrt(1/2 * 2 * (4 + 2*4 + 4))
    = sqrt(1.4) * (5/6) * h * 4 / ||.||, h = 1/sqrt(2) (the C_2 weight 2 on the mixed
    derivative enters as the 2*4).  rhobar^Omega = 1 (the two cells' averages are
    1 +- 1/12), and the norm is (1 - 2 b)^2 / 2 at the 6-point rule's points.  Degree-1
    modes (present: (x - y)^2 has them) stay, degree-2 modes decay by exp(-dt sigma^2)."""
    m = _unit_square()
    o = oracle.Oracle(m, 2)
    E = 1.0 / 0.4
    u = _modal(o, m, [lambda x, y: (1 + 0.5 * (x - y) ** 2, 0, 0, E),
                      lambda x, y: (1 - 0.5 * (x - y) ** 2, 0, 0, E)])
    dt = 0.01
    f = o.oe(u, dt)
    h = 1 / math.sqrt(2)
    nrm = 0.5 * (1 - 2 * B6) ** 2
    sigma2 = math.sqrt(1.4) * (5.0 / 6.0) * h * 4.0 / nrm
    fac = _damping_factors(o, u, f, 0)
    for c in range(2):
        assert abs(fac[(c, 1)] - 1.0) < 1e-13                 # sigma^0 = sigma^1 = 0
        assert abs(fac[(c, 2)] - math.exp(-dt * sigma2)) < 1e-13, (fac[(c, 2)], math.exp(-dt * sigma2))


@pytest.mark.parametrize("k", [1, 2])
def test_rioe_momentum_hand_computed(k):
    """RIOE for the momentum (eqs. RIOESys:Coef1/Coef2, RIOESys:CoefM): m = (2 phi, phi)
    with phi = +-(x - y) (a gradient jump only), rho = 1, E constant.  Across the
    diagonal n = (-1, 1)/sqrt(2): m_n = -phi/sqrt(2), m_t = m.(-n_y, n_x) = -3 phi/sqrt(2),
    so delta(m) = max(delta(m_n), delta(m_t)) takes m_t.  phi = |x - y| has mean 1/3 in
    each cell, and |||m - mbar||| = sqrt(5) ||phi - 1/3|| with ||phi - 1/3|| = 1/3
    (3-point rule) or 1 - 2 b - 1/3 (6-point rule).  v = 0 at the edge's ends, so
    beta = sqrt(1.4 p) with p = 0.4 E there.  sigma^1 = beta A^{k,1} * 3/sqrt(2) * sqrt(8)
    / (sqrt(5) ||phi||).  Both momentum components get that one factor; the
    component-wise OE (the control) gives each component its own."""
    m = _unit_square()
    E = 2.5
    fields = [lambda x, y: (1.0, 2 * (x - y), (x - y), E), lambda x, y: (1.0, -2 * (x - y), -(x - y), E)]
    dt = 0.002
    o = oracle.Oracle(m, k)
    u = _modal(o, m, fields)
    f = o.oe(u, dt)
    nphi = 1.0 / 3.0 if k == 1 else (1 - 2 * B6) - 1.0 / 3.0
    A1 = 3.0 if k == 1 else 1.0
    beta = math.sqrt(1.4 * 0.4 * E)
    sigma1 = beta * A1 * (3 / math.sqrt(2)) * math.sqrt(8.0) / (math.sqrt(5) * nphi)
    for var in (1, 2):
        fac = _damping_factors(o, u, f, var)
        for c in range(2):
            assert abs(fac[(c, 1)] - math.exp(-dt * sigma1)) < 1e-13, (var, c, fac[(c, 1)])
    # component-wise: m1 = 2 phi has ||m1 - m1bar|| = 2 ||phi||, jump 2x phi's, so the
    # same sigma^1 as phi alone: beta A sqrt(8) / ||phi||; the same for m2
    ocw = oracle.Oracle(m, k, oe_mode=1)
    fcw = ocw.oe(u, dt)
    s_cw = beta * A1 * math.sqrt(8.0) / nphi
    for var in (1, 2):
        fac = _damping_factors(ocw, u, fcw, var)
        for c in range(2):
            assert abs(fac[(c, 1)] - math.exp(-dt * s_cw)) < 1e-13, (var, c, fac[(c, 1)])


# ----------------------------------------------------------------------------- alpha, eq. 1250

@pytest.mark.parametrize("k", [1, 2])
def test_alpha_hand_computed_point_set(k):
    """alpha = max over every edge Gauss point of |v.n| + c (eq. 1250).  On the unit
    square take rho = 1 + x + 2y, v = (0, w), p = 1 (every conservative variable is
    linear).  The sound speed is largest where rho is smallest: along the bottom edge
    (normal (0, -1), |v.n| = w) at its first Gauss point x = s_1 = 1/2 - sqrt(3)/6 (P1)
    or 1/2 - sqrt(15)/10 (P2), so alpha = w + sqrt(1.4 / (1 + s_1)).  Vertices would give
    w + sqrt(1.4), edge midpoints w + sqrt(1.4 / 1.5); the left edge (|v.n| = 0) and the
    diagonal (|v.n| = w/sqrt(2), rho >= 1 + 3 s_1) give less."""
    m = _unit_square()
    o = oracle.Oracle(m, k)
    w = 0.3
    g = 1.4

    def state(x, y):
        r = 1 + x + 2 * y
        return (r, 0.0, r * w, 1.0 / (g - 1) + 0.5 * r * w * w)

    u = _modal(o, m, [state, state])
    s1 = 0.5 - math.sqrt(3) / 6 if k == 1 else 0.5 - math.sqrt(15) / 10
    want = w + math.sqrt(g / (1 + s1))
    assert abs(o.alpha_of(u) - want) < 1e-14 * want, (o.alpha_of(u), want)


# ----------------------------------------------------------------------------- threads

@pytest.mark.parametrize("k", [1, 2])
def test_threads_bitwise_equal_to_one(k):
    """The cell loops under OpenMP give, bit for bit, the one-thread result: every
    floating-point reduction over cells is taken serially in cell order."""
    m, kind, p = workloads.quadrant_delaunay(n_cells=3000, seed=31)
    runs = []
    for n in (1, 4):
        oracle.set_threads(n)
        o = oracle.Oracle(m, k)
        o.init_problem(kind, p)
        for _ in range(3):
            assert o.step() == 0
        runs.append((o.state(0), o.scalars()))
    oracle.set_threads(0)
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][1] == runs[1][1]
