"""Pins of the oracle's u* form of the P2 limiter with the optimal decomposition
(Sec. 4.4 applied to the decomposition of eq. 1139): u* formed with the optimal edge
weights equals the mean of the two internal nodes (the decomposition is exact and
weights its two nodes alike), each of its two steps limits no more than the node
form's (u* is a convex combination of the nodes; rho is linear and rho e concave),
the limited state is positive at the edge points and at u*, and P1 has no u* form."""

import numpy as np
import pytest

import oracle
from synth import workloads


def _oscillating_state(o, seed):
    """the workload's initial state with large random higher modes: some limiter
    nodes of the result have rho < 0"""
    u = o.state(0)
    rng = np.random.default_rng(seed)
    u[:, 1:, :] += 0.6 * rng.normal(size=u[:, 1:, :].shape) * np.abs(u[:, :1, :])
    return u


def test_ustar_is_the_mean_of_the_internal_nodes():
    """(ubar - sum_i w_i sum_nu w_nu u(x_i,nu)) / (1 - sum_i w_i) with the optimal edge
    weights equals (u(n_1) + u(n_2)) / 2, for every variable and cell of a random
    state; the edge-point slots are the node form's."""
    m, _, _ = workloads.quadrant_delaunay(n_cells=600, seed=41)
    rng = np.random.default_rng(7)
    u = rng.normal(size=(4, 6, m.n_cell))
    nodes = oracle.Oracle(m, 2).limiter_node_values(u)
    ustar = oracle.Oracle(m, 2, limiter_form="ustar").limiter_node_values(u)
    assert np.array_equal(ustar[:, :9], nodes[:, :9])
    mean = 0.5 * (nodes[:, 9] + nodes[:, 10])
    scale = np.abs(u).max()
    for t in (9, 10):
        assert np.abs(ustar[:, t] - mean).max() < 1e-13 * scale
    # and it is not one of the nodes
    assert np.abs(ustar[:, 9] - nodes[:, 9]).max() > 1e-3 * scale


def test_ustar_limits_no_more_than_the_node_form():
    """Density step, on a state at rest with uniform energy (so theta_2 = 1): theta_1 of
    the u* form >= that of the node form in every cell (rho is linear, so rho(u*) is
    the nodes' mean).  Energy step, on a state with cell-wise constant density (so
    theta_1 = 1): theta_2 of the u* form >= that of the node form (rho e is concave on
    rho > 0, so rho e(u*) >= the smaller nodal value).  Averages are untouched and
    the forms differ in some cells."""
    m, kind, p = workloads.quadrant_delaunay(n_cells=800, seed=42)
    on = oracle.Oracle(m, 2)
    ou = oracle.Oracle(m, 2, limiter_form="ustar")
    on.init_problem(kind, p)
    base = on.state(0)
    rng = np.random.default_rng(11)
    cases = []
    u = base.copy()                      # density step only
    u[1:3] = 0.0
    u[3, 1:] = 0.0
    u[0, 1:] = 0.6 * rng.normal(size=u[0, 1:].shape) * u[0, :1]
    cases.append((u, 0))
    u = base.copy()                      # energy step only
    u[0, 1:] = 0.0
    u[1:, 1:] = 0.3 * rng.normal(size=u[1:, 1:].shape) * np.abs(u[1:, :1]).max(axis=0)
    cases.append((u, 3))
    for u, var in cases:
        ln, bn = on.limit(u)
        lu, bu = ou.limit(u)
        assert bn == 0 and bu == 0
        assert np.array_equal(ln[:, 0], u[:, 0]) and np.array_equal(lu[:, 0], u[:, 0])
        # theta of the step from the first higher mode of the variable it scales
        tn, tu = ln[var, 1] / u[var, 1], lu[var, 1] / u[var, 1]
        assert (tn < 1 - 1e-9).sum() > 20
        assert np.all(tu >= tn * (1 - 1e-12) - 1e-15)
        assert (tu > tn * (1 + 1e-6)).any()


def test_ustar_limited_state_is_positive_at_its_points():
    """after the u* form: rho >= eps_1 and rho e >= eps_2 at the 9 edge points and at
    u* (Sec. 4.4), up to rounding"""
    m, kind, p = workloads.quadrant_delaunay(n_cells=800, seed=43)
    ou = oracle.Oracle(m, 2, limiter_form="ustar")
    ou.init_problem(kind, p)
    u = _oscillating_state(ou, 12)
    assert (ou.limiter_node_values(u)[..., 0] < 0).any()
    lim, bad = ou.limit(u)
    assert bad == 0
    v = ou.limiter_node_values(lim)
    rho = v[..., 0]
    e = v[..., 3] - 0.5 * (v[..., 1] ** 2 + v[..., 2] ** 2) / rho
    assert rho.min() >= 1e-13 * (1 - 1e-9) - 1e-15
    assert e.min() >= 1e-13 * (1 - 1e-9) - 1e-14


def test_p1_has_no_ustar_form():
    """P1: the optimal decomposition's limiter is eq. 1944 in both forms (bitwise)"""
    m, kind, p = workloads.quadrant_delaunay(n_cells=500, seed=44)
    on = oracle.Oracle(m, 1)
    ou = oracle.Oracle(m, 1, limiter_form="ustar")
    on.init_problem(kind, p)
    u = _oscillating_state(on, 13)
    assert np.array_equal(on.limit(u)[0], ou.limit(u)[0])


def test_limiter_form_is_checked():
    m, _, _ = workloads.quadrant_delaunay(n_cells=100, seed=45)
    with pytest.raises(ValueError):
        oracle.Oracle(m, 2, limiter_form="centroid")
