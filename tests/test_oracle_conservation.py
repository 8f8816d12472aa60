"""Pins of the identity that lets the residual pass know the domain momentum average of
the state it writes before writing it: the DG residual in divergence form conserves
sum_K |K| ubar_K up to the flux through the boundary, so

    sum_K |K| d(mbar_K)/dt = -(A + alpha B),

with A + alpha B the boundary momentum flux the residual takes at the edge Gauss points:
F(u).n at transmissive edges, ((m.n)^2/rho + p) n + alpha (m.n) n at reflective ones
(the LF viscosity term of the mirrored state).  Checked against the oracle's own
residual on transmissive, reflective and periodic meshes, with random higher modes."""

import numpy as np
import pytest

import oracle
from synth import mesh as smesh
from synth import problems, workloads

GW = {1: np.array([0.5, 0.5]), 2: np.array([5.0, 8.0, 5.0]) / 18.0}


def boundary_flux(o, u, gamma=1.4):
    """(A, B) of state u: sums over boundary edges of l w_nu times the transmissive flux
    or the wall parts, from the oracle's values at the edge Gauss points.  All boundary
    edges of a mesh carry the same tag here, given by o.wall."""
    k = o.k
    ne = k + 1
    mesh = o.mesh_arrays()
    vals = o.limiter_node_values(u)            # (nc, 3 ne + 2, 4): edge points first
    A, B = np.zeros(2), np.zeros(2)
    for c, i in zip(*np.nonzero(mesh["nbr"] < 0)):
        n = mesh["nrm"][c, i]
        for nu in range(ne):
            q = vals[c, i * ne + nu]
            lw = mesh["len"][c, i] * GW[k][nu]
            rho, m = q[0], q[1:3]
            p = (gamma - 1.0) * (q[3] - 0.5 * (m @ m) / rho)
            mn = m @ n
            if o.wall:
                A += lw * (mn * mn / rho + p) * n
                B += lw * mn * n
            else:
                A += lw * (m * mn / rho + p * n)
    return A, B


def _perturbed(o, seed, amp=0.05):
    u = o.state(0)
    rng = np.random.default_rng(seed)
    u[:, 1:, :] += amp * rng.normal(size=u[:, 1:, :].shape) * np.abs(u[:, :1, :])
    return u


def _cases():
    q = workloads.quadrant_delaunay(n_cells=900, seed=61)
    box = smesh.poisson_delaunay(900, lo=(0.0, 0.0), hi=(10.0, 10.0), seed=62)
    box.edge_bc = workloads.wall_tags(box, lambda x, y: (x == 0) | (x == 10) | (y == 0) | (y == 10))
    v = workloads.periodic_vortex(n=12)
    return {"transmissive": (q, False), "reflective": ((box, problems.PROBLEM_VORTEX, problems.vortex_params()), True),
            "periodic": (v, False)}


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("case", ["transmissive", "reflective", "periodic"])
def test_residual_momentum_sum_is_the_boundary_flux(case, k):
    (m, kind, p), wall = _cases()[case]
    o = oracle.Oracle(m, k)
    o.wall = wall
    assert o.init_problem(kind, p) == 0
    u = _perturbed(o, 7 + k)
    alpha = o.alpha_of(u)
    L = o.residual(u, alpha)                    # d/dt of the modal coefficients
    area = o.mesh_arrays()["area"]
    lhs = np.array([area @ L[1, 0], area @ L[2, 0]])
    A, B = boundary_flux(o, u)
    # scale: the sum of the magnitudes of the cells' flux contributions
    scale = np.abs(area * np.abs(L[1:3, 0]).sum(axis=0)).sum() + 1.0
    assert np.abs(lhs + (A + alpha * B)).max() <= 1e-12 * scale, (lhs, A, B, alpha)
    if case == "periodic":
        assert np.abs(A).max() == 0.0 and np.abs(B).max() == 0.0
    if case == "reflective":
        assert np.abs(B).max() > 1e-3          # the viscosity term is exercised
