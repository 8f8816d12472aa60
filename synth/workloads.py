"""Named workloads: a mesh plus a problem, built from fixed seeds.

* periodic_vortex    32 x 32 jittered periodic grid on [0,10]^2 (2048 cells), vortex
* quadrant_delaunay  Poisson-disk Delaunay mesh of the unit square, four-quadrant
                     Riemann data (rho in [0.14,1.5], p in [0.03,1.5])
* blast_delaunay     Delaunay mesh of [-1.1,1.1]^2 with the origin as a vertex,
                     near-vacuum blast (ambient p = 1e-10, E_total = 0.25)
* batch_instances    n meshes with log-uniform sizes, P1/P2 split, two-state data
* serving_requests   a seeded request stream: log-uniform sizes, P1 or P2, Riemann
                     or vortex data, final times, Poisson arrival times
* implosion          the implosion quadrant [0,0.3]^2 with reflective walls, low state
                     in x + y <= 0.15 (Example EulerImp), optionally turned clockwise
                     by pi/4 with its data (the rotation-invariance test)
* largest_periodic   86 x 127 copies of the periodic vortex block: 22,368,256 cells,
                     the most whole blocks within the largest P2 mesh (22,369,621 cells,
                     a state buffer below 4 GiB), vortex data
"""

import numpy as np

from .mesh import periodic_jittered_grid, poisson_delaunay, find_vertex, tile_periodic_grid
from .problems import (PROBLEM_VORTEX, PROBLEM_QUADRANT, PROBLEM_BLAST, PROBLEM_TWO_STATE,
                       vortex_params, quadrant_riemann_params, blast_params, two_state_params)
from .rng import Stream


def periodic_vortex(n=32, seed=1):
    m = periodic_jittered_grid(n=n, length=10.0, jitter=0.1, seed=seed)
    return m, PROBLEM_VORTEX, vortex_params()


def largest_periodic(seed=1):
    base = periodic_jittered_grid(n=32, length=10.0, jitter=0.1, seed=seed)
    return tile_periodic_grid(base, 86, 127), PROBLEM_VORTEX, vortex_params()


def quadrant_delaunay(n_cells=200_000, seed=2):
    m = poisson_delaunay(n_cells, lo=(0.0, 0.0), hi=(1.0, 1.0), seed=seed,
                         name=f"quadrant{n_cells}")
    return m, PROBLEM_QUADRANT, quadrant_riemann_params(seed)


def blast_delaunay(n_cells=1_000_000, seed=3):
    m = poisson_delaunay(n_cells, lo=(-1.1, -1.1), hi=(1.1, 1.1), seed=seed,
                         extra_points=np.array([[0.0, 0.0]]), name=f"blast{n_cells}")
    ov = find_vertex(m, (0.0, 0.0))
    assert ov >= 0
    return m, PROBLEM_BLAST, blast_params(ov)


def implosion(n_cells=20_000, seed=6, rotate=False, inner=(0.125, 0.14)):
    """Example EulerImp on a seeded Delaunay stand-in for its mesh: (rho, v, p) =
    (0.125, 0, 0.14) where x + y < 0.15, (1, 0, 1) elsewhere, every wall reflective.
    inner: (rho, p) of the region x + y < 0.15 in place of the example's.
    rotate: the mesh turned clockwise by pi/4, x' = M x with M = [[c, c], [-c, c]],
    c = sqrt(2)/2 (same cells and ids); the data turn with it (v = 0, so only the
    dividing line moves)."""
    m = poisson_delaunay(n_cells, lo=(0.0, 0.0), hi=(0.3, 0.3), seed=seed, name=f"implosion{n_cells}")
    m.edge_bc = np.ones((m.n_cell, 3), np.int32)       # every boundary edge is a wall
    lo_state, hi_state = [float(inner[0]), 0.0, 0.0, float(inner[1])], [1.0, 0.0, 0.0, 1.0]
    if not rotate:
        p = np.array([0.15, 0.0, 1.0, 1.0] + lo_state + hi_state)
        return m, PROBLEM_TWO_STATE, p
    c = np.sqrt(2.0) / 2.0
    M = np.array([[c, c], [-c, c]])
    m.xy = np.ascontiguousarray(m.xy @ M.T)
    m.name += "_rot"
    p = np.array([0.15 * c, -0.15 * c, 1.0, 0.0] + lo_state + hi_state)
    return m, PROBLEM_TWO_STATE, p


def wall_tags(m, on_line):
    """(n_cell, 3) tags: 1 for the edges (opposite vertex i) whose two ends satisfy
    on_line(x, y), else 0."""
    x, y = m.xy[m.tri, 0], m.xy[m.tri, 1]
    on = on_line(x, y)
    tags = np.zeros((m.n_cell, 3), np.int32)
    for i in range(3):
        tags[:, i] = on[:, (i + 1) % 3] & on[:, (i + 2) % 3]
    return tags


def batch_sizes(n_inst=64, lo=5_000, hi=500_000, seed=4):
    st = Stream(seed * 31 + 1)
    sizes = st.log_uniform(n_inst, lo, hi).astype(np.int64)
    degree = np.where(st.uniform(n_inst) < 0.5, 1, 2)
    return sizes, degree


def batch_instance(i, size, seed=4):
    m = poisson_delaunay(int(size), seed=seed * 1000 + i, name=f"inst{i}")
    return m, PROBLEM_TWO_STATE, two_state_params(seed * 1000 + i)


def serving_requests(n_req=32, rate=50.0, seed=5, lo=1_000, hi=2_000_000, scale=1, t_lo=0.05, t_hi=0.5,
                     t_scale=1.0):
    """Request specs of a serving run (meshes are built by serving_request).

    Sizes log-uniform in [lo, hi] / scale triangles, degree 1 or 2 and Riemann
    (two states at rest across a random line in the unit square, rho and p
    log-uniform in [0.14, 1.5], reflective walls) or vortex data (Delaunay mesh of
    [0,10]^2) with
    probability 1/2 each, t_end uniform in [t_lo, t_hi] times t_scale, arrivals a
    Poisson process of the given rate per second (exponential gaps by inversion)."""
    st = Stream(seed * 53 + 7)
    sizes = np.maximum(st.log_uniform(n_req, lo, hi) / scale, 64).astype(np.int64)
    degree = np.where(st.uniform(n_req) < 0.5, 1, 2)
    vortex = st.uniform(n_req) < 0.5
    t_end = st.uniform(n_req, t_lo, t_hi) * t_scale
    gaps = -np.log(1.0 - st.uniform(n_req)) / rate
    arrival = np.cumsum(gaps) - gaps[0]
    return [dict(id=i, n_cells=int(sizes[i]), k=int(degree[i]), vortex=bool(vortex[i]), t_end=float(t_end[i]),
                 arrival=float(arrival[i]), seed=seed * 10_000 + i) for i in range(n_req)]


def serving_request(spec):
    """(mesh, kind, params) of one request spec."""
    if spec["vortex"]:
        m = poisson_delaunay(spec["n_cells"], lo=(0.0, 0.0), hi=(10.0, 10.0), seed=spec["seed"],
                             name=f"req{spec['id']}")
        return m, PROBLEM_VORTEX, vortex_params()
    # walls: a discontinuity that meets a transmissive (extrapolated) boundary can
    # grow there on fine meshes, which would stall the request's time step
    m = poisson_delaunay(spec["n_cells"], seed=spec["seed"], name=f"req{spec['id']}")
    m.edge_bc = np.ones((m.n_cell, 3), np.int32)
    return m, PROBLEM_TWO_STATE, two_state_params(spec["seed"], lo=0.14, hi=1.5)
