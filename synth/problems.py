"""Parameter vectors of the initial-value problems (inputs, not method arithmetic).

Layouts (float64 vectors handed unchanged to `dg_init_problem` and to the oracle):

* PROBLEM_VORTEX (0): [x0, y0, eps, rho_inf, u_inf, v_inf, p_inf]
  Isentropic vortex: with (xb, yb) = (x - x0, y - y0), r2 = xb^2 + yb^2,
  du = -eps/(2 pi) e^{(1-r2)/2} yb, dv = eps/(2 pi) e^{(1-r2)/2} xb,
  T = 1 - (gamma-1) eps^2/(8 gamma pi^2) e^{1-r2}, rho = rho_inf T^{1/(gamma-1)},
  p = rho^gamma (for rho_inf = p_inf = 1).  It translates with (u_inf, v_inf).
* PROBLEM_QUADRANT (1): [xc, yc, (rho, u, v, p) for quadrants q = 0..3]
  q = [x >= xc] + 2 [y >= yc].
* PROBLEM_BLAST (2): [E_total, p_ambient, rho, origin_vertex_id]
  Cell averages only: rho everywhere, zero velocity, ambient E = p/(gamma-1); the
  cells that have the origin vertex share E_total in proportion to their area.
* PROBLEM_TWO_STATE (3): [px, py, nx, ny, (rho, u, v, p)_L, (rho, u, v, p)_R]
  State L where (x - px) nx + (y - py) ny < 0, else R.
"""

import numpy as np

from .rng import Stream

PROBLEM_VORTEX = 0
PROBLEM_QUADRANT = 1
PROBLEM_BLAST = 2
PROBLEM_TWO_STATE = 3


def vortex_params(x0=5.0, y0=5.0, eps=5.0, rho=1.0, u=1.0, v=1.0, p=1.0) -> np.ndarray:
    return np.array([x0, y0, eps, rho, u, v, p], dtype=np.float64)


def quadrant_riemann_params(seed: int = 2, xc=0.5, yc=0.5) -> np.ndarray:
    """Four random constant states: rho log-uniform in [0.14, 1.5], p log-uniform in
    [0.03, 1.5], velocity components uniform in [-0.75, 0.75]."""
    st = Stream(seed * 7919 + 17)
    rho = st.log_uniform(4, 0.14, 1.5)
    p = st.log_uniform(4, 0.03, 1.5)
    u = st.uniform(4, -0.75, 0.75)
    v = st.uniform(4, -0.75, 0.75)
    out = [xc, yc]
    for q in range(4):
        out += [rho[q], u[q], v[q], p[q]]
    return np.array(out, dtype=np.float64)


def blast_params(origin_vertex: int, e_total=0.25, p_ambient=1e-10, rho=1.0) -> np.ndarray:
    return np.array([e_total, p_ambient, rho, float(origin_vertex)], dtype=np.float64)


def two_state_params(seed: int, lo=1e-3, hi=10.0, box=((0.0, 0.0), (1.0, 1.0))) -> np.ndarray:
    """Random line through the box, two states with rho, p log-uniform in [lo, hi], v = 0."""
    st = Stream(seed * 104729 + 3)
    (x0, y0), (x1, y1) = box
    px, py = st.uniform(1, x0, x1)[0], st.uniform(1, y0, y1)[0]
    ang = st.uniform(1, 0.0, 2.0 * np.pi)[0]
    rho = st.log_uniform(2, lo, hi)
    p = st.log_uniform(2, lo, hi)
    return np.array([px, py, np.cos(ang), np.sin(ang),
                     rho[0], 0.0, 0.0, p[0], rho[1], 0.0, 0.0, p[1]], dtype=np.float64)


def vortex_exact_primitive(x, y, t, params, gamma=1.4, period=None):
    """Exact (rho, u, v, p) of the translating vortex at time t.

    With `period` set the nearest periodic image of the centre is used.
    """
    x0, y0, eps, rho_inf, u_inf, v_inf, p_inf = params[:7]
    cx = x0 + u_inf * t
    cy = y0 + v_inf * t
    xb = np.asarray(x, float) - cx
    yb = np.asarray(y, float) - cy
    if period is not None:
        xb = xb - period * np.round(xb / period)
        yb = yb - period * np.round(yb / period)
    r2 = xb * xb + yb * yb
    g = eps / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * np.pi * np.pi) * np.exp(1.0 - r2)
    rho = rho_inf * T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma * (p_inf / rho_inf ** gamma)
    return rho, u_inf - g * yb, v_inf + g * xb, p
