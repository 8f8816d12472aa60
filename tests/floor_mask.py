"""Cells whose results are ill-conditioned in FP64 because a limiter node sits at
the density floor, for stage-by-stage comparisons of two FP64 codes.

The BP limiter (Sec. 4.4) first scales the density's higher modes so that the
smallest node density is eps_1 = min(rho_bar, 1e-13); the internal energy of that
density-limited state is then formed at its nodes, and E - |m|^2 / (2 rho) at a
node with rho = eps_1 carries the rounding of rho (about 1e-17 absolute, so a
relative 1e-4 at 1e-13) into theta_2.  A stored state with a node at eps_1 passes
the same division on to whatever reads that node later: the LF flux and alpha at
edge Gauss points, beta at the vertices.  So a cell is set aside when a node of a
state the limiter forms there (its input, its density-limited state, its output)
has a density within 10 eps_1, and so are the cells that read such a cell: each
stage couples a cell to its edge neighbours twice, through the residual's flux
and through the filter's jumps.  A node at the internal-energy floor divides
nothing (its pressure and sound speed are merely small), so it is not set aside.

Two ways of comparing use this:
* same input: both codes run one stage from the same u^n, stage input, Delta t
  and alpha (`same_input_masks`);
* independent trajectories: each code steps on its own, and the cells set aside
  at a stage stay set aside, grown by two rings of neighbours per stage
  (`independent_mask`).
"""

import numpy as np

EPS_BP = 1e-13


def near_floor(o, u, factor=10.0):
    """Cells of state u with a limiter node whose density is within factor * eps_1
    of the floor (node values from the oracle)."""
    rho = o.limiter_node_values(u)[..., 0]
    eps1 = np.minimum(np.abs(u[0, 0, :]), EPS_BP)
    return (rho <= factor * eps1[:, None]).any(axis=1)


def grow(mask, nbr, layers):
    """mask plus `layers` rings of edge neighbours (nbr: (n_cell, 3), -1 at a
    boundary edge)."""
    m = mask.copy()
    for _ in range(layers):
        hit = np.zeros_like(m)
        for i in range(3):
            nb = nbr[:, i]
            ok = nb >= 0
            hit[ok] |= m[nb[ok]]
        m |= hit
    return m


def limiter_floor(o, pres, outs, dt, oe=True):
    """Cells near the density floor in a state the limiter forms: its input (the oracle's OE
    filter of each pre-filter state in `pres`; where the density step acts, the
    density-limited state has a node at eps, and that node's density is below
    10 eps in the input) or its output (each of `outs`)."""
    mask = np.zeros(o.nc, bool)
    for pre in pres:
        mask |= near_floor(o, o.oe(pre, dt) if oe else pre)
    for out in outs:
        mask |= near_floor(o, out)
    return mask


def same_input_masks(o, u_in, pres, outs, dt, nbr, oe=True):
    """(pre-filter mask, output mask) of one stage run by both codes from the same
    input: the pre-filter state reads the input's floor cells and their
    neighbours; the output adds the limiter's own floor cells and one more ring
    (the filter's jumps)."""
    m_pre = grow(near_floor(o, u_in), nbr, 1)
    m_out = grow(m_pre, nbr, 1) | limiter_floor(o, pres, outs, dt, oe)
    return m_pre, m_out


def independent_mask(o, pres, outs, dt, nbr, prev, oe=True):
    """The set-aside cells after a stage of two independent trajectories: the
    limiter's floor cells of this stage plus the previous set grown by two rings
    (`prev`: the set before the stage; for the first stage, the initial state's
    floor cells)."""
    return limiter_floor(o, pres, outs, dt, oe) | grow(prev, nbr, 2)


def var_scales(ref):
    """Scale of each conservative variable: the largest |coefficient| of rho and E,
    and for the momentum components sqrt(2 max rho max E), which bounds |m| on every
    admissible state (E >= |m|^2 / (2 rho)); a momentum that is zero in the data
    would otherwise be measured against its own rounding noise."""
    r, e = np.abs(ref[0]).max(), np.abs(ref[3]).max()
    sm = max(np.sqrt(2.0 * r * e), np.abs(ref[1]).max(), np.abs(ref[2]).max())
    return np.array([r, sm, sm, e])


def masked_err(a, b, mask=None):
    """max over variables of max |a - b| over the cells outside mask, over the
    variable's scale."""
    sc = var_scales(b)
    keep = slice(None) if mask is None else ~mask
    out = 0.0
    for v in range(4):
        d = np.abs(a[v] - b[v])[:, keep]
        if d.size:
            out = max(out, d.max() / sc[v])
    return out


def oracle_stage(o, st, u_n, u_in, dt, alpha, oe=True, bp=True):
    """Stage st of the oracle from given inputs: the pre-filter state (residual with
    LF viscosity alpha, SSP combination) and the output (OE filter, then limiter),
    each step enabled as in the codes' configuration."""
    a, b = (0.0, 0.75, 1.0 / 3.0)[st], (1.0, 0.25, 2.0 / 3.0)[st]
    pre = a * u_n + b * (u_in + dt * o.residual(u_in, alpha))
    out = o.oe(pre, dt) if oe else pre.copy()
    if bp:
        out = o.limit(out)[0]
    return pre, out


def alpha_tolerance(o, state, floor=1e-13):
    """Relative bound for the max wave speed of a limited state.

    The density at an edge Gauss point is a sum of O(rho_bar) terms; where the
    limiter put it near its 1e-13 floor, two FP64 evaluation orders differ by about
    1e-16 rho_bar absolutely, and the sound speed (~ rho^-1/2) inherits half that
    relative error.  Bound: 1e-15 max_K rho_bar_K / rho_min_K, at least `floor`."""
    npt = 3 * (o.k + 1)
    vals = o.limiter_node_values(state)[:, :npt, 0]
    ratio = (np.abs(state[0, 0, :]) / np.maximum(vals.min(axis=1), 1e-13)).max()
    return max(floor, 1e-15 * ratio)


def same_input_stages(s, o, steps, say, oe=True, bp=True, tol=1e-12, max_frac=0.1):
    """Every stage of `steps` steps of the HIP solver s, each against the oracle's
    stage run from the solver's own inputs (u^n, stage input, Delta t and its LF
    viscosity): alpha within its conditioning bound, then the pre-filter state and
    the output within tol of each variable's scale outside the set-aside cells,
    the momentum norm of the solver's own pre-filter state (mbar from the solver's
    conservation bookkeeping) against the oracle's direct average, and after each
    step alpha and Delta t of the new u^n.  Returns the largest set-aside count."""
    nbr = o.mesh_arrays()["nbr"]
    minck = o.scalars()["minck"]
    worst = 0
    for step in range(steps):
        u_n = s.read_state(0)
        for st in range(3):
            u_in = u_n if st == 0 else s.read_state(1)
            d = s.diag()
            dt, a_gpu = d["dt"], d["alpha_stage"]
            a_or = o.alpha_of(u_in)
            a_tol = alpha_tolerance(o, u_in)
            assert abs(a_gpu - a_or) <= a_tol * a_or, (step, st, a_gpu, a_or, a_tol)
            want_pre, want_out = oracle_stage(o, st, u_n, u_in, dt, a_gpu, oe, bp)
            s.stage(st)
            pre, out = s.read_state(2), s.read_state(1)
            m_pre, m_out = same_input_masks(o, u_in, [want_pre, pre], [want_out, out], dt, nbr, oe)
            e_pre, e_out = masked_err(pre, want_pre, m_pre), masked_err(out, want_out, m_out)
            worst = max(worst, int(m_out.sum()))
            say(f"  step {step} stage {st}: alpha rel {abs(a_gpu - a_or) / a_or:.1e} (bound {a_tol:.1e}), "
                f"pre {e_pre:.2e} out {e_out:.2e}, set aside {int(m_pre.sum())}/{int(m_out.sum())} of {o.nc}")
            assert e_pre <= tol and e_out <= tol, (step, st, e_pre, e_out)
            if oe:
                o.oe(pre, dt)
                n_gpu, n_orc = s.diag()["nrm_m"], o.scalars()["nrm_m"]
                assert abs(n_gpu - n_orc) <= tol * max(n_orc, var_scales(pre)[1]), (step, st, n_gpu, n_orc)
        d = s.diag()
        ug = s.readback()[0]
        ag = o.alpha_of(ug)
        a_tol = alpha_tolerance(o, ug, floor=1e-12)
        assert abs(d["alpha"] - ag) <= a_tol * ag, (d["alpha"], ag, a_tol)
        assert abs(d["dt"] - minck / ag) <= a_tol * d["dt"], (d["dt"], minck / ag, a_tol)
        assert d["step"] == step + 1
    assert worst <= max_frac * o.nc
    return worst
