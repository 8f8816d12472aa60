"""dg_stage_noalloc (partial records in the library's own device array) against
dg_stage, through the C ABI: two calls in a row on one GPU, the second on a
smaller mesh, each compared bit for bit with the allocating entry point."""

import sys

import numpy as np
import pytest

from synth import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():   # collected on CPU-only hosts, skipped there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2409_09620_amd import Solver  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(mesh, k, kind, params, **cfg):
    a, b = Solver(mesh, k), Solver(mesh, k)
    a.init_problem(kind, params, **cfg)
    b.init_problem(kind, params, **cfg)
    return a, b


def _run_and_compare(mesh, k, kind, params, steps=2, **cfg):
    a, b = _pair(mesh, k, kind, params, **cfg)
    for _ in range(steps):
        for s in range(3):
            a.stage(s)
            b.stage_noalloc(s)
    for which in (0, 1, 2):
        ua, ub = a.read_state(which), b.read_state(which)
        assert np.array_equal(ua, ub), (which, np.abs(ua - ub).max())
    da, db = a.diag(), b.diag()
    for key in ("t", "dt", "alpha", "step", "n_limited", "nrm_m"):
        assert da[key] == db[key], (key, da[key], db[key])
    assert da["ubar"] == db["ubar"] and da["nrm"] == db["nrm"]
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_stage_twice(precision):
    # first call on a 12k-cell P2 mesh, then on a 900-cell P1 mesh: the second
    # call's reduction must not see records left by the first
    m1, kind1, p1 = workloads.quadrant_delaunay(n_cells=12000, seed=41)
    say(f"[gpu case] noalloc {precision} P2 quadrant cells={m1.n_cell}")
    _run_and_compare(m1, 2, kind1, p1, precision=precision)
    m2, kind2, p2 = workloads.blast_delaunay(n_cells=900, seed=42)
    say(f"[gpu case] noalloc {precision} P1 blast cells={m2.n_cell}")
    _run_and_compare(m2, 1, kind2, p2, precision=precision)


def test_noalloc_rejects_bad_stage():
    m, kind, p = workloads.quadrant_delaunay(n_cells=500, seed=43)
    s = Solver(m, 2)
    s.init_problem(kind, p)
    with pytest.raises(Exception):
        s.stage_noalloc(3)
    s.close()


def test_skipped_stages_keep_their_domain_values():
    """A stage that leaves the admissible set makes the rest of its attempt skip
    their passes; their reductions then read whatever the shared array holds (here
    another context's records, written in between) and must leave this context's
    domain averages and norms as dg_stage leaves them."""
    m, kind, p = workloads.blast_delaunay(n_cells=3000, seed=23)
    a, b = _pair(m, 2, kind, p, c_ssp=4.0)
    mo, kind_o, p_o = workloads.quadrant_delaunay(n_cells=5000, seed=44)
    other = Solver(mo, 2)
    other.init_problem(kind_o, p_o)
    say(f"[gpu case] noalloc skipped stages, blast cells={m.n_cell}, other cells={mo.n_cell}")
    for it in range(4):
        for s in range(3):
            a.stage(s)
            b.stage_noalloc(s)
            other.stage_noalloc(s)
            da, db = a.diag(), b.diag()
            assert da["ubar"] == db["ubar"] and da["nrm"] == db["nrm"] and da["nrm_m"] == db["nrm_m"], (it, s)
    assert a.diag()["n_restarts"] >= 1 and b.diag()["n_restarts"] == a.diag()["n_restarts"]
    for which in (0, 1, 2):
        assert np.array_equal(a.read_state(which), b.read_state(which)), which
    for s in (a, b, other):
        s.close()
