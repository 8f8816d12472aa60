"""Batched stepping (dg_batch_*) on the GPU, through the C ABI.

A member's reductions run over its own 256-cell groups in a fixed order, so its
result must be the same bit for bit alone, in any mix and under any schedule;
against the FP64 oracle it meets the same bound as the single-instance path.
"""

import sys

import numpy as np
import pytest

import oracle
from synth import mesh as smesh
from synth import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():   # collected on CPU-only hosts, skipped there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2409_09620_amd import Batch, DgError, Solver  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(a, b):
    out = 0.0
    for v in range(4):
        scale = max(np.abs(b[v]).max(), 1e-300)
        out = max(out, np.abs(a[v] - b[v]).max() / scale)
    return out


MEMBERS = {
    "p2_quadrant_3k": lambda: (2,) + workloads.quadrant_delaunay(n_cells=3000, seed=21),
    "p1_quadrant_2k": lambda: (1,) + workloads.quadrant_delaunay(n_cells=2000, seed=22),
    "p1_vortex": lambda: (1,) + workloads.periodic_vortex(n=16),
    "p2_vortex": lambda: (2,) + workloads.periodic_vortex(n=10),
    "p2_two_state_1k": lambda: (2,) + workloads.batch_instance(3, 1000),
    "p1_two_state_700": lambda: (1,) + workloads.batch_instance(4, 700),
    # cells in random order: most neighbours beyond the tiles' halo cap (global-memory path)
    "p2_quadrant_3k_shuffled": lambda: _shuffled(2, workloads.quadrant_delaunay(n_cells=3000, seed=21), 33),
    "p1_quadrant_2k_shuffled": lambda: _shuffled(1, workloads.quadrant_delaunay(n_cells=2000, seed=22), 34),
}


def _shuffled(k, w, seed):
    m, kind, p = w
    return (k, smesh.shuffle_cells(m, seed), kind, p)
_CACHE = {}


def member(name, precision="fp64"):
    if name not in _CACHE:
        _CACHE[name] = MEMBERS[name]()
    k, m, kind, p = _CACHE[name]
    s = Solver(m, k)
    s.init_problem(kind, p, precision=precision)
    return s


@pytest.mark.parametrize("names", [["p2_quadrant_3k", "p1_quadrant_2k", "p1_vortex", "p2_vortex"],
                                   ["p2_quadrant_3k_shuffled", "p1_quadrant_2k_shuffled", "p2_vortex"]])
def test_members_match_oracle(names):
    say(f"[gpu case] batch of {names}")
    sols = [member(n) for n in names]
    b = Batch(sols)
    b.step(3)
    for n, s in zip(names, sols):
        k, m, kind, p = _CACHE[n]
        o = oracle.Oracle(m, k)
        o.init_problem(kind, p)
        for _ in range(3):
            assert o.step() == 0
        u, t, step = s.readback()
        e = rel_err(u, o.state(0))
        say(f"{n}: batch vs oracle after 3 steps {e:.2e}")
        assert step == 3 and abs(t - o.scalars()["t"]) <= 1e-13 * max(1.0, t)
        assert e < 1e-11


def test_alone_and_in_mix_bitwise():
    names = list(MEMBERS)
    say(f"[gpu case] mix {names}")
    alone = {}
    for n in names:
        s = member(n)
        b = Batch([s])
        b.step(4)
        alone[n] = s.readback()[0]
        b.close()
    sols = [member(n) for n in names]
    b = Batch(sols[::-1])                # another order as well
    b.step(4)
    for n, s in zip(names, sols):
        assert np.array_equal(s.readback()[0], alone[n]), n


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_schedule_does_not_change_results(precision):
    names = ["p2_quadrant_3k", "p1_quadrant_2k", "p2_two_state_1k", "p2_quadrant_3k_shuffled"]
    ref = None
    for cg, occ in ((1, 100), (8, 100), (3, 50), (16, 25)):
        sols = [member(n, precision) for n in names]
        b = Batch(sols)
        b.set_schedule(cg, occ)
        sch = b.schedule()
        say(f"[gpu case] {precision} schedule {sch}")
        b.step(3)
        out = [s.readback()[0] for s in sols]
        if ref is None:
            ref = out
        else:
            for n, x, y in zip(names, out, ref):
                assert np.array_equal(x, y), (n, cg, occ)


@pytest.mark.parametrize("n", ["p2_quadrant_3k", "p1_quadrant_2k_shuffled"])
def test_batch_matches_single_instance_path(n):
    """dg_step groups its reductions per workgroup, the batch per 256 cells: the two
    agree to round-off."""
    a, b_ = member(n), member(n)
    for _ in range(5):
        a.step()
    B = Batch([b_])
    B.step(5)
    assert rel_err(b_.readback()[0], a.readback()[0]) < 1e-12


def test_members_stop_at_their_own_t_end():
    names = ["p1_vortex", "p2_vortex", "p2_quadrant_3k"]
    t_ends = [0.05, 0.08, 0.002]
    sols = [member(n) for n in names]
    for s, t in zip(sols, t_ends):
        s.set_t_end(t)
    b = Batch(sols)
    steps = b.run(10_000)
    act, st = b.status()
    say(f"batch run: {steps} steps, status {st.tolist()}")
    assert act == 0
    for s, t, n in zip(sols, t_ends, names):
        u, tt, k = s.readback()
        assert abs(tt - t) < 1e-14, (n, tt, t)
        # same as running the instance alone to its t_end
        ref = member(n)
        ref.step_to(t)
        assert ref.readback()[2] == k
        assert rel_err(u, ref.readback()[0]) < 1e-11
    before = [s.readback()[0] for s in sols]
    b.step(2)                            # every member is inactive: nothing changes
    for s, x in zip(sols, before):
        assert np.array_equal(s.readback()[0], x)


def test_autotune_keeps_state_and_results():
    names = ["p2_quadrant_3k", "p1_quadrant_2k", "p2_two_state_1k", "p1_vortex"]
    sols = [member(n) for n in names]
    b = Batch(sols)
    b.step(1)
    before = [s.readback() for s in sols]
    d_before = [s.diag() for s in sols]
    best = b.autotune(reps=2)
    say(f"autotune: {best}")
    assert best["chunk_groups"] in (1, 2, 4, 8, 16) and best["occupancy_pct"] in (50, 100)
    for s, (u, t, k), d in zip(sols, before, d_before):
        u2, t2, k2 = s.readback()
        assert np.array_equal(u, u2) and t == t2 and k == k2
        assert s.diag() == d
    b.step(2)
    ref = [member(n) for n in names]
    rb = Batch(ref)
    rb.step(3)
    for s, r in zip(sols, ref):
        assert np.array_equal(s.readback()[0], r.readback()[0])


def test_sixty_four_uneven_instances():
    """64 members, log-uniform sizes (scaled down 1:100 from 5k-500k), P1/P2 50/50,
    two-state data: every member equals its own single-member batch bit for bit."""
    sizes, degree = workloads.batch_sizes(n_inst=64)
    sizes = np.maximum(sizes // 100, 60)
    insts = [(int(d),) + workloads.batch_instance(i, int(sz)) for i, (sz, d) in enumerate(zip(sizes, degree))]
    say(f"[gpu case] 64 instances, {sum(m.n_cell for _, m, _, _ in insts)} cells")
    sols = []
    for k, m, kind, p in insts:
        s = Solver(m, k)
        s.init_problem(kind, p)
        sols.append(s)
    b = Batch(sols)
    b.autotune(reps=1)
    b.step(3)
    act, st = b.status()
    assert act == 64 and np.all(st[:, 1] == 0) and np.all(st[:, 3] == 3)
    for i in (0, 7, 21, 63):
        k, m, kind, p = insts[i]
        s = Solver(m, k)
        s.init_problem(kind, p)
        one = Batch([s])
        one.step(3)
        assert np.array_equal(s.readback()[0], sols[i].readback()[0]), i


def test_reinitialised_member_is_refused():
    sols = [member("p1_vortex"), member("p2_vortex")]
    b = Batch(sols)
    b.step(1)
    k, m, kind, p = _CACHE["p1_vortex"]
    sols[0].init_problem(kind, p)
    with pytest.raises(DgError) as e:
        b.step(1)
    assert e.value.status == -6
