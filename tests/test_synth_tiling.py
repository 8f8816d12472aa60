"""The periodic tiling that the largest-mesh GPU test runs on, checked with the
oracle alone: on a x b copies of a periodic jittered-grid block, data that are the
block's data in every copy step to the block's step in every copy (the method is
local and translation invariant, and its global scalars are the same maxima and
sums), up to the rounding of coordinates shifted by whole periods."""

import numpy as np

import oracle
from synth import mesh as smesh
from synth import workloads


def test_tiling_tables():
    base = smesh.periodic_jittered_grid(n=8, seed=3)
    big = smesh.tile_periodic_grid(base, 3, 2)
    assert big.n_cell == 6 * base.n_cell and big.n_vert == 6 * base.n_vert
    cxy = big.cell_xy.reshape(6, base.n_cell, 3, 2)
    for q in range(6):
        shift = np.array([(q % 3) * 10.0, (q // 3) * 10.0])
        assert np.array_equal(cxy[q], base.cell_xy.reshape(-1, 3, 2) + shift)
    # every vertex id resolves to the cell's own (wrapped) corner
    L = np.array([30.0, 20.0])
    d = (big.xy[big.tri] - big.cell_xy.reshape(-1, 3, 2)) / L
    assert np.abs(d - np.rint(d)).max() < 1e-12
    # every edge is shared by exactly two cells (a closed periodic surface)
    e = np.sort(np.stack([big.tri[:, [1, 2]], big.tri[:, [2, 0]], big.tri[:, [0, 1]]], axis=1).reshape(-1, 2), axis=1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    assert (cnt == 2).all()


def test_tiled_step_is_the_block_step():
    base, kind, p = workloads.periodic_vortex(n=8)
    big = smesh.tile_periodic_grid(base, 3, 2)
    ob = oracle.Oracle(base, 2)
    assert ob.init_problem(kind, p) == 0
    u0 = ob.state(0)
    ot = oracle.Oracle(big, 2)
    assert ot.init_modal(np.tile(u0, (1, 1, 6))) == 0
    assert ob.step() == 0 and ot.step() == 0
    ub = ob.state(0)
    ut = ot.state(0).reshape(4, 6, 6, base.n_cell)
    scale = np.abs(ub).max(axis=(1, 2))
    err = (np.abs(ut - ub[:, :, None, :]).max(axis=(1, 2, 3)) / scale).max()
    assert err < 1e-12, err
    assert abs(ot.scalars()["t"] - ob.scalars()["t"]) < 1e-15
