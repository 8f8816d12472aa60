"""CPU checks of the batch planning (host logic, no device): the chunk table
covers every reduction group of every instance exactly once, and the split gives
each XCD one contiguous range of near-equal estimated cost."""

import ctypes

import numpy as np
import pytest

import paper_2409_09620_amd as pkg
from paper_2409_09620_amd import DgError, binding
from synth import workloads

GROUP = 256


def _cost(n_cell, k, chunks):
    c = []
    for inst, g0, g1 in chunks:
        cells = min(g1 * GROUP, n_cell[inst]) - g0 * GROUP
        c.append(cells * (2.0 if k[inst] == 2 else 1.0))
    return np.array(c)


@pytest.mark.parametrize("chunk_groups", [1, 3, 16])
def test_plan_covers_every_group_once(chunk_groups):
    sizes, degree = workloads.batch_sizes(n_inst=64)
    sizes = sizes // 50 + 1               # same spread, small enough for a quick check
    chunks, split = pkg.plan_chunks(sizes, degree, chunk_groups)
    seen = {}
    for inst, g0, g1 in chunks:
        assert 0 < g1 - g0 <= chunk_groups
        seen.setdefault(int(inst), []).append((int(g0), int(g1)))
    assert sorted(seen) == list(range(len(sizes)))
    for i, runs in seen.items():
        ng = -(-int(sizes[i]) // GROUP)
        assert runs[0][0] == 0 and runs[-1][1] == ng
        assert all(a[1] == b[0] for a, b in zip(runs, runs[1:]))   # contiguous, in order
    # instances appear in order
    assert np.all(np.diff(chunks[:, 0]) >= 0)


def test_split_is_contiguous_and_balanced():
    sizes, degree = workloads.batch_sizes(n_inst=64)
    chunks, split = pkg.plan_chunks(sizes, degree, 4)
    assert split[0] == 0 and split[8] == len(chunks)
    assert np.all(np.diff(split) >= 0)
    cost = _cost(sizes, degree, chunks)
    per_x = np.array([cost[split[x]:split[x + 1]].sum() for x in range(8)])
    # every range is within one chunk of the mean
    assert np.all(np.abs(per_x - cost.sum() / 8) <= cost.max() + 1e-9)


def test_single_small_instance():
    chunks, split = pkg.plan_chunks([10], [2], 1)
    assert chunks.tolist() == [[0, 0, 1]]
    assert split[0] == 0 and split[8] == 1


def test_plan_rejects_bad_input():
    with pytest.raises(DgError):
        pkg.plan_chunks([100, 0], [1, 2], 1)
    with pytest.raises(DgError):
        pkg.plan_chunks([100], [3], 1)
    with pytest.raises(DgError):
        pkg.plan_chunks([100], [1], 0)


def test_batch_and_t_end_need_initialised_contexts():
    L = pkg.load_library()
    h = ctypes.c_void_p()
    assert L.dg_create(ctypes.byref(h), -1, None) == 0
    try:
        arr = (ctypes.c_void_p * 1)(h.value)
        b = ctypes.c_void_p()
        assert L.dg_batch_create(ctypes.byref(b), arr, 1, None) == -6     # DG_E_STATE
        assert b.value is None
        assert L.dg_batch_create(ctypes.byref(b), arr, 0, None) == -1     # DG_E_ARG
        assert L.dg_set_t_end(h, 1.0) == -6
    finally:
        L.dg_destroy(h)
    assert "dg_batch_create" in binding.symbols_declared()
