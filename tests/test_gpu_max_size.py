"""The largest meshes the library takes: DG_MAX_CELLS(2) = 22,369,621 P2 cells, here
22,368,256 (10,922 copies of a 2048-cell periodic jittered-grid block), and
DG_MAX_CELLS(1) = 44,739,242 P1 cells, here 44,738,560 (21,845 copies).  One step
(P2: FP64 and the mixed form; P1: FP64) of the periodic vortex, given in every copy
as the oracle's projected data on the block, against the oracle's step on the
block in every copy (the tiling property is checked with the oracle alone in
test_synth_tiling).  The state buffers' byte offsets reach 4,294,705,152 (P2) and
4,294,901,760 (P1) of the 4 GiB that the kernels' 32-bit offsets address, the
mesh block from |K| (88 B per cell) 3.9 GB at P1."""

import sys
import time

import numpy as np
import pytest

import oracle
from synth import mesh as smesh
from synth import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():   # collected on CPU-only hosts, skipped there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2409_09620_amd import Solver, binding  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


# FP64: the parity bound of a stage; mixed: its FP32 bulk, as in test_gpu_mixed
TOL = {"fp64": 1e-12, "mixed": 50 * 2.0 ** -24}


TILES = {2: (86, 127), 1: (85, 257)}   # a x b = DG_MAX_CELLS(k) // 2048 blocks


@pytest.mark.parametrize("k,precision", [(2, "fp64"), (2, "mixed"), (1, "fp64")])
def test_largest_mesh_one_step(k, precision):
    base, kind, p = workloads.periodic_vortex(n=32)
    blocks = binding.max_cells(k) // base.n_cell
    a, b = TILES[k]
    assert a * b == blocks and (blocks + 1) * base.n_cell > binding.max_cells(k)
    t0 = time.time()
    big = smesh.tile_periodic_grid(base, a, b)
    say(f"[gpu case] largest P{k} mesh, {precision}: {big.n_cell} cells ({blocks} blocks), "
        f"built in {time.time() - t0:.1f} s")
    ob = oracle.Oracle(base, k)
    assert ob.init_problem(kind, p) == 0
    u0 = ob.state(0)
    s = Solver(big, k)
    say(f"[gpu case] uploaded at {time.time() - t0:.1f} s")
    s.init_modal(np.tile(u0, (1, 1, blocks)), precision=precision)
    d, so = s.diag(), ob.scalars()
    tol = TOL[precision]
    assert abs(d["alpha"] - so["alpha"]) <= tol * so["alpha"]
    # min C|K| comes from coordinates shifted by up to 10 max(a, b): their rounding,
    # relative to the cell size h, bounds how far it moves
    geo = 8 * 2.0 ** -52 * 10.0 * max(a, b) / base.meta["h"]
    assert abs(d["dt"] - so["dt"]) <= max(tol, geo) * so["dt"], (d["dt"], so["dt"], geo)
    say(f"[gpu case] initialised at {time.time() - t0:.1f} s; one step")
    s.step()
    assert ob.step() == 0
    u, t, step = s.readback()
    say(f"[gpu case] read back at {time.time() - t0:.1f} s")
    assert step == 1 and abs(t - ob.scalars()["t"]) <= max(tol, geo) * ob.scalars()["t"]
    ub = ob.state(0)
    err = 0.0
    for v in range(4):
        scale = np.abs(ub[v]).max()
        for l in range(ub.shape[1]):
            blk = u[v, l].reshape(blocks, base.n_cell)
            err = max(err, np.abs(blk - ub[v, l][None, :]).max() / scale)
    say(f"[gpu case] largest P{k} mesh, {precision}: max rel deviation from the block's step {err:.2e}")
    s.close()
    assert err < tol, err
