"""The largest P2 mesh the library takes: DG_MAX_CELLS(2) = 22,369,621 cells, here
22,368,256 (10,922 copies of a 2048-cell periodic jittered-grid block).  One step
(FP64 and the mixed form) of the periodic vortex, given in every copy as the oracle's projected data on
the block, against the oracle's step on the block in every copy (the tiling
property is checked with the oracle alone in test_synth_tiling).  The state buffers'
byte offsets reach 4,294,705,152 of the 4 GiB that the kernels' 32-bit offsets
address."""

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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_largest_p2_mesh_one_step(precision):
    base, kind, p = workloads.periodic_vortex(n=32)
    blocks = binding.max_cells(2) // base.n_cell
    a, b = 86, 127
    assert a * b == blocks and (blocks + 1) * base.n_cell > binding.max_cells(2)
    t0 = time.time()
    big = smesh.tile_periodic_grid(base, a, b)
    say(f"[gpu case] largest P2 mesh, {precision}: {big.n_cell} cells ({blocks} blocks), "
        f"built in {time.time() - t0:.1f} s")
    ob = oracle.Oracle(base, 2)
    assert ob.init_problem(kind, p) == 0
    u0 = ob.state(0)
    s = Solver(big, 2)
    say(f"[gpu case] uploaded at {time.time() - t0:.1f} s")
    s.init_modal(np.tile(u0, (1, 1, blocks)), precision=precision)
    d, so = s.diag(), ob.scalars()
    tol = TOL[precision]
    assert abs(d["alpha"] - so["alpha"]) <= tol * so["alpha"]
    assert abs(d["dt"] - so["dt"]) <= tol * so["dt"]   # also min C|K| from shifted coordinates
    say(f"[gpu case] initialised at {time.time() - t0:.1f} s; one step")
    s.step()
    assert ob.step() == 0
    u, t, step = s.readback()
    say(f"[gpu case] read back at {time.time() - t0:.1f} s")
    assert step == 1 and abs(t - ob.scalars()["t"]) <= tol * ob.scalars()["t"]
    ub = ob.state(0)
    err = 0.0
    for v in range(4):
        scale = np.abs(ub[v]).max()
        for l in range(ub.shape[1]):
            blk = u[v, l].reshape(blocks, base.n_cell)
            err = max(err, np.abs(blk - ub[v, l][None, :]).max() / scale)
    say(f"[gpu case] largest P2 mesh, {precision}: max rel deviation from the block's step {err:.2e}")
    assert err < tol, err
