"""CPU checks of the HIP library: it loads, exports every declared symbol, and its
host-side mesh precompute matches the oracle's (integer tables bit for bit)."""

import ctypes
import os

import numpy as np
import pytest

import oracle
import paper_2409_09620_amd as pkg
from paper_2409_09620_amd import binding
from synth import mesh as smesh
from synth import workloads


def test_library_exports_every_declared_symbol():
    L = pkg.load_library()
    names = pkg.symbols_declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_workspace_bytes():
    L = pkg.load_library()
    b1, b2 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.dg_workspace_bytes(1000, 1, ctypes.byref(b1)) == 0
    assert L.dg_workspace_bytes(1000, 2, ctypes.byref(b2)) == 0
    # three state buffers of 4 (L+1) doubles plus geometry per cell
    assert b2.value > b1.value > 1000 * 8 * (3 * 12)
    assert L.dg_workspace_bytes(0, 1, ctypes.byref(b1)) == -1
    assert L.dg_workspace_bytes(10, 3, ctypes.byref(b1)) == -1


def test_size_limit():
    """DG_MAX_CELLS(k) cells are accepted, one more is refused before any array is read."""
    L = pkg.load_library()
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                             "oedg.h")).read()
    assert "#define DG_MAX_CELLS(k) ((int32_t)(0xffffffffu / (32u * (unsigned)(((k) + 1) * ((k) + 2) / 2))))" in text
    b = ctypes.c_size_t(0)
    for k, n_max in ((1, 44_739_242), (2, 22_369_621)):
        assert binding.max_cells(k) == n_max
        assert n_max * 32 * ((k + 1) * (k + 2) // 2) < 2 ** 32 <= (n_max + 1) * 32 * ((k + 1) * (k + 2) // 2)
        assert L.dg_workspace_bytes(n_max, k, ctypes.byref(b)) == 0
        assert L.dg_workspace_bytes(n_max + 1, k, ctypes.byref(b)) == -1
    h = ctypes.c_void_p()
    assert L.dg_create(ctypes.byref(h), -1, None) == 0
    n = binding.max_cells(2) + 1
    tri = np.zeros((n, 3), np.int32)
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    assert L.dg_mesh_upload(h, 2, 3, binding._ptr(xy), n, binding._ptr(tri), None, None) == -1
    assert b"too large" in L.dg_last_error(h)
    L.dg_destroy(h)


def _meshes():
    return [("periodic", smesh.periodic_jittered_grid(n=7, seed=4)),
            ("delaunay", smesh.poisson_delaunay(900, seed=12)),
            ("blast", workloads.blast_delaunay(n_cells=700, seed=5)[0])]


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("idx", [0, 1, 2])
def test_host_mesh_tables_match_oracle(k, idx):
    name, m = _meshes()[idx]
    lib = pkg.host_mesh_tables(m, k)
    o = oracle.Oracle(m, k).mesh_arrays()
    for key in ("tri", "nbr", "nbe", "perm"):
        assert np.array_equal(lib[key], o[key]), key
    # same length formula in both codes: C^DCW |K| agrees to the last bits
    assert np.abs(lib["ck"] - o["ck"]).max() <= 4e-16 * np.abs(o["ck"]).max()
    assert abs(lib["minck"] - o["minck"]) <= 4e-16 * o["minck"]
    # limiter points: P1 the vertices opposite the two longest edges, P2 the oracle's
    # internal nodes (physical) mapped to reference coordinates of the oriented cell
    ref_v = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    if k == 1:
        for s in range(2):
            want = ref_v[o["limv"][:, s]]
            assert np.array_equal(lib["node_ref"][2 * s], want[:, 0])
            assert np.array_equal(lib["node_ref"][2 * s + 1], want[:, 1])
        return
    V = m.cell_coords()
    Vo = np.empty_like(V)
    for c in range(m.n_cell):
        for q in range(3):
            src = int(np.nonzero(m.tri[c] == o["tri"][c, q])[0][0])
            Vo[c, q] = V[c, src]
    J = np.stack([Vo[:, 1] - Vo[:, 0], Vo[:, 2] - Vo[:, 0]], axis=2)   # columns
    for s in range(2):
        d = o["node"][:, s, :] - Vo[:, 0]
        ref = np.linalg.solve(J, d[..., None])[..., 0]
        assert np.abs(lib["node_ref"][2 * s] - ref[:, 0]).max() < 1e-12
        assert np.abs(lib["node_ref"][2 * s + 1] - ref[:, 1]).max() < 1e-12


def test_host_mesh_errors():
    L = pkg.load_library()
    good = smesh.poisson_delaunay(60, seed=1)

    def upload(xy, tri, k=1):
        h = ctypes.c_void_p()
        assert L.dg_create(ctypes.byref(h), -1, None) == 0
        xy = np.ascontiguousarray(xy, np.float64)
        tri = np.ascontiguousarray(tri, np.int32)
        st = L.dg_mesh_upload(h, k, len(xy), binding._ptr(xy), len(tri), binding._ptr(tri), None, None)
        msg = L.dg_last_error(h)
        # device calls on a host-only context are refused
        st2 = L.dg_stage(h, 0)
        L.dg_destroy(h)
        return st, msg, st2

    assert upload(good.xy, good.tri)[0] == 0
    assert upload(good.xy, good.tri)[2] == -6
    bad = good.tri.copy()
    bad[3, 1] = len(good.xy) + 5
    assert upload(good.xy, bad)[0] == -2                      # vertex id out of range
    deg = good.tri.copy()
    deg[0, 2] = deg[0, 1]
    assert upload(good.xy, deg)[0] == -2                      # zero-area cell
    assert upload(good.xy, good.tri, k=3)[0] == -1            # bad degree
    assert upload(good.xy, np.zeros((0, 3)))[0] == -2         # no cells
    nm = np.concatenate([good.tri, good.tri[:1]])             # duplicated cell: non-manifold edges
    assert upload(good.xy, nm)[0] == -2


def test_product_path_has_no_fallback():
    """The binding loads only the built HIP library and never the oracle."""
    import inspect
    src = inspect.getsource(binding)
    assert "oracle" not in src.replace("never the oracle", "")
    assert "import torch" in src


def test_config_defaults_and_layout():
    """dg_config_default fills the binding's mirror of dg_config field by field."""
    L = pkg.load_library()
    c = binding.DgConfig()
    c.decomposition = 7
    c.limiter_form = 7
    L.dg_config_default(ctypes.byref(c))
    assert (c.k, c.oe_enable, c.oe_mode, c.bp_enable, c.precision) == (2, 1, 0, 1, 0)
    assert c.gamma == 1.4 and c.c_ssp == 1.0 and c.max_restarts == 8
    assert c.decomposition == binding.DG_DECOMP_DCW
    assert c.limiter_form == binding.DG_LIMITER_NODES   # the last field: the layouts agree
    assert ctypes.sizeof(binding.DgConfig) == 56


def test_boundary_tags_are_checked():
    L = pkg.load_library()
    m = smesh.poisson_delaunay(80, seed=3)
    walls = workloads.wall_tags(m, lambda x, y: y == 0.0)
    assert walls.sum() > 0

    def upload(tags):
        h = ctypes.c_void_p()
        assert L.dg_create(ctypes.byref(h), -1, None) == 0
        xy = np.ascontiguousarray(m.xy, np.float64)
        tri = np.ascontiguousarray(m.tri, np.int32)
        t = np.ascontiguousarray(tags, np.int32)
        st = L.dg_mesh_upload(h, 2, len(xy), binding._ptr(xy), len(tri), binding._ptr(tri), None, binding._ptr(t))
        L.dg_destroy(h)
        return st

    assert upload(walls) == 0
    assert upload(np.ones_like(walls)) == 0        # tags of shared edges are ignored
    bad = walls.copy()
    bad[np.nonzero(walls)[0][0], np.nonzero(walls)[1][0]] = 2
    assert upload(bad) == -1
    inner = np.full_like(walls, 5)
    inner[walls.astype(bool)] = 0                  # unknown tags on shared edges only
    onb = workloads.wall_tags(m, lambda x, y: (x == 0) | (x == 1) | (y == 0) | (y == 1)).astype(bool)
    inner[onb] = 0
    assert upload(inner) == 0


def test_header_constants_match_the_binding():
    """Every DG_ enum constant of include/oedg.h has the same value in the binding."""
    import re
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                             "oedg.h")).read()
    consts = dict((n, int(v)) for n, v in re.findall(r"\b(DG_[A-Z0-9_]+)\s*=\s*(-?\d+)", text))
    assert len(consts) >= 17
    for name, val in consts.items():
        if name.startswith("DG_E_") or name == "DG_OK":
            assert binding.STATUS[val] == name
        else:
            assert getattr(binding, name) == val, name


def test_library_loads_after_torch_in_a_fresh_process():
    """The serving admission check sizes a request through the library before any
    solver exists; the library must still come up on torch's HIP runtime, the only
    one mapped into the process (a second runtime sees no device)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2409_09620_amd.serving import footprint_bytes\n"
            "assert 'torch' not in sys.modules\n"
            "assert footprint_bytes(1000, 2) > 0\n"
            "assert 'torch' in sys.modules\n"
            "hip = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "assert len(hip) == 1 and 'torch' in next(iter(hip)), hip\n" % root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]


@pytest.mark.parametrize("maker", ["quadrant", "periodic"])
def test_host_precompute_on_many_tiles(maker):
    """The precompute of a mesh of many 256-cell tiles: the library checks its own
    tables as it builds them (each edge inside a tile owned by exactly one of its two
    cells for the filter's edge work, at most two owned inside the tile per cell) and
    fails the upload if they do not hold; the integer tables still match the oracle."""
    if maker == "quadrant":
        m = workloads.quadrant_delaunay(20_000)[0]
    else:
        m = smesh.periodic_jittered_grid(n=64, seed=9)
    lib = pkg.host_mesh_tables(m, 2)
    o = oracle.Oracle(m, 2).mesh_arrays()
    for key in ("nbr", "nbe"):
        assert np.array_equal(lib[key], o[key]), key
