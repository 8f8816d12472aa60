"""FP64 CPU oracle of the BP RI-OEDG stage (TEST INFRASTRUCTURE ONLY).

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py`
may import this package.  The HIP library never links, loads or calls it, and the
two share no code.  The arithmetic lives in `oedg_oracle.c` (plain C, compiled
with -ffp-contract=off); this module only marshals numpy arrays.

State arrays use the layout [var rho,m1,m2,E][mode][cell] (float64), the same
layout as the C-ABI of the HIP library.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oedg_oracle.c")
_SO = os.path.join(_HERE, "_liboracle.so")
_lib = None

_D = ctypes.c_double
_I = ctypes.c_int
_L = ctypes.c_long
_P = ctypes.c_void_p


def build(force: bool = False) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=gnu11", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        sig = {
            "orc_create": (_P, [_I, _I, _P, _I, _P, _P]),
            "orc_set_threads": (_I, [_I]),
            "orc_destroy": (None, [_P]),
            "orc_export_mesh": (_I, [_P] + [_P] * 11),
            "orc_config": (_I, [_P, _D, _D, _I, _I, _I]),
            "orc_init_modal": (_I, [_P, _P]),
            "orc_init_problem": (_I, [_P, _I, _P]),
            "orc_start": (_I, [_P]),
            "orc_stage": (_I, [_P, _I]),
            "orc_step": (_I, [_P]),
            "orc_finish_step": (_I, [_P]),
            "orc_run": (_I, [_P, _D, _L, _P]),
            "orc_get_state": (_I, [_P, _I, _P]),
            "orc_get_scalars": (_I, [_P, _P]),
            "orc_set_time": (_I, [_P, _D, _D, _D, _L]),
            "orc_set_max_restarts": (_I, [_P, _I]),
            "orc_apply_residual": (_I, [_P, _P, _D, _P]),
            "orc_apply_oe": (_I, [_P, _P, _D]),
            "orc_apply_limiter": (_I, [_P, _P]),
            "orc_alpha_of": (_D, [_P, _P]),
            "orc_limiter_node_values": (_I, [_P, _P, _P]),
            "orc_mass": (_I, [_P, _P]),
            "orc_basis": (None, [_D, _D, _P, _P, _P]),
            "orc_quadrature": (_I, [_I, _P, _P]),
            "orc_decompose": (_I, [_I, _P, _P, _P, _P, _P, _P]),
            "orc_set_bc": (_I, [_P, _P]),
            "orc_set_decomp": (_I, [_P, _I]),
            "orc_set_limiter_form": (_I, [_P, _I]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


SCALARS = ["t", "dt", "alpha", "step", "active", "err", "n_limited", "minck",
           "ubar_rho", "ubar_m1", "ubar_m2", "ubar_E",
           "nrm_rho", "nrm_m1", "nrm_m2", "nrm_E", "nrm_m", "zero_rho", "zero_E", "zero_m", "n_restarts"]


class Oracle:
    """One mesh and state in the FP64 oracle."""

    def __init__(self, mesh, k, gamma=1.4, cssp=1.0, oe=True, bp=True, oe_mode=0, max_restarts=8,
                 decomposition="dcw", edge_bc=None, limiter_form="nodes"):
        """decomposition: "dcw" (the optimal one) or "zxs" (the classical one) for the
        limiter and Delta t; edge_bc: (n_cell, 3) tags of boundary edges, the edge
        opposite input vertex i (0 transmissive, 1 reflective), default from
        mesh.edge_bc; limiter_form: "nodes" (the optimal decomposition's nodes) or
        "ustar" (P2: the u* form of Sec. 4.4 with the optimal edge weights)."""
        self.k = int(k)
        self.nm = (k + 1) * (k + 2) // 2
        self.nc = mesh.n_cell
        xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
        tri = np.ascontiguousarray(mesh.tri, dtype=np.int32)
        cxy = None if mesh.cell_xy is None else np.ascontiguousarray(mesh.cell_xy, dtype=np.float64)
        h = lib().orc_create(self.k, mesh.n_vert, _ptr(xy), self.nc, _ptr(tri), _ptr(cxy))
        if not h:
            raise ValueError("oracle: invalid mesh")
        self.h = h
        lib().orc_config(h, gamma, cssp, int(oe), int(bp), int(oe_mode))
        lib().orc_set_max_restarts(h, int(max_restarts))
        if edge_bc is None:
            edge_bc = getattr(mesh, "edge_bc", None)
        if edge_bc is not None:
            bc = np.ascontiguousarray(edge_bc, dtype=np.int32).reshape(self.nc, 3)
            if lib().orc_set_bc(h, _ptr(bc)) != 0:
                raise ValueError("oracle: boundary tags must be 0 or 1")
        if decomposition not in ("dcw", "zxs"):
            raise ValueError("decomposition is 'dcw' or 'zxs'")
        lib().orc_set_decomp(h, 1 if decomposition == "zxs" else 0)
        if limiter_form not in ("nodes", "ustar"):
            raise ValueError("limiter_form is 'nodes' or 'ustar'")
        lib().orc_set_limiter_form(h, 1 if limiter_form == "ustar" else 0)

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "h", None) and callable(lib):
            lib().orc_destroy(self.h)
            self.h = None

    # ---------------------------------------------------------------- mesh
    def mesh_arrays(self):
        nc = self.nc
        out = dict(tri=np.zeros((nc, 3), np.int32), nbr=np.zeros((nc, 3), np.int32),
                   nbe=np.zeros((nc, 3), np.int32), perm=np.zeros((nc, 3), np.int32),
                   limv=np.zeros((nc, 2), np.int32), area=np.zeros(nc), len=np.zeros((nc, 3)),
                   nrm=np.zeros((nc, 3, 2)), node=np.zeros((nc, 2, 2)), ck=np.zeros(nc))
        minck = np.zeros(1)
        lib().orc_export_mesh(self.h, *[_ptr(out[k]) for k in
                                        ("tri", "nbr", "nbe", "perm", "limv", "area", "len", "nrm",
                                         "node", "ck")], _ptr(minck))
        out["minck"] = float(minck[0])
        return out

    def mass(self):
        m = np.zeros((self.nc, self.nm))
        lib().orc_mass(self.h, _ptr(m))
        return m

    # ---------------------------------------------------------------- state
    def shape(self):
        return (4, self.nm, self.nc)

    def init_problem(self, kind, params):
        p = np.ascontiguousarray(params, dtype=np.float64)
        lib().orc_init_problem(self.h, int(kind), _ptr(p))
        return lib().orc_start(self.h)

    def init_modal(self, u, limit=True):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape())
        lib().orc_init_modal(self.h, _ptr(u))
        return lib().orc_start(self.h)

    def state(self, which=0):
        out = np.zeros(self.shape())
        lib().orc_get_state(self.h, int(which), _ptr(out))
        return out

    def scalars(self):
        s = np.zeros(len(SCALARS))
        lib().orc_get_scalars(self.h, _ptr(s))
        return dict(zip(SCALARS, s.tolist()))

    def set_time(self, t, dt, alpha, step=0):
        lib().orc_set_time(self.h, t, dt, alpha, int(step))

    def stage(self, s):
        return lib().orc_stage(self.h, int(s))

    def step(self):
        return lib().orc_step(self.h)

    def finish_step(self):
        """Bookkeeping that ends a step run stage by stage (u^n, t, alpha, Delta t)."""
        return lib().orc_finish_step(self.h)

    def run(self, t_end=float("inf"), max_steps=1 << 62):
        done = ctypes.c_long(0)
        r = lib().orc_run(self.h, float(t_end), int(max_steps), ctypes.byref(done))
        return r, done.value

    # ---------------------------------------------------------------- building blocks
    def residual(self, u, alpha):
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros(self.shape())
        lib().orc_apply_residual(self.h, _ptr(u), float(alpha), _ptr(out))
        return out

    def oe(self, u, dt):
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        lib().orc_apply_oe(self.h, _ptr(u), float(dt))
        return u

    def limit(self, u):
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        bad = lib().orc_apply_limiter(self.h, _ptr(u))
        return u, bad

    def alpha_of(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        return lib().orc_alpha_of(self.h, _ptr(u))

    def limiter_node_values(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        npt = 8 if self.k == 1 else 11
        out = np.zeros((self.nc, npt, 4))
        lib().orc_limiter_node_values(self.h, _ptr(u), _ptr(out))
        return out


def basis(xi, eta):
    p, dx, de = np.zeros(6), np.zeros(6), np.zeros(6)
    lib().orc_basis(float(xi), float(eta), _ptr(p), _ptr(dx), _ptr(de))
    return p, dx, de


def quadrature(which):
    pts, w = np.zeros(36), np.zeros(12)
    n = lib().orc_quadrature(int(which), _ptr(pts), _ptr(w))
    if which <= 2:
        return pts[:3 * n].reshape(n, 3), w[:n]
    return pts[:n], w[:n]


def decompose(k, v):
    """Optimal decomposition of one triangle v (3,2): edge weights in sorted order,
    internal nodes (2,2), node weights, C^DCW, and the sorted edge order."""
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(6)
    w, nodes, nw, cd = np.zeros(3), np.zeros(4), np.zeros(2), np.zeros(1)
    perm = np.zeros(3, np.int32)
    lib().orc_decompose(int(k), _ptr(v), _ptr(w), _ptr(nodes), _ptr(nw), _ptr(cd), _ptr(perm))
    return w, nodes.reshape(2, 2), nw, float(cd[0]), perm


def set_threads(n):
    """Threads of the oracle's cell loops, n <= 0 for one per processor (results
    are bit for bit those of one thread); returns the number in use."""
    return int(lib().orc_set_threads(int(n)))
