"""ctypes binding of the C ABI in include/oedg.h (argument marshalling only).

Every stage step runs in the HIP library; this module never computes any part
of the method.  If the library is not built, loading fails loudly.
"""

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_LIB = os.path.join(_HERE, "_lib", "liboedg.so")
_HEADER = os.path.join(_ROOT, "include", "oedg.h")

DG_OE_RI = 0
DG_OE_CW = 1
DG_PREC_FP64 = 0
DG_PREC_MIXED = 1
PRECISION = {"fp64": DG_PREC_FP64, "mixed": DG_PREC_MIXED}
DG_DECOMP_DCW = 0
DG_DECOMP_ZXS = 1
DECOMPOSITION = {"dcw": DG_DECOMP_DCW, "zxs": DG_DECOMP_ZXS}
DG_LIMITER_NODES = 0
DG_LIMITER_USTAR = 1
LIMITER_FORM = {"nodes": DG_LIMITER_NODES, "ustar": DG_LIMITER_USTAR}
DG_BC_TRANSMISSIVE = 0
DG_BC_REFLECTIVE = 1


def max_cells(k):
    """DG_MAX_CELLS(k): the largest mesh at degree k (its FP64 state buffer of
    4 (k+1)(k+2)/2 doubles per cell stays below 4 GiB)."""
    return 0xFFFFFFFF // (32 * ((k + 1) * (k + 2) // 2))


STATUS = {0: "DG_OK", -1: "DG_E_ARG", -2: "DG_E_MESH", -3: "DG_E_NOMEM", -4: "DG_E_HIP",
          -5: "DG_E_BOUNDS", -6: "DG_E_STATE"}

_lib = None
_c_d, _c_i, _c_p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
_c_i32, _c_i64, _c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t


class DgConfig(ctypes.Structure):
    _fields_ = [("k", _c_i), ("gamma", _c_d), ("c_ssp", _c_d), ("oe_enable", _c_i),
                ("oe_mode", _c_i), ("bp_enable", _c_i), ("precision", _c_i), ("max_restarts", _c_i),
                ("decomposition", _c_i), ("limiter_form", _c_i)]


class DgDiag(ctypes.Structure):
    _fields_ = [("t", _c_d), ("dt", _c_d), ("alpha", _c_d), ("step", _c_i64),
                ("n_limited", _c_i64), ("n_bad", _c_i64), ("n_cfl_excursions", _c_i64),
                ("ubar", _c_d * 4), ("nrm", _c_d * 4), ("nrm_m", _c_d), ("active", _c_i),
                ("n_flat", _c_i64), ("n_restarts", _c_i64), ("alpha_stage", _c_d),
                ("min_rho_node", _c_d), ("min_p_node", _c_d)]


class DgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _edge_tags(mesh, nc):
    """mesh.edge_bc as the (n_cell, 3) int32 array of dg_mesh_upload, or None."""
    bc = getattr(mesh, "edge_bc", None)
    return None if bc is None else np.ascontiguousarray(bc, dtype=np.int32).reshape(nc, 3)


def lib_path():
    return _LIB


def symbols_declared():
    """Names of the functions declared in include/oedg.h."""
    text = open(_HEADER).read()
    return sorted(set(re.findall(r"\b(dg_[a-z_]+)\s*\(", text)))


_SIGS = {
    "dg_config_default": (None, [_c_p]),
    "dg_create": (_c_i, [_c_p, _c_i, _c_p]),
    "dg_workspace_bytes": (_c_i, [_c_i32, _c_i, _c_p]),
    "dg_bind_workspace": (_c_i, [_c_p, _c_p, _c_sz]),
    "dg_mesh_upload": (_c_i, [_c_p, _c_i, _c_i32, _c_p, _c_i32, _c_p, _c_p, _c_p]),
    "dg_mesh_tables": (_c_i, [_c_p] * 8),
    "dg_init": (_c_i, [_c_p, _c_p, _c_p]),
    "dg_init_problem": (_c_i, [_c_p, _c_p, _c_i, _c_p, _c_i]),
    "dg_stage": (_c_i, [_c_p, _c_i]),
    "dg_stage_noalloc": (_c_i, [_c_p, _c_i]),
    "dg_step": (_c_i, [_c_p, _c_p]),
    "dg_step_to": (_c_i, [_c_p, _c_d, _c_i64, _c_p]),
    "dg_readback": (_c_i, [_c_p, _c_p, _c_p, _c_p]),
    "dg_read_state": (_c_i, [_c_p, _c_i, _c_p]),
    "dg_diag": (_c_i, [_c_p, _c_p]),
    "dg_sizes": (_c_i, [_c_p, _c_p, _c_p, _c_p]),
    "dg_profile_enable": (_c_i, [_c_p, _c_i]),
    "dg_profile_read": (_c_i, [_c_p, _c_p, _c_p]),
    "dg_last_error": (ctypes.c_char_p, [_c_p]),
    "dg_destroy": (None, [_c_p]),
    "dg_set_t_end": (_c_i, [_c_p, _c_d]),
    "dg_batch_create": (_c_i, [_c_p, _c_p, _c_i, _c_p]),
    "dg_batch_set_schedule": (_c_i, [_c_p, _c_i, _c_i]),
    "dg_batch_get_schedule": (_c_i, [_c_p, _c_p, _c_p, _c_p, _c_p]),
    "dg_batch_autotune": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_p]),
    "dg_batch_step": (_c_i, [_c_p, _c_i64]),
    "dg_batch_run": (_c_i, [_c_p, _c_i64, _c_p]),
    "dg_batch_status": (_c_i, [_c_p, _c_p, _c_p]),
    "dg_plan_chunks": (_c_i, [_c_i, _c_p, _c_p, _c_i, _c_p, _c_i, _c_p, _c_p]),
    "dg_batch_last_error": (ctypes.c_char_p, [_c_p]),
    "dg_batch_destroy": (None, [_c_p]),
}


def load_library():
    """Loads the built HIP library (no fallback: raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"HIP library {_LIB} is not built; run __graft_entry__.build()")
        # torch first: its HIP runtime then satisfies the library's libamdhip64
        # dependency, so the process holds one runtime, the one that owns the
        # workspace and the streams.  Loaded the other way round, the library
        # binds a second runtime, which finds no device once torch's has the GPU.
        import torch  # noqa: F401
        L = ctypes.CDLL(_LIB)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class Solver:
    """One mesh and state on one GPU.

    mesh: object with xy (n_vert,2) float64, tri (n_cell,3) int32 and optional
    cell_xy (n_cell,6); k: degree 1 or 2.  Device memory comes from a torch
    tensor bound as the library's workspace, and work runs on torch's current
    stream of `device`.
    """

    def __init__(self, mesh, k, device=0, torch_workspace=True):
        import torch
        L = load_library()
        self.k = int(k)
        self.nm = (self.k + 1) * (self.k + 2) // 2
        self.nc = int(mesh.tri.shape[0])
        self.device = int(device)
        self._torch = torch
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = L.dg_create(ctypes.byref(h), self.device, ctypes.c_void_p(self.stream.cuda_stream))
        if st != 0:
            raise DgError(st, "dg_create failed")
        self.h = h
        self._ws = None
        if torch_workspace and self.nc > 0:
            nbytes = ctypes.c_size_t(0)
            self._check(L.dg_workspace_bytes(self.nc, self.k, ctypes.byref(nbytes)))
            self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
            base = self._ws.data_ptr()
            aligned = (base + 255) & ~255
            self._check(L.dg_bind_workspace(self.h, ctypes.c_void_p(aligned), nbytes.value))
        xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
        tri = np.ascontiguousarray(mesh.tri, dtype=np.int32)
        cxy = getattr(mesh, "cell_xy", None)
        cxy = None if cxy is None else np.ascontiguousarray(cxy, dtype=np.float64)
        bc = _edge_tags(mesh, self.nc)
        self._check(L.dg_mesh_upload(self.h, self.k, int(xy.shape[0]), _ptr(xy), self.nc, _ptr(tri),
                                     _ptr(cxy), _ptr(bc)))

    # ------------------------------------------------------------------ plumbing
    def _check(self, st):
        if st != 0:
            msg = load_library().dg_last_error(self.h)
            raise DgError(st, msg.decode() if msg else "")
        return st

    def close(self):
        if getattr(self, "h", None):
            load_library().dg_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def config(self, oe=True, bp=True, oe_mode=DG_OE_RI, gamma=1.4, c_ssp=1.0, precision="fp64", max_restarts=8,
               decomposition="dcw", limiter_form="nodes"):
        """precision: "fp64" or "mixed" (FP32 bulk, FP64 averages and limiter);
        max_restarts: retries (each with half the time step) of a step whose stage
        leaves the admissible set; decomposition: "dcw" (optimal) or "zxs"
        (classical) for the limiter's node set and the time step; limiter_form:
        "nodes" or "ustar" (P2 with the optimal decomposition: the u* form)."""
        cfg = DgConfig()
        load_library().dg_config_default(ctypes.byref(cfg))
        cfg.k = self.k
        cfg.gamma = gamma
        cfg.c_ssp = c_ssp
        cfg.oe_enable = int(oe)
        cfg.bp_enable = int(bp)
        cfg.oe_mode = int(oe_mode)
        if precision not in PRECISION:
            raise ValueError(f"precision must be one of {sorted(PRECISION)}")
        cfg.precision = PRECISION[precision]
        cfg.max_restarts = int(max_restarts)
        if decomposition not in DECOMPOSITION:
            raise ValueError(f"decomposition must be one of {sorted(DECOMPOSITION)}")
        cfg.decomposition = DECOMPOSITION[decomposition]
        if limiter_form not in LIMITER_FORM:
            raise ValueError(f"limiter_form must be one of {sorted(LIMITER_FORM)}")
        cfg.limiter_form = LIMITER_FORM[limiter_form]
        return cfg

    def shape(self):
        return (4, self.nm, self.nc)

    # ------------------------------------------------------------------ API
    def init_problem(self, kind, params, **cfg):
        p = np.ascontiguousarray(params, dtype=np.float64)
        c = self.config(**cfg)
        self._check(load_library().dg_init_problem(self.h, ctypes.byref(c), int(kind), _ptr(p), len(p)))

    def init_modal(self, u, **cfg):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape())
        c = self.config(**cfg)
        self._check(load_library().dg_init(self.h, ctypes.byref(c), _ptr(u)))

    def stage(self, s):
        self._check(load_library().dg_stage(self.h, int(s)))

    def stage_noalloc(self, s):
        """dg_stage with the partial records in the library's device array
        (no device memory of its own; calls overlapping on one GPU race)."""
        self._check(load_library().dg_stage_noalloc(self.h, int(s)))

    def set_t_end(self, t_end):
        """Stop time of this instance's run (also when stepped inside a Batch)."""
        self._check(load_library().dg_set_t_end(self.h, float(t_end)))

    def step(self, want_dt=False):
        dt = ctypes.c_double(0)
        self._check(load_library().dg_step(self.h, ctypes.byref(dt) if want_dt else None))
        return dt.value if want_dt else None

    def step_to(self, t_end=float("inf"), max_steps=(1 << 62)):
        n = ctypes.c_int64(0)
        self._check(load_library().dg_step_to(self.h, float(t_end), int(max_steps), ctypes.byref(n)))
        return n.value

    def readback(self):
        """(u^n, t, step).  After DG_E_BOUNDS the library still copies the state it
        kept (the u^n of the failed step), and so does this."""
        u = np.zeros(self.shape())
        t = ctypes.c_double(0)
        s = ctypes.c_int64(0)
        st = load_library().dg_readback(self.h, _ptr(u), ctypes.byref(t), ctypes.byref(s))
        if st != -5:
            self._check(st)
        return u, t.value, s.value

    def read_state(self, which):
        u = np.zeros(self.shape())
        self._check(load_library().dg_read_state(self.h, int(which), _ptr(u)))
        return u

    def diag(self):
        d = DgDiag()
        self._check(load_library().dg_diag(self.h, ctypes.byref(d)))
        out = {k: getattr(d, k) for k, _ in DgDiag._fields_}
        out["ubar"] = list(d.ubar)
        out["nrm"] = list(d.nrm)
        return out

    KERNELS = ("residual", "filter")   # dg_profile_read's order (DG_PROFILE_KERNELS)

    def profile(self, enable=True):
        self._check(load_library().dg_profile_enable(self.h, int(enable)))

    def profile_read(self):
        """{kernel: (total_ms, launches)} since the last read (synchronises)."""
        ms = np.zeros(len(self.KERNELS))
        n = np.zeros(len(self.KERNELS), np.int64)
        self._check(load_library().dg_profile_read(self.h, _ptr(ms), _ptr(n)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.KERNELS)}

    def mesh_tables(self):
        nc = self.nc
        out = dict(tri=np.zeros((nc, 3), np.int32), nbr=np.zeros((nc, 3), np.int32),
                   nbe=np.zeros((nc, 3), np.int32), perm=np.zeros((nc, 3), np.int32),
                   node_ref=np.zeros((4, nc)), ck=np.zeros(nc))
        minck = ctypes.c_double(0)
        self._check(load_library().dg_mesh_tables(
            self.h, _ptr(out["tri"]), _ptr(out["nbr"]), _ptr(out["nbe"]), _ptr(out["perm"]),
            _ptr(out["node_ref"]), _ptr(out["ck"]), ctypes.byref(minck)))
        out["minck"] = minck.value
        return out


def host_mesh_tables(mesh, k):
    """Mesh tables built by the library's host precompute, through a host-only
    context (no device needed)."""
    L = load_library()
    h = ctypes.c_void_p()
    st = L.dg_create(ctypes.byref(h), -1, None)
    if st != 0:
        raise DgError(st, "dg_create(DG_HOST_ONLY) failed")
    try:
        xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
        tri = np.ascontiguousarray(mesh.tri, dtype=np.int32)
        cxy = getattr(mesh, "cell_xy", None)
        cxy = None if cxy is None else np.ascontiguousarray(cxy, dtype=np.float64)
        nc = int(tri.shape[0])
        bc = _edge_tags(mesh, nc)
        st = L.dg_mesh_upload(h, int(k), int(xy.shape[0]), _ptr(xy), nc, _ptr(tri), _ptr(cxy), _ptr(bc))
        if st != 0:
            raise DgError(st, L.dg_last_error(h).decode())
        out = dict(tri=np.zeros((nc, 3), np.int32), nbr=np.zeros((nc, 3), np.int32),
                   nbe=np.zeros((nc, 3), np.int32), perm=np.zeros((nc, 3), np.int32),
                   node_ref=np.zeros((4, nc)), ck=np.zeros(nc))
        minck = ctypes.c_double(0)
        st = L.dg_mesh_tables(h, _ptr(out["tri"]), _ptr(out["nbr"]), _ptr(out["nbe"]), _ptr(out["perm"]),
                              _ptr(out["node_ref"]), _ptr(out["ck"]), ctypes.byref(minck))
        if st != 0:
            raise DgError(st, L.dg_last_error(h).decode())
        out["minck"] = minck.value
        return out
    finally:
        L.dg_destroy(h)


class Batch:
    """Several initialised Solvers on one device stepped together (dg_batch_*).

    The solvers must outlive the batch and keep their mesh and configuration
    while it exists.  Work runs on torch's current stream of their device."""

    def __init__(self, solvers):
        import torch
        L = load_library()
        if not solvers:
            raise ValueError("empty batch")
        self.solvers = list(solvers)
        self.stream = torch.cuda.current_stream(self.solvers[0].device)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = ctypes.c_void_p()
        st = L.dg_batch_create(ctypes.byref(h), arr, len(self.solvers), ctypes.c_void_p(self.stream.cuda_stream))
        self.h = h if h.value else None
        if st != 0:
            msg = L.dg_batch_last_error(self.h).decode() if self.h else "dg_batch_create failed"
            self.close()
            raise DgError(st, msg)

    def _check(self, st):
        if st != 0:
            raise DgError(st, load_library().dg_batch_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            load_library().dg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._check(load_library().dg_batch_step(self.h, int(n)))

    def run(self, max_steps=(1 << 62)):
        n = ctypes.c_int64(0)
        self._check(load_library().dg_batch_run(self.h, int(max_steps), ctypes.byref(n)))
        return n.value

    def status(self):
        """(number of active members, array (n, 4) of active, error, t, step)."""
        act = ctypes.c_int(0)
        out = np.zeros((len(self.solvers), 4))
        self._check(load_library().dg_batch_status(self.h, ctypes.byref(act), _ptr(out)))
        return act.value, out

    def set_schedule(self, chunk_groups, occupancy_pct=100):
        self._check(load_library().dg_batch_set_schedule(self.h, int(chunk_groups), int(occupancy_pct)))

    def schedule(self):
        cg, occ, nch = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        grid = (ctypes.c_int * 2)()   # residual, filter
        self._check(load_library().dg_batch_get_schedule(self.h, ctypes.byref(cg), ctypes.byref(occ),
                                                         ctypes.byref(nch), grid))
        return {"chunk_groups": cg.value, "occupancy_pct": occ.value, "n_chunks": nch.value, "grid": list(grid)}

    def autotune(self, reps=3):
        cg, occ, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
        self._check(load_library().dg_batch_autotune(self.h, int(reps), ctypes.byref(cg), ctypes.byref(occ),
                                                     ctypes.byref(ms)))
        return {"chunk_groups": cg.value, "occupancy_pct": occ.value, "ms_stage": ms.value}


def plan_chunks(n_cell, k, chunk_groups=1):
    """Host-only chunk table of instances with n_cell[i] cells at degree k[i]:
    (chunks (n, 3) int32 of instance, first group, end group; split (9,) int32)."""
    L = load_library()
    nc = np.ascontiguousarray(n_cell, dtype=np.int32)
    kk = np.ascontiguousarray(k, dtype=np.int32)
    n = ctypes.c_int(0)
    st = L.dg_plan_chunks(len(nc), _ptr(nc), _ptr(kk), int(chunk_groups), None, 0, ctypes.byref(n), None)
    if st != 0:
        raise DgError(st, "dg_plan_chunks failed")
    chunks = np.zeros((n.value, 3), np.int32)
    split = np.zeros(9, np.int32)
    st = L.dg_plan_chunks(len(nc), _ptr(nc), _ptr(kk), int(chunk_groups), _ptr(chunks), n.value,
                          ctypes.byref(n), _ptr(split))
    if st != 0:
        raise DgError(st, "dg_plan_chunks failed")
    return chunks, split
