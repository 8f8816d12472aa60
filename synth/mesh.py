"""Seeded triangle meshes.

Two families stand in for the paper's EasyMesh meshes (not available here):

* `periodic_jittered_grid`: an n x n grid of squares on [0, L]^2, each square cut
  along its (i,j)-(i+1,j+1) diagonal into two triangles, interior vertices jittered
  independently in x and y by U(-j h, j h).  Periodic: triangles reference wrapped
  vertex ids, and `cell_xy` carries every cell's unwrapped vertex coordinates.
* `poisson_delaunay`: Poisson-disk points in a rectangle (boundary points at spacing
  about r so the hull is the rectangle, optional extra fixed points such as the
  origin) triangulated by Qhull's Delaunay.

Both emit triangles counter-clockwise and sorted along a Hilbert curve through the
cell centroids, so consecutive cells are spatial neighbours.
"""

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .rng import Stream


@dataclass
class Mesh:
    xy: np.ndarray                  # (n_vert, 2) float64 vertex coordinates
    tri: np.ndarray                 # (n_cell, 3) int32 vertex ids, CCW
    cell_xy: Optional[np.ndarray] = None   # (n_cell, 6) unwrapped coords (periodic only)
    periodic: bool = False
    edge_bc: Optional[np.ndarray] = None   # (n_cell, 3) int32 tags of boundary edges (edge opposite vertex i):
                                           # 0 transmissive, 1 reflective; None: all transmissive
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_cell(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.xy.shape[0])

    def cell_coords(self) -> np.ndarray:
        """(n_cell, 3, 2) vertex coordinates of every cell (unwrapped if periodic)."""
        if self.cell_xy is not None:
            return self.cell_xy.reshape(-1, 3, 2)
        return self.xy[self.tri]


# --------------------------------------------------------------------------- ordering

def _hilbert_d(order: int, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Index along a Hilbert curve of 2^order x 2^order cells (vectorised xy2d)."""
    x = x.astype(np.int64).copy()
    y = y.astype(np.int64).copy()
    d = np.zeros_like(x)
    s = 1 << (order - 1)
    while s > 0:
        rx = ((x & s) > 0).astype(np.int64)
        ry = ((y & s) > 0).astype(np.int64)
        d += s * s * ((3 * rx) ^ ry)
        # rotate the quadrant
        flip = ry == 0
        swap_x = flip & (rx == 1)
        x = np.where(swap_x, s - 1 - x, x)
        y = np.where(swap_x, s - 1 - y, y)
        xt = np.where(flip, y, x)
        yt = np.where(flip, x, y)
        x, y = xt, yt
        s >>= 1
    return d


def hilbert_order(points: np.ndarray, order: int = 16) -> np.ndarray:
    """Stable permutation sorting `points` (n,2) along a Hilbert curve."""
    if len(points) == 0:
        return np.zeros(0, dtype=np.int64)
    lo = points.min(axis=0)
    span = np.maximum(points.max(axis=0) - lo, 1e-300)
    n = (1 << order) - 1
    q = np.clip(((points - lo) / span.max()) * n, 0, n).astype(np.int64)
    d = _hilbert_d(order, q[:, 0], q[:, 1])
    return np.argsort(d, kind="stable")


def shuffle_cells(mesh: Mesh, seed: int) -> Mesh:
    """The same mesh with its cells in a seeded random order (vertex ids and each
    cell's vertex order kept).  Without locality most of a tile's neighbours fall
    outside its halo, which exercises the stage kernels' global-memory path."""
    keys = Stream(seed).bits(mesh.n_cell)
    p = np.argsort(keys, kind="stable")
    return Mesh(xy=mesh.xy, tri=np.ascontiguousarray(mesh.tri[p]),
                cell_xy=None if mesh.cell_xy is None else np.ascontiguousarray(mesh.cell_xy[p]),
                periodic=mesh.periodic,
                edge_bc=None if mesh.edge_bc is None else np.ascontiguousarray(mesh.edge_bc[p]),
                name=mesh.name + "_shuffled", meta=dict(mesh.meta))


# --------------------------------------------------------------------------- periodic grid

def periodic_jittered_grid(n: int = 32, length: float = 10.0, jitter: float = 0.1,
                           seed: int = 1, order_cells: bool = True) -> Mesh:
    h = length / n
    st = Stream(seed)
    # unwrapped (n+1)^2 grid, interior vertices jittered in x then y, row-major in (j, i)
    gx, gy = np.meshgrid(np.arange(n + 1) * h, np.arange(n + 1) * h, indexing="xy")
    interior = np.zeros((n + 1, n + 1), dtype=bool)
    interior[1:n, 1:n] = True
    k = int(interior.sum())
    jx = st.uniform(k, -jitter * h, jitter * h)
    jy = st.uniform(k, -jitter * h, jitter * h)
    gx = gx.copy()
    gy = gy.copy()
    gx[interior] += jx
    gy[interior] += jy

    def wid(i, j):
        return (i % n) + n * (j % n)

    xy = np.zeros((n * n, 2))
    for j in range(n):
        for i in range(n):
            xy[wid(i, j)] = (gx[j, i], gy[j, i])

    tri = []
    cxy = []
    for j in range(n):
        for i in range(n):
            a, b, c, d = (i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)
            for t in ((a, b, c), (a, c, d)):
                tri.append([wid(*p) for p in t])
                cxy.append([v for p in t for v in (gx[p[1], p[0]], gy[p[1], p[0]])])
    tri = np.asarray(tri, dtype=np.int32)
    cxy = np.asarray(cxy, dtype=np.float64)
    if order_cells:
        cen = cxy.reshape(-1, 3, 2).mean(axis=1)
        p = hilbert_order(cen)
        tri, cxy = tri[p], cxy[p]
    return Mesh(xy=xy, tri=np.ascontiguousarray(tri), cell_xy=np.ascontiguousarray(cxy),
                periodic=True, name=f"periodic{n}x{n}",
                meta=dict(n=n, length=length, jitter=jitter, seed=seed, h=h))


def tile_periodic_grid(base: Mesh, a: int, b: int) -> Mesh:
    """a x b copies of a `periodic_jittered_grid` block, itself periodic: block
    (A, B) is the base shifted by (A L, B L), and block q = A + a B holds cells
    q n_base ... (q + 1) n_base - 1 in the base's order, each with the base cell's
    vertex order.  Data periodic with the base's period therefore has, on the
    tiling, the base's solution in every block."""
    n, h, L = base.meta["n"], base.meta["h"], base.meta["length"]
    N, M = n * a, n * b                                  # squares of the tiling
    cxy = base.cell_xy.reshape(-1, 3, 2)
    ij = np.rint(cxy / h).astype(np.int64)               # grid indices 0..n of each vertex (jitter < h/2)
    blk = np.arange(a * b, dtype=np.int64)
    A, B = blk % a, blk // a
    I = (A[:, None, None] * n + ij[None, :, :, 0]) % N
    J = (B[:, None, None] * n + ij[None, :, :, 1]) % M
    tri = (I + N * J).astype(np.int32).reshape(-1, 3)
    del I, J
    shift = np.stack([A * L, B * L], axis=1).astype(np.float64)            # (a b, 2)
    cell_xy = (cxy[None, :, :, :] + shift[:, None, None, :]).reshape(-1, 6)
    vi, vj = np.meshgrid(np.arange(N), np.arange(M), indexing="xy")
    vi, vj = vi.ravel(), vj.ravel()                      # vertex I + N J, row-major in J
    xy = base.xy[(vi % n) + n * (vj % n)] + np.stack([(vi // n) * L, (vj // n) * L], axis=1)
    return Mesh(xy=np.ascontiguousarray(xy), tri=np.ascontiguousarray(tri),
                cell_xy=np.ascontiguousarray(cell_xy), periodic=True,
                name=f"{base.name}_tiled{a}x{b}", meta=dict(base.meta, tiles=(a, b)))


# --------------------------------------------------------------------------- Poisson disk

def _boundary_points(lo, hi, r):
    """Points along the rectangle's sides at equal spacing of at least r."""
    pts = []
    for a in range(2):
        span = hi[a] - lo[a]
        m = max(1, int(np.floor(span / r)))
        t = lo[a] + span * np.arange(m + 1) / m
        for other in (lo[1 - a], hi[1 - a]):
            p = np.zeros((m + 1, 2))
            p[:, a] = t
            p[:, 1 - a] = other
            pts.append(p)
    pts = np.concatenate(pts)
    return np.unique(pts, axis=0)


_PDS_LIB = None


def build_helpers(force: bool = False) -> str:
    """Compile the Poisson-disk helper (synth/pds.c) next to its source."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    so = os.path.join(here, "_pds.so")
    src = os.path.join(here, "pds.c")
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        tmp = so + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, so)
    return so


def _pds_lib():
    global _PDS_LIB
    if _PDS_LIB is None:
        import ctypes
        lib = ctypes.CDLL(build_helpers())
        lib.pds_sample.restype = ctypes.c_int
        lib.pds_sample.argtypes = [ctypes.c_double] * 5 + [ctypes.c_ulonglong, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        _PDS_LIB = lib
    return _PDS_LIB


def poisson_disk(r: float, lo, hi, seed: int, k: int = 30,
                 fixed: Optional[np.ndarray] = None) -> np.ndarray:
    """Bridson Poisson-disk sample with minimum spacing r; `fixed` points come first."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    fixed = np.zeros((0, 2)) if fixed is None else np.ascontiguousarray(fixed, dtype=np.float64)
    cap = int(1.2 * np.prod(hi - lo) / (r * r)) + len(fixed) + 64
    out = np.zeros((cap, 2))
    n = _pds_lib().pds_sample(float(r), float(lo[0]), float(lo[1]), float(hi[0]), float(hi[1]),
                              int(seed) & 0xFFFFFFFFFFFFFFFF, int(k),
                              fixed.ctypes.data, len(fixed), out.ctypes.data, cap)
    if n < 0:
        raise RuntimeError("poisson_disk: capacity exceeded")
    return out[:n].copy()


def _delaunay(points: np.ndarray) -> np.ndarray:
    from scipy.spatial import Delaunay
    tri = Delaunay(points, qhull_options="Qbb Qc Qz Q12").simplices.astype(np.int64)
    p = points[tri]
    det = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - \
          (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    flip = det < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    keep = np.abs(det) > 1e-14 * np.abs(det).max()
    return tri[keep]


def poisson_delaunay(n_cells: int, lo=(0.0, 0.0), hi=(1.0, 1.0), seed: int = 2,
                     extra_points: Optional[np.ndarray] = None, name: str = "") -> Mesh:
    """Delaunay mesh of seeded Poisson-disk points with about `n_cells` triangles.

    Bridson sampling with 30 tries settles at about 0.62 points per r^2, and a
    Delaunay mesh of P points has about 2P triangles, which fixes r.
    """
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    area = float(np.prod(hi - lo))
    r = float(np.sqrt(0.622 * area / max(n_cells / 2.0, 4.0)))
    fixed = _boundary_points(lo, hi, r)
    if extra_points is not None:
        fixed = np.unique(np.concatenate([fixed, np.asarray(extra_points, float).reshape(-1, 2)]),
                          axis=0)
    pts = poisson_disk(r, lo, hi, seed, fixed=fixed)
    tri = _delaunay(pts)
    # order vertices by first use along the Hilbert-sorted cells, then cells
    cen = pts[tri].mean(axis=1)
    p = hilbert_order(cen)
    tri = tri[p]
    used, first = np.unique(tri.ravel(), return_index=True)
    vorder = used[np.argsort(first, kind="stable")]
    remap = np.full(len(pts), -1, dtype=np.int64)
    remap[vorder] = np.arange(len(vorder))
    xy = pts[vorder]
    tri = remap[tri].astype(np.int32)
    return Mesh(xy=np.ascontiguousarray(xy), tri=np.ascontiguousarray(tri), periodic=False,
                name=name or f"delaunay{len(tri)}",
                meta=dict(seed=seed, r=float(r), lo=lo.tolist(), hi=hi.tolist(),
                          n_target=int(n_cells)))


def find_vertex(mesh: Mesh, point) -> int:
    """Id of the mesh vertex equal to `point` (exact match), or -1."""
    hit = np.nonzero((mesh.xy[:, 0] == point[0]) & (mesh.xy[:, 1] == point[1]))[0]
    return int(hit[0]) if len(hit) else -1
