"""Seeded synthetic triangular meshes: the inputs of the smoothing workloads.

This package is input plumbing shared by the oracle tests, the GPU tests and
the benchmark.  It holds none of the smoothing arithmetic (no triangle
quality, no centroid, no accept test): it places nodes, lists CCW triangles,
builds the node->neighbour and node->triangle CSR arrays the library takes as
input, and derives the boundary mask.

The paper measures on Delaunay meshes of uniformly random points (Sec. 4);
those meshes and the tools that made them are not available, so jittered
structured grids and an annulus of the same kind (planar, valence about 6,
one boundary loop or two) stand in for them.

Recipes (all draws from ``numpy.random.Generator(PCG64(seed))``):

* grid ``n``: node (i, j) at (i*h, j*h), h = 1/(n-1), id j*n + i.  Cell (i, j)
  (row-major, j outer) yields two CCW triangles.  With a = (i,j), b = (i+1,j),
  c = (i+1,j+1), d = (i,j+1): diagonal "/" gives (a,b,c), (a,c,d); diagonal
  "\\" gives (a,b,d), (b,c,d).  ``diag="unionjack"``: "/" iff (i+j) even;
  ``"random"``: "/" iff a uniform draw per cell is < 0.5 (first draw block);
  ``"slash"``: always "/".
* jitter J: one uniform draw in [-J*h, +J*h) per coordinate of every node
  (second draw block, shape (N, 2)), applied to interior nodes only.
* annulus (n_r rings, n_t angles): parameter node (i, j) with i the ring index
  and j the angle index (periodic), id j*n_r + i, r_i = r0 + (r1-r0) i/(n_r-1),
  theta_j = 2 pi j / n_t; jitter of +-J of (dr, dtheta) in parameter space on
  the interior rings, then (r cos theta, r sin theta).  The map has positive
  Jacobian in (r, theta) order, so parameter-CCW triangles stay CCW.
* permutation: a random relabelling of the nodes and a random order of the
  triangles (vertex order inside a triangle kept), after which the CSR arrays
  are rebuilt from the new triangle list.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_libmgen.so")
_lib = None


def build_native(force: bool = False) -> str:
    """Compile the adjacency builder (plain C) next to this file."""
    src = os.path.join(_HERE, "_mgen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _native():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_native()
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        lib.mg_build_adjacency.argtypes = [ctypes.c_int32, ctypes.c_int32, p, p, p, p, p, p,
                                           ctypes.POINTER(ctypes.c_int64)]
        lib.mg_build_adjacency.restype = ctypes.c_int
        lib.mg_delaunay.argtypes = [ctypes.c_int32, p, p, p, ctypes.POINTER(ctypes.c_int32)]
        lib.mg_delaunay.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclasses.dataclass
class Mesh:
    """A planar triangular mesh with the adjacency arrays the library takes.

    coords   (N, 2) float64, xy interleaved
    tris     (T, 3) int32, CCW, stored vertex order
    nbr_ptr  (N+1,) int32 / nbr_idx (nnz,) int32: node->neighbour CSR
    tri_ptr  (N+1,) int32 / tri_idx (3T,) int32: node->triangle CSR
    boundary (N,) uint8, nonzero = fixed
    """
    coords: np.ndarray
    tris: np.ndarray
    nbr_ptr: np.ndarray
    nbr_idx: np.ndarray
    tri_ptr: np.ndarray
    tri_idx: np.ndarray
    boundary: np.ndarray
    name: str = ""

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_interior(self) -> int:
        return int(np.count_nonzero(self.boundary == 0))

    def copy(self) -> "Mesh":
        return Mesh(*(np.array(getattr(self, f.name), copy=True) if isinstance(getattr(self, f.name), np.ndarray)
                      else getattr(self, f.name) for f in dataclasses.fields(self)))

    def arrays(self):
        return (self.coords, self.nbr_ptr, self.nbr_idx, self.tri_ptr, self.tri_idx, self.tris, self.boundary)


def build_adjacency(n_nodes: int, tris: np.ndarray):
    """node->neighbour CSR (first-appearance order), node->triangle CSR
    (ascending), boundary mask by the recorded-twice rule."""
    tris = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    T = tris.shape[0]
    nbr_ptr = np.zeros(n_nodes + 1, np.int32)
    nbr_idx = np.zeros(max(6 * T, 1), np.int32)
    tri_ptr = np.zeros(n_nodes + 1, np.int32)
    tri_idx = np.zeros(max(3 * T, 1), np.int32)
    bnd = np.zeros(n_nodes, np.uint8)
    nnz = ctypes.c_int64(0)
    rc = _native().mg_build_adjacency(n_nodes, T, tris.ctypes.data, nbr_ptr.ctypes.data, nbr_idx.ctypes.data,
                                      tri_ptr.ctypes.data, tri_idx.ctypes.data, bnd.ctypes.data, ctypes.byref(nnz))
    if rc != 0:
        raise ValueError("mg_build_adjacency failed (%d)" % rc)
    return nbr_ptr, nbr_idx[: nnz.value].copy(), tri_ptr, tri_idx[: 3 * T].copy(), bnd


def _grid_tris(nx: int, ny: int, diag: np.ndarray, periodic_y: bool = False) -> np.ndarray:
    """Two CCW triangles per cell; node id j*nx + i; cells row-major (j outer).
    ``diag`` is a bool array of shape (ncy, nx-1): True = "/" diagonal."""
    ncx = nx - 1
    ncy = ny if periodic_y else ny - 1
    j, i = np.meshgrid(np.arange(ncy, dtype=np.int64), np.arange(ncx, dtype=np.int64), indexing="ij")
    jn = (j + 1) % ny if periodic_y else j + 1
    a = j * nx + i
    b = j * nx + i + 1
    c = jn * nx + i + 1
    d = jn * nx + i
    slash = diag.reshape(ncy, ncx)
    t1 = np.where(slash[..., None], np.stack([a, b, c], -1), np.stack([a, b, d], -1))
    t2 = np.where(slash[..., None], np.stack([a, c, d], -1), np.stack([b, c, d], -1))
    tris = np.stack([t1, t2], axis=2).reshape(-1, 3)
    return tris.astype(np.int32)


def _diagonals(kind: str, ncy: int, ncx: int, rng) -> np.ndarray:
    if kind == "unionjack":
        j, i = np.meshgrid(np.arange(ncy), np.arange(ncx), indexing="ij")
        return ((i + j) % 2 == 0)
    if kind == "random":
        return rng.random((ncy, ncx)) < 0.5
    if kind == "slash":
        return np.ones((ncy, ncx), bool)
    if kind == "backslash":
        return np.zeros((ncy, ncx), bool)
    raise ValueError(kind)


def make_grid(n: int, diag: str = "random", jitter: float = 0.0, seed: int = 0,
              h: Optional[float] = None, name: str = "") -> Mesh:
    """Jittered n x n unit-square grid (see module docstring for the recipe).
    ``h`` overrides the spacing (used for dyadic fixed-point meshes)."""
    if n < 2:
        raise ValueError("n >= 2")
    rng = np.random.Generator(np.random.PCG64(seed))
    hh = 1.0 / (n - 1) if h is None else float(h)
    dg = _diagonals(diag, n - 1, n - 1, rng)
    tris = _grid_tris(n, n, dg)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    coords = np.stack([i.ravel() * hh, j.ravel() * hh], axis=1).astype(np.float64)
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = build_adjacency(n * n, tris)
    if jitter:
        jit = rng.uniform(-jitter * hh, jitter * hh, size=(n * n, 2))
        interior = bnd == 0
        coords[interior] += jit[interior]
    return Mesh(coords, tris, nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd,
                name=name or "grid%d_%s_j%g_s%d" % (n, diag, jitter, seed))


def make_annulus(n_r: int, n_t: int, r0: float = 0.3, r1: float = 1.0, diag: str = "random",
                 jitter: float = 0.4, seed: int = 0, name: str = "") -> Mesh:
    """Annulus with n_r rings x n_t angular positions, periodic in angle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dg = _diagonals(diag, n_t, n_r - 1, rng)
    tris = _grid_tris(n_r, n_t, dg, periodic_y=True)
    N = n_r * n_t
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = build_adjacency(N, tris)
    j, i = np.meshgrid(np.arange(n_t), np.arange(n_r), indexing="ij")
    pr = i.ravel().astype(np.float64)
    pt = j.ravel().astype(np.float64)
    if jitter:
        jit = rng.uniform(-jitter, jitter, size=(N, 2))
        interior = bnd == 0
        pr[interior] += jit[interior, 0]
        pt[interior] += jit[interior, 1]
    r = r0 + (r1 - r0) * pr / (n_r - 1)
    th = 2.0 * math.pi * pt / n_t
    coords = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    return Mesh(coords, tris, nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd,
                name=name or "annulus%dx%d_%s_j%g_s%d" % (n_r, n_t, diag, jitter, seed))


def permute_mesh(m: Mesh, seed: int) -> Mesh:
    """Random node relabelling + random triangle order; CSR rebuilt."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = m.n_nodes
    new_of_old = rng.permutation(N).astype(np.int64)
    tri_order = rng.permutation(m.n_tris)
    coords = np.empty_like(m.coords)
    coords[new_of_old] = m.coords
    tris = new_of_old[m.tris[tri_order]].astype(np.int32)
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = build_adjacency(N, tris)
    return Mesh(coords, tris, nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd, name=m.name + "_perm%d" % seed)


def relabel_keep_rows(m: Mesh, new_of_old: np.ndarray) -> Mesh:
    """Relabel nodes by ``new_of_old`` keeping every row's order and every
    triangle's vertex order (only the ids change, and rows move with their
    node).  Triangle ids are unchanged."""
    new_of_old = np.asarray(new_of_old, dtype=np.int64)
    N = m.n_nodes
    old_of_new = np.empty(N, np.int64)
    old_of_new[new_of_old] = np.arange(N)
    coords = m.coords[old_of_new]
    bnd = m.boundary[old_of_new]
    deg = np.diff(m.nbr_ptr.astype(np.int64))[old_of_new]
    nbr_ptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    rows = [m.nbr_idx[m.nbr_ptr[o]:m.nbr_ptr[o + 1]] for o in old_of_new]
    nbr_idx = new_of_old[np.concatenate(rows)].astype(np.int32) if rows else np.zeros(0, np.int32)
    tdeg = np.diff(m.tri_ptr.astype(np.int64))[old_of_new]
    tri_ptr = np.concatenate([[0], np.cumsum(tdeg)]).astype(np.int32)
    trows = [m.tri_idx[m.tri_ptr[o]:m.tri_ptr[o + 1]] for o in old_of_new]
    tri_idx = np.concatenate(trows).astype(np.int32)
    tris = new_of_old[m.tris].astype(np.int32)
    return Mesh(coords, tris, nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd, name=m.name + "_relabel")


def star_mesh(center, ring) -> Mesh:
    """One interior node (id 0) surrounded by a CCW ring of boundary nodes;
    triangles (0, r_k, r_{k+1})."""
    ring = [tuple(map(float, p)) for p in ring]
    k = len(ring)
    coords = np.array([tuple(map(float, center))] + ring, dtype=np.float64)
    tris = np.array([[0, 1 + q, 1 + (q + 1) % k] for q in range(k)], dtype=np.int32)
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = build_adjacency(k + 1, tris)
    return Mesh(coords, tris, nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd, name="star%d" % k)


LATTICE_BITS = 20


def delaunay_triangles(xi: np.ndarray, yi: np.ndarray) -> np.ndarray:
    """CCW Delaunay triangles of distinct integer lattice points (exact
    predicates; see mg_delaunay)."""
    xi = np.ascontiguousarray(xi, dtype=np.int64)
    yi = np.ascontiguousarray(yi, dtype=np.int64)
    n = xi.size
    out = np.zeros(max(3 * (2 * n), 3), np.int32)
    nt = ctypes.c_int32(0)
    rc = _native().mg_delaunay(n, xi.ctypes.data, yi.ctypes.data, out.ctypes.data, ctypes.byref(nt))
    if rc != 0:
        raise ValueError("mg_delaunay failed (%d)" % rc)
    return out[: 3 * nt.value].reshape(-1, 3).copy()


def random_lattice_points(n: int, seed: int):
    """n distinct points drawn uniformly from the 2^20 x 2^20 lattice, in
    draw order: (xi, yi) integers."""
    rng = np.random.Generator(np.random.PCG64(seed))
    side = 1 << LATTICE_BITS
    codes = np.empty(0, np.int64)
    while codes.size < n:
        draw = rng.integers(0, side * side, size=n + n // 8 + 16, dtype=np.int64)
        allc = np.concatenate([codes, draw])
        _, first = np.unique(allc, return_index=True)
        codes = allc[np.sort(first)]
    codes = codes[:n]
    return codes % side, codes // side


def make_delaunay(n: int, seed: int = 0, name: str = "") -> Mesh:
    """Delaunay mesh of n uniformly random points in the unit square (the
    paper's test meshes, Sec. 4): points on the 2^20 lattice, coordinates
    lattice / 2^20 (exact), node id = draw order, triangles in construction
    order; the boundary is the convex hull."""
    xi, yi = random_lattice_points(n, seed)
    tris = delaunay_triangles(xi, yi)
    coords = np.stack([xi, yi], axis=1).astype(np.float64) * (2.0 ** -LATTICE_BITS)
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = build_adjacency(n, tris)
    return Mesh(coords, tris, nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd, name or "delaunay%d_s%d" % (n, seed))


def batch_sides(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Side lengths round(exp(U(ln lo, ln hi)))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
