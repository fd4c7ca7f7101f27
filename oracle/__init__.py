"""ORACLE -- test infrastructure only.

Python access to the plain FP64 CPU Smart Laplacian in ``slref.c`` and to the
exact rational brute force in ``exact.py``.  Only ``tests/``, the package
smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with the GPU library and imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslref.so")
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile slref.c with gcc (no contraction, no fast-math)."""
    src = os.path.join(_HERE, "slref.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + CFLAGS + ["-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _c():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        d, p, i32, i64 = ctypes.c_double, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.slref_quality.argtypes = [d] * 6
        lib.slref_quality.restype = d
        lib.slref_sweep_jacobi.argtypes = [p, p, i32, p, p, p, p, p, p, ctypes.c_int, ctypes.c_int, p,
                                           ctypes.POINTER(d)]
        lib.slref_sweep_jacobi.restype = i64
        lib.slref_smooth.argtypes = [p, i32, p, p, p, p, p, i32, p, i32, d, ctypes.c_int, ctypes.c_int, p, p, p]
        lib.slref_smooth.restype = i32
        lib.slref_smooth_colored.argtypes = [p, i32, p, p, p, p, p, i32, p, i32, d, ctypes.c_int, p, p, p, p]
        lib.slref_smooth_colored.restype = i32
        f = ctypes.c_float
        lib.slref32_quality.argtypes = [f] * 6
        lib.slref32_quality.restype = f
        lib.slref32_smooth.argtypes = [p, i32, p, p, p, p, p, i32, p, i32, d, ctypes.c_int, ctypes.c_int, p, p, p]
        lib.slref32_smooth.restype = i32
        lib.slref_color.argtypes = [i32, p, p, p, p]
        lib.slref_color.restype = i32
        lib.slref_priority.argtypes = [ctypes.c_uint64]
        lib.slref_priority.restype = ctypes.c_uint64
        lib.slref_max_threads.argtypes = []
        lib.slref_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _arr(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def quality(x0, y0, x1, y1, x2, y2) -> float:
    """Quality 4*sqrt(3)*A/sum(l^2) of one triangle in stored vertex order."""
    return _c().slref_quality(x0, y0, x1, y1, x2, y2)


def quality32(x0, y0, x1, y1, x2, y2) -> float:
    """The same quality in IEEE single precision (arguments rounded to float)."""
    return _c().slref32_quality(x0, y0, x1, y1, x2, y2)


def max_threads() -> int:
    return _c().slref_max_threads()


class Result:
    def __init__(self, coords, iterations_run, flags, disp, accepted, colors=None):
        self.coords = coords
        self.iterations_run = iterations_run
        self.flags = flags          # (iterations_run, N) uint8: 1 acc, 0 rej, 2 fixed
        self.disp = disp            # (iterations_run,) largest squared displacement per sweep
        self.accepted = accepted    # (iterations_run,) accepted count per sweep
        self.colors = colors


def smooth(mesh, iterations: int, tol: float = 0.0, accept_gt: bool = False, threads: int = 1,
           want_flags: bool = True, form: str = "jacobi", precision: str = "f64") -> Result:
    """Run the oracle on a ``meshgen.Mesh`` (or any object with the same
    array attributes).  ``form``: "jacobi" (Form A) or "colored" (Form B).
    ``precision``: "f64", or "f32" (Form A in single precision: coordinates
    rounded to float on entry, float results returned as doubles)."""
    lib = _c()
    X = _arr(mesh.coords, np.float64).copy()
    n = X.shape[0]
    nbr_ptr, nbr_idx = _arr(mesh.nbr_ptr, np.int32), _arr(mesh.nbr_idx, np.int32)
    tri_ptr, tri_idx = _arr(mesh.tri_ptr, np.int32), _arr(mesh.tri_idx, np.int32)
    tris, bnd = _arr(mesh.tris, np.int32), _arr(mesh.boundary, np.uint8)
    flags = np.zeros((max(iterations, 1), n), np.uint8) if want_flags else None
    disp = np.zeros(max(iterations, 1), np.float64)
    acc = np.zeros(max(iterations, 1), np.int64)
    fptr = flags.ctypes.data if flags is not None else None
    if precision not in ("f64", "f32"):
        raise ValueError(precision)
    if precision == "f32":
        if form != "jacobi":
            raise ValueError("single precision is Form A only")
        k = lib.slref32_smooth(X.ctypes.data, n, nbr_ptr.ctypes.data, nbr_idx.ctypes.data, tri_ptr.ctypes.data,
                               tri_idx.ctypes.data, tris.ctypes.data,
                               tris.shape[0] if tris.ndim == 2 else len(tris) // 3, bnd.ctypes.data, iterations,
                               tol, int(accept_gt), threads, fptr, disp.ctypes.data, acc.ctypes.data)
        colors = None
    elif form == "jacobi":
        k = lib.slref_smooth(X.ctypes.data, n, nbr_ptr.ctypes.data, nbr_idx.ctypes.data, tri_ptr.ctypes.data,
                             tri_idx.ctypes.data, tris.ctypes.data, tris.shape[0] if tris.ndim == 2 else len(tris) // 3,
                             bnd.ctypes.data, iterations, tol, int(accept_gt), threads, fptr, disp.ctypes.data,
                             acc.ctypes.data)
        colors = None
    elif form == "colored":
        colors = np.zeros(n, np.int32)
        k = lib.slref_smooth_colored(X.ctypes.data, n, nbr_ptr.ctypes.data, nbr_idx.ctypes.data,
                                     tri_ptr.ctypes.data, tri_idx.ctypes.data, tris.ctypes.data,
                                     tris.shape[0] if tris.ndim == 2 else len(tris) // 3, bnd.ctypes.data,
                                     iterations, tol, int(accept_gt), fptr, disp.ctypes.data, acc.ctypes.data,
                                     colors.ctypes.data)
    else:
        raise ValueError(form)
    if k < 0:
        raise ValueError("oracle rejected the input")
    return Result(X, k, flags[:k] if flags is not None else None, disp[:k], acc[:k], colors)


def sweep(mesh, X, accept_gt: bool = False, threads: int = 1):
    """One Jacobi sweep from positions X; returns (Xnew, flags, accepted, max_disp_sq)."""
    lib = _c()
    X = _arr(X, np.float64)
    n = X.shape[0]
    out = np.empty_like(X)
    flags = np.zeros(n, np.uint8)
    d2 = ctypes.c_double(0.0)
    tris = _arr(mesh.tris, np.int32)
    a = lib.slref_sweep_jacobi(X.ctypes.data, out.ctypes.data, n, _arr(mesh.nbr_ptr, np.int32).ctypes.data,
                               _arr(mesh.nbr_idx, np.int32).ctypes.data, _arr(mesh.tri_ptr, np.int32).ctypes.data,
                               _arr(mesh.tri_idx, np.int32).ctypes.data, tris.ctypes.data,
                               _arr(mesh.boundary, np.uint8).ctypes.data, int(accept_gt), threads,
                               flags.ctypes.data, ctypes.byref(d2))
    return out, flags, int(a), d2.value


def colors(mesh):
    n = mesh.coords.shape[0]
    col = np.zeros(n, np.int32)
    nc = _c().slref_color(n, _arr(mesh.nbr_ptr, np.int32).ctypes.data, _arr(mesh.nbr_idx, np.int32).ctypes.data,
                          _arr(mesh.boundary, np.uint8).ctypes.data, col.ctypes.data)
    return col, nc


def priority(v: int) -> int:
    return int(_c().slref_priority(v))
