"""smartlap -- Smart Laplacian mesh smoothing on MI355X (gfx950).

A thin ctypes binding over ``libsmartlap.so`` (C ABI in
``include/smartlap.h``).  The binding only marshals arguments: every step of
the smoothing runs in the library's HIP kernels.  PyTorch is used for device
memory and streams only.  There is no CPU path: if the library is not built,
or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmartlap.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "smartlap.h")

SL_OK, SL_EINVAL, SL_ETOPO, SL_ENOMEM, SL_EDEVICE, SL_EBUSY, SL_ECANCELED, SL_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "SL_OK", -1: "SL_EINVAL", -2: "SL_ETOPO", -3: "SL_ENOMEM", -4: "SL_EDEVICE", -5: "SL_EBUSY",
                -6: "SL_ECANCELED", -7: "SL_ETIMEOUT"}
FORMS = {"jacobi": 0, "colored": 1}
ACCEPT = {"ge": 0, "gt": 1}
LAYOUTS = {"aos": 0, "soa": 1}
REORDER = {"none": 0, "hilbert": 1}
KERNELS = {"auto": 0, "node": 1, "tile": 2, "resident": 3, "lanes": 4}
PRECISIONS = {"f64": 0, "f32": 1}


class SmartlapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("accept", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("reorder", ctypes.c_int32), ("block_size", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("tile_nodes", ctypes.c_int32), ("tile_wg_per_cu", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("lane_width", ctypes.c_int32), ("flags_out", ctypes.c_void_p)]


class Report(ctypes.Structure):
    _fields_ = [("iterations_run", ctypes.c_int32), ("n_colors", ctypes.c_int32),
                ("max_disp_sq_last", ctypes.c_double), ("accepted_last", ctypes.c_int64),
                ("accepted_total", ctypes.c_int64), ("setup_ms", ctypes.c_double), ("sweep_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("kernel_used", ctypes.c_int32), ("tile_nodes", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MeshDesc(ctypes.Structure):
    _fields_ = [("coords", ctypes.c_void_p), ("n_nodes", ctypes.c_int32), ("n_tris", ctypes.c_int32),
                ("nbr_ptr", ctypes.c_void_p), ("nbr_idx", ctypes.c_void_p), ("tri_ptr", ctypes.c_void_p),
                ("tri_idx", ctypes.c_void_p), ("tris", ctypes.c_void_p), ("boundary", ctypes.c_void_p)]


class BatchReport(ctypes.Structure):
    _fields_ = [("setup_ms", ctypes.c_double), ("sweep_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("node_updates", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("meshes_on_tile_path", ctypes.c_int32), ("graph_used", ctypes.c_int32),
                ("graph_ms", ctypes.c_double), ("results_ms", ctypes.c_double),
                ("meshes_resident", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneCandidate(ctypes.Structure):
    _fields_ = [("tile_nodes", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("ns_per_update", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_nodes", ctypes.c_int32), ("tile_wg_per_cu", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("n_candidates", ctypes.c_int32), ("candidates", TuneCandidate * 16),
                ("sampled_meshes", ctypes.c_int32), ("sampled_free_nodes", ctypes.c_int64),
                ("tune_ms", ctypes.c_double), ("lane_width", ctypes.c_int32)]

    def as_dict(self):
        return {"tile_nodes": self.tile_nodes, "tile_wg_per_cu": self.tile_wg_per_cu, "block_size": self.block_size,
                "lane_width": self.lane_width,
                "candidates": [(c.tile_nodes, c.wg_per_cu, c.ns_per_update)
                               for c in self.candidates[: self.n_candidates]],
                "sampled_meshes": self.sampled_meshes, "sampled_free_nodes": self.sampled_free_nodes,
                "tune_ms": self.tune_ms}


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("sweeps_per_step", ctypes.c_int32), ("setup_threads", ctypes.c_int32)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("submitted_s", ctypes.c_double), ("admitted_s", ctypes.c_double), ("started_s", ctypes.c_double),
                ("done_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("node_updates", ctypes.c_int64), ("queued", ctypes.c_int32),
                ("active", ctypes.c_int32), ("hbm_in_use", ctypes.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def _check_current():
    """Raises if the in-tree library was built from other sources than the
    ones beside it (a library older than its sources would test old code)."""
    from . import build as _build
    if not os.path.isdir(_build.CSRC):
        return
    try:
        with open(_build.DIGEST) as f:
            have = f.read().strip()
    except OSError:
        have = None
    if have != _build.source_digest():
        raise RuntimeError("libsmartlap.so was not built from the sources in csrc/ "
                           "(rebuild: python -m paper_1502_00355_amd.build)")


def lib():
    """The loaded library; raises if it has not been built, or was built from
    other sources than the package holds."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsmartlap.so is not built (python -m paper_1502_00355_amd.build)")
        if os.path.abspath(LIB_PATH) == os.path.join(_HERE, "libsmartlap.so"):
            _check_current()
        L = ctypes.CDLL(LIB_PATH)
        p, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.sl_options_default.argtypes = [ctypes.POINTER(Options)]
        L.sl_options_default.restype = None
        L.sl_last_error.restype = ctypes.c_char_p
        L.sl_version.restype = ctypes.c_char_p
        sig = [p, i32, p, p, p, p, p, i32, p, i32, d, ctypes.POINTER(Options), ctypes.POINTER(Report)]
        L.smooth_mesh.argtypes = sig
        L.smooth_mesh.restype = ctypes.c_int
        L.smooth_mesh_device.argtypes = sig + [p]
        L.smooth_mesh_device.restype = ctypes.c_int
        L.smooth_mesh_device_noalloc.argtypes = sig + [p]
        L.smooth_mesh_device_noalloc.restype = ctypes.c_int
        L.sl_batch_smooth.argtypes = [ctypes.POINTER(MeshDesc), i32, i32, d, ctypes.POINTER(Options),
                                      ctypes.POINTER(Report), ctypes.POINTER(BatchReport)]
        L.sl_batch_smooth.restype = ctypes.c_int
        adj = [p, i32, i32, p, p, ctypes.c_int64, p, p, p, ctypes.POINTER(ctypes.c_int64)]
        L.sl_build_adjacency.argtypes = adj
        L.sl_build_adjacency.restype = ctypes.c_int
        L.sl_build_adjacency_device.argtypes = adj + [p]
        L.sl_build_adjacency_device.restype = ctypes.c_int
        L.sl_autotune.argtypes = [ctypes.POINTER(MeshDesc), i32, ctypes.POINTER(Options), ctypes.POINTER(Tuning)]
        L.sl_autotune.restype = ctypes.c_int
        L.sl_autotune_reset.argtypes = []
        L.sl_autotune_reset.restype = None
        L.sl_server_config_default.argtypes = [ctypes.POINTER(ServerConfig)]
        L.sl_server_config_default.restype = None
        L.sl_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(Options), ctypes.POINTER(p)]
        L.sl_server_create.restype = ctypes.c_int
        L.sl_server_submit.argtypes = [p, ctypes.POINTER(MeshDesc), i32, d, d, ctypes.POINTER(ctypes.c_uint64)]
        L.sl_server_submit.restype = ctypes.c_int
        L.sl_server_poll.argtypes = [p, ctypes.c_uint64, p, ctypes.POINTER(Report), ctypes.POINTER(RequestTimes)]
        L.sl_server_poll.restype = ctypes.c_int
        L.sl_server_cancel.argtypes = [p, ctypes.c_uint64]
        L.sl_server_cancel.restype = ctypes.c_int
        L.sl_server_get_stats.argtypes = [p, ctypes.POINTER(ServerStats)]
        L.sl_server_get_stats.restype = ctypes.c_int
        L.sl_server_destroy.argtypes = [p]
        L.sl_server_destroy.restype = None
        L.sl_mesh_create.argtypes = [ctypes.POINTER(MeshDesc), ctypes.POINTER(Options), ctypes.POINTER(p)]
        L.sl_mesh_create.restype = ctypes.c_int
        L.sl_mesh_create_device.argtypes = [p, i32, p, p, p, p, p, i32, p, ctypes.POINTER(Options), p,
                                            ctypes.POINTER(p)]
        L.sl_mesh_create_device.restype = ctypes.c_int
        L.sl_mesh_smooth_async.argtypes = [p, i32, d, p]
        L.sl_mesh_smooth_async.restype = ctypes.c_int
        L.sl_mesh_smooth_batch_async.argtypes = [ctypes.POINTER(p), i32, i32, d, p, ctypes.POINTER(BatchReport)]
        L.sl_mesh_smooth_batch_async.restype = ctypes.c_int
        L.sl_mesh_download.argtypes = [p, p, ctypes.POINTER(Report)]
        L.sl_mesh_download.restype = ctypes.c_int
        L.sl_mesh_download_device.argtypes = [p, p, p]
        L.sl_mesh_download_device.restype = ctypes.c_int
        L.sl_mesh_get_report.argtypes = [p, ctypes.POINTER(Report)]
        L.sl_mesh_get_report.restype = ctypes.c_int
        L.sl_mesh_destroy.argtypes = [p]
        L.sl_mesh_destroy.restype = None
        L.sl_release_cached_memory.argtypes = []
        L.sl_release_cached_memory.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != SL_OK:
        raise SmartlapError(status, lib().sl_last_error().decode())


def make_options(form="jacobi", accept="ge", layout="aos", reorder="hilbert", block_size=0, kernel="auto",
                 tile_nodes=0, tile_wg_per_cu=0, precision="f64", lane_width=0, flags_ptr=None):
    o = Options()
    lib().sl_options_default(ctypes.byref(o))
    o.form = FORMS[form] if isinstance(form, str) else int(form)
    o.accept = ACCEPT[accept] if isinstance(accept, str) else int(accept)
    o.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
    o.reorder = REORDER[reorder] if isinstance(reorder, str) else int(reorder)
    o.block_size = int(block_size)
    o.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.tile_nodes = int(tile_nodes)
    o.tile_wg_per_cu = int(tile_wg_per_cu)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.lane_width = int(lane_width)
    o.flags_out = flags_ptr
    return o


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def smooth_mesh(coords, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, boundary, iterations: int, tol: float = 0.0,
                want_flags: bool = False, **opts):
    """Host arrays in, host arrays out.  Returns (coords, report, flags) where
    flags is None or an (iterations, ceil(n/8)) uint8 bit array."""
    X = _c(coords, np.float64).copy()
    n = X.shape[0]
    arrs = [_c(nbr_ptr, np.int32), _c(nbr_idx, np.int32), _c(tri_ptr, np.int32), _c(tri_idx, np.int32),
            _c(tris, np.int32).reshape(-1), _c(boundary, np.uint8)]
    flags = np.zeros((iterations, (n + 7) // 8), np.uint8) if want_flags else None
    o = make_options(flags_ptr=flags.ctypes.data if (flags is not None and flags.size) else None, **opts)
    rep = Report()
    st = lib().smooth_mesh(X.ctypes.data, n, arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                           arrs[3].ctypes.data, arrs[4].ctypes.data, arrs[4].size // 3, arrs[5].ctypes.data,
                           int(iterations), float(tol), ctypes.byref(o), ctypes.byref(rep))
    _check(st)
    return X, rep, flags


def smooth_mesh_device(coords, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, boundary, iterations: int,
                       tol: float = 0.0, flags=None, stream=None, **opts) -> Report:
    """Device tensors (torch, on the current device); ``coords`` (n, 2)
    float64 is overwritten.  ``flags``: optional uint8 device tensor of
    iterations * ceil(n/8) bytes.  Runs on ``stream`` (default: torch's
    current stream)."""
    return _device_call(lib().smooth_mesh_device, coords, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, boundary,
                        iterations, tol, flags, stream, opts)


def smooth_mesh_device_noalloc(coords, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, boundary, iterations: int,
                               tol: float = 0.0, flags=None, stream=None, **opts) -> Report:
    """As smooth_mesh_device, through the entry point that allocates no
    device memory (every array of the call lives in the library's static
    workspace; meshes too large for it raise SL_ENOMEM)."""
    return _device_call(lib().smooth_mesh_device_noalloc, coords, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris,
                        boundary, iterations, tol, flags, stream, opts)


def _device_call(fn, coords, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, boundary, iterations, tol, flags, stream,
                 opts) -> Report:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    for t, dt in ((coords, torch.float64), (nbr_ptr, torch.int32), (nbr_idx, torch.int32), (tri_ptr, torch.int32),
                  (tri_idx, torch.int32), (tris, torch.int32), (boundary, torch.uint8)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError("expected a contiguous %s device tensor" % dt)
    if flags is not None and (not flags.is_cuda or flags.dtype != torch.uint8):
        raise TypeError("flags must be a uint8 device tensor")
    o = make_options(flags_ptr=flags.data_ptr() if flags is not None and flags.numel() else None, **opts)
    rep = Report()
    st = fn(coords.data_ptr(), coords.shape[0], nbr_ptr.data_ptr(), nbr_idx.data_ptr(), tri_ptr.data_ptr(),
            tri_idx.data_ptr(), tris.data_ptr(), tris.numel() // 3, boundary.data_ptr(), int(iterations), float(tol),
            ctypes.byref(o), ctypes.byref(rep), ctypes.c_void_p(stream.cuda_stream))
    _check(st)
    return rep


def _desc(mesh, copy_coords=True):
    """(MeshDesc, arrays kept alive) for a host mesh; coords copied (output)
    unless copy_coords is False (read-only use)."""
    X = _c(mesh.coords, np.float64)
    if copy_coords:
        X = X.copy()
    keep = [X] + [_c(getattr(mesh, f), np.int32) for f in ("nbr_ptr", "nbr_idx", "tri_ptr", "tri_idx")]
    tr = _c(mesh.tris, np.int32).reshape(-1)
    b = _c(mesh.boundary, np.uint8)
    keep += [tr, b]
    d = MeshDesc(X.ctypes.data, X.shape[0], tr.size // 3, keep[1].ctypes.data, keep[2].ctypes.data,
                 keep[3].ctypes.data, keep[4].ctypes.data, tr.ctypes.data, b.ctypes.data)
    return d, keep


def batch_smooth(meshes, iterations: int, tol: float = 0.0, **opts):
    """Smooths many meshes in one batched run.  Returns (list of result
    coordinate arrays, list of Report, BatchReport)."""
    if len(meshes) > 64:
        # the output copies on host threads (numpy copies run without the
        # GIL): a first copy into fresh pages is bound by page faults
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
            descs, keeps = zip(*ex.map(_desc, meshes))
    else:
        descs, keeps = zip(*[_desc(m) for m in meshes])
    arr = (MeshDesc * len(descs))(*descs)
    reps = (Report * len(descs))()
    br = BatchReport()
    o = make_options(**opts)
    st = lib().sl_batch_smooth(arr, len(descs), int(iterations), float(tol), ctypes.byref(o), reps, ctypes.byref(br))
    _check(st)
    return [k[0] for k in keeps], list(reps), br


def build_adjacency(n_nodes: int, tris):
    """Host triangle list -> (nbr_ptr, nbr_idx, tri_ptr, tri_idx, boundary),
    built on the device (sl_build_adjacency)."""
    tr = _c(tris, np.int32).reshape(-1)
    T = tr.size // 3
    nnz = ctypes.c_int64(0)
    _check(lib().sl_build_adjacency(tr.ctypes.data, T, int(n_nodes), None, None, 0, None, None, None,
                                    ctypes.byref(nnz)))
    nbr_ptr = np.empty(n_nodes + 1, np.int32)
    nbr_idx = np.empty(max(nnz.value, 1), np.int32)
    tri_ptr = np.empty(n_nodes + 1, np.int32)
    tri_idx = np.empty(max(3 * T, 1), np.int32)
    bnd = np.empty(n_nodes, np.uint8)
    _check(lib().sl_build_adjacency(tr.ctypes.data, T, int(n_nodes), nbr_ptr.ctypes.data, nbr_idx.ctypes.data,
                                    nbr_idx.size, tri_ptr.ctypes.data, tri_idx.ctypes.data, bnd.ctypes.data,
                                    ctypes.byref(nnz)))
    return nbr_ptr, nbr_idx[: nnz.value], tri_ptr, tri_idx[: 3 * T], bnd


def build_adjacency_device(tris, n_nodes: int, stream=None):
    """Device int32 triangle tensor (n_tris, 3) or (3*n_tris,) -> device
    tensors (nbr_ptr, nbr_idx, tri_ptr, tri_idx, boundary)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    if not tris.is_cuda or tris.dtype != torch.int32 or not tris.is_contiguous():
        raise TypeError("expected a contiguous int32 device tensor")
    T = tris.numel() // 3
    dev = tris.device
    nnz = ctypes.c_int64(0)
    h = ctypes.c_void_p(stream.cuda_stream)
    _check(lib().sl_build_adjacency_device(tris.data_ptr(), T, int(n_nodes), None, None, 0, None, None, None,
                                           ctypes.byref(nnz), h))
    nbr_ptr = torch.empty(n_nodes + 1, dtype=torch.int32, device=dev)
    nbr_idx = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
    tri_ptr = torch.empty(n_nodes + 1, dtype=torch.int32, device=dev)
    tri_idx = torch.empty(max(3 * T, 1), dtype=torch.int32, device=dev)
    bnd = torch.empty(n_nodes, dtype=torch.uint8, device=dev)
    _check(lib().sl_build_adjacency_device(tris.data_ptr(), T, int(n_nodes), nbr_ptr.data_ptr(), nbr_idx.data_ptr(),
                                           nbr_idx.numel(), tri_ptr.data_ptr(), tri_idx.data_ptr(), bnd.data_ptr(),
                                           ctypes.byref(nnz), h))
    return nbr_ptr, nbr_idx[: nnz.value], tri_ptr, tri_idx[: 3 * T], bnd


def autotune(meshes, **opts) -> Tuning:
    """Times the sweep launch shapes on (a sample of) these host meshes and
    makes the fastest the device's automatic choice (sl_autotune)."""
    descs, keeps = zip(*[_desc(m, copy_coords=False) for m in meshes])
    arr = (MeshDesc * len(descs))(*descs)
    t = Tuning()
    o = make_options(**opts)
    _check(lib().sl_autotune(arr, len(descs), ctypes.byref(o), ctypes.byref(t)))
    return t


def autotune_reset():
    lib().sl_autotune_reset()


class RequestResult:
    def __init__(self, status, coords, report, times, message=""):
        self.status = status
        self.coords = coords
        self.report = report
        self.times = times
        self.message = message


class Server:
    """Continuous-batching smoothing server (sl_server_* in the C ABI).
    The arrays of a submitted mesh are kept referenced here until its
    result has been polled."""

    def __init__(self, hbm_budget_bytes=0, max_active=0, sweeps_per_step=0, setup_threads=0, **opts):
        cfg = ServerConfig()
        lib().sl_server_config_default(ctypes.byref(cfg))
        if hbm_budget_bytes:
            cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        if max_active:
            cfg.max_active = int(max_active)
        if sweeps_per_step:
            cfg.sweeps_per_step = int(sweeps_per_step)
        if setup_threads:
            cfg.setup_threads = int(setup_threads)
        self.config = cfg
        o = make_options(**opts)
        h = ctypes.c_void_p()
        _check(lib().sl_server_create(ctypes.byref(cfg), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, mesh, iterations: int, tol: float = 0.0, deadline_s: float = 0.0) -> int:
        d, keep = _desc(mesh)
        rid = ctypes.c_uint64()
        _check(lib().sl_server_submit(self._h, ctypes.byref(d), int(iterations), float(tol), float(deadline_s),
                                      ctypes.byref(rid)))
        self._keep[rid.value] = (d, keep)
        return rid.value

    def poll(self, rid: int):
        """None while the request runs, else a RequestResult."""
        d, keep = self._keep[rid]
        out = np.empty((d.n_nodes, 2), np.float64)
        rep, tm = Report(), RequestTimes()
        st = lib().sl_server_poll(self._h, rid, out.ctypes.data, ctypes.byref(rep), ctypes.byref(tm))
        if st == SL_EBUSY:
            return None
        del self._keep[rid]
        msg = lib().sl_last_error().decode() if st != SL_OK else ""
        return RequestResult(st, out if st == SL_OK else None, rep, tm, msg)

    def wait(self, rid: int, timeout: float = 600.0, interval: float = 0.0005):
        import time
        t0 = time.time()
        while True:
            r = self.poll(rid)
            if r is not None:
                return r
            if time.time() - t0 > timeout:
                raise TimeoutError("request %d not done after %g s" % (rid, timeout))
            time.sleep(interval)

    def cancel(self, rid: int):
        _check(lib().sl_server_cancel(self._h, rid))

    def stats(self) -> ServerStats:
        s = ServerStats()
        _check(lib().sl_server_get_stats(self._h, ctypes.byref(s)))
        return s

    def close(self):
        if self._h:
            lib().sl_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Mesh:
    """A mesh kept on the device (sl_mesh_* in the C ABI): set up once,
    smoothed any number of times; sweeps continue where the last call
    stopped.  ``Mesh(host_mesh, **opts)`` uploads a host mesh;
    ``Mesh.from_device(tensors, **opts)`` takes device tensors as returned by
    ``to_device``."""

    def __init__(self, mesh=None, _handle=None, **opts):
        self._h = None
        if _handle is not None:
            self._h, self.n_nodes = _handle
            return
        d, keep = _desc(mesh, copy_coords=False)
        o = make_options(**opts)
        h = ctypes.c_void_p()
        _check(lib().sl_mesh_create(ctypes.byref(d), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.n_nodes = d.n_nodes

    @classmethod
    def from_device(cls, tensors, stream=None, **opts):
        import torch
        coords, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, boundary = tensors
        if stream is None:
            stream = torch.cuda.current_stream()
        o = make_options(**opts)
        h = ctypes.c_void_p()
        _check(lib().sl_mesh_create_device(coords.data_ptr(), coords.shape[0], nbr_ptr.data_ptr(),
                                           nbr_idx.data_ptr(), tri_ptr.data_ptr(), tri_idx.data_ptr(),
                                           tris.data_ptr(), tris.numel() // 3, boundary.data_ptr(), ctypes.byref(o),
                                           ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        return cls(_handle=(h, coords.shape[0]))

    @staticmethod
    def _stream(stream):
        import torch
        return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)

    def smooth_async(self, iterations: int, tol: float = 0.0, stream=None):
        """Queues sweeps on ``stream`` (default: torch's current stream);
        returns without waiting when tol <= 0."""
        _check(lib().sl_mesh_smooth_async(self._h, int(iterations), float(tol), self._stream(stream)))

    def download(self):
        """(positions (n, 2) float64 in the caller's node order, Report)."""
        out = np.empty((self.n_nodes, 2), np.float64)
        rep = Report()
        _check(lib().sl_mesh_download(self._h, out.ctypes.data, ctypes.byref(rep)))
        return out, rep

    def download_device(self, out, stream=None):
        """Queues the positions into the (n, 2) float64 device tensor ``out``."""
        import torch
        if not out.is_cuda or out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != 2 * self.n_nodes:
            raise TypeError("expected a contiguous (n, 2) float64 device tensor")
        _check(lib().sl_mesh_download_device(self._h, out.data_ptr(), self._stream(stream)))

    def report(self) -> Report:
        rep = Report()
        _check(lib().sl_mesh_get_report(self._h, ctypes.byref(rep)))
        return rep

    def close(self):
        if self._h:
            lib().sl_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def smooth_batch_async(handles, iterations: int, tol: float = 0.0, stream=None) -> BatchReport:
    """Sweeps several Mesh handles together (sl_mesh_smooth_batch_async)."""
    arr = (ctypes.c_void_p * len(handles))(*[h._h.value for h in handles])
    br = BatchReport()
    _check(lib().sl_mesh_smooth_batch_async(arr, len(handles), int(iterations), float(tol), Mesh._stream(stream),
                                            ctypes.byref(br)))
    return br


def release_cached_memory():
    """Returns the device memory the library keeps for reuse (sl_release_cached_memory)."""
    _check(lib().sl_release_cached_memory())


def to_device(mesh, device="cuda"):
    """Copies a mesh's arrays (objects with the meshgen.Mesh attributes) to
    device tensors: (coords, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris, boundary)."""
    import torch
    f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)  # noqa: E731
    return (f(mesh.coords, np.float64), f(mesh.nbr_ptr, np.int32), f(mesh.nbr_idx, np.int32),
            f(mesh.tri_ptr, np.int32), f(mesh.tri_idx, np.int32), f(mesh.tris, np.int32).reshape(-1),
            f(mesh.boundary, np.uint8))


def unpack_flags(bits: np.ndarray, n: int) -> np.ndarray:
    """(iterations, ceil(n/8)) bit bytes -> (iterations, n) 0/1."""
    bits = np.asarray(bits, dtype=np.uint8)
    return np.unpackbits(bits, axis=1, bitorder="little")[:, :n]


def header_symbols():
    """Function names declared with SL_API in include/smartlap.h."""
    import re
    src = open(HEADER).read()
    return re.findall(r"^SL_API\s+[^;(]*?\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
