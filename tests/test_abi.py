"""The C-ABI library loads and exports every entry point its header declares.

No compute call is made here (no GPU in this environment); only argument
checks that return before any device work.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import paper_1502_00355_amd as sl


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sl.LIB_PATH):
        pytest.fail("libsmartlap.so not built: run __graft_entry__.build()")
    return sl.lib()


def test_header_symbols_are_exported(L):
    names = sl.header_symbols()
    assert {"smooth_mesh", "smooth_mesh_device", "sl_last_error", "sl_options_default", "sl_version"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", sl.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for n in names:
        assert n in exported, n
        getattr(L, n)


def test_library_built_from_other_sources_is_refused(L, monkeypatch):
    """The binding refuses an in-tree library whose recorded source digest
    differs from the sources beside it, so that no test runs old code."""
    from paper_1502_00355_amd import build
    monkeypatch.setattr(sl, "_lib", None)
    monkeypatch.setattr(build, "source_digest", lambda: "0" * 64)
    with pytest.raises(RuntimeError, match="not built from the sources"):
        sl.lib()


def test_only_the_c_abi_is_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", sl.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert exported <= set(sl.header_symbols()) | {"_init", "_fini"}, exported - set(sl.header_symbols())


def test_option_defaults(L):
    o = sl.Options()
    L.sl_options_default(ctypes.byref(o))
    assert (o.form, o.accept, o.layout, o.reorder, o.block_size, o.kernel) == (0, 0, 0, 1, 0, 0)
    assert (o.tile_nodes, o.tile_wg_per_cu, o.lane_width) == (0, 0, 0)
    assert not o.flags_out
    assert L.sl_version().startswith(b"smartlap")


def _call(n_nodes=4, iterations=1, null_coords=False):
    X = np.zeros((4, 2))
    ptr = np.zeros(5, np.int32)
    idx = np.zeros(1, np.int32)
    b = np.ones(4, np.uint8)
    return sl.lib().smooth_mesh(None if null_coords else X.ctypes.data, n_nodes, ptr.ctypes.data, idx.ctypes.data,
                                ptr.ctypes.data, idx.ctypes.data, idx.ctypes.data, 0, b.ctypes.data, iterations,
                                0.0, None, None)


def test_argument_errors_before_device_work(L):
    assert _call(n_nodes=0) == sl.SL_EINVAL
    assert b"n_nodes" in L.sl_last_error()
    assert _call(iterations=-1) == sl.SL_EINVAL
    assert _call(null_coords=True) == sl.SL_EINVAL
    assert b"null" in L.sl_last_error()


def test_server_config_defaults(L):
    c = sl.ServerConfig()
    L.sl_server_config_default(ctypes.byref(c))
    assert c.hbm_budget_bytes == 200 << 30 and c.max_active == 256 and c.sweeps_per_step == 8


def test_tile_option_errors_before_device_work(L):
    X = np.zeros((4, 2))
    ptr = np.zeros(5, np.int32)
    idx = np.zeros(1, np.int32)
    b = np.ones(4, np.uint8)
    for kw in ({"tile_nodes": 384}, {"tile_wg_per_cu": 9}, {"tile_wg_per_cu": -1}, {"block_size": 96},
               {"lane_width": 6}, {"lane_width": 32}, {"kernel": "lanes", "precision": "f32"},
               {"kernel": 7}, {"form": 5}):
        o = sl.make_options(**kw)
        st = L.smooth_mesh(X.ctypes.data, 4, ptr.ctypes.data, idx.ctypes.data, ptr.ctypes.data, idx.ctypes.data,
                           idx.ctypes.data, 0, b.ctypes.data, 1, 0.0, ctypes.byref(o), None)
        assert st == sl.SL_EINVAL, kw
    assert b"tile_wg_per_cu" in L.sl_last_error() or b"form" in L.sl_last_error()


def test_autotune_argument_errors(L):
    t = sl.Tuning()
    assert L.sl_autotune(None, 1, None, ctypes.byref(t)) == sl.SL_EINVAL
    d = sl.MeshDesc()
    d.n_nodes = 0
    arr = (sl.MeshDesc * 1)(d)
    assert L.sl_autotune(arr, 1, None, ctypes.byref(t)) == sl.SL_EINVAL
    assert b"n_nodes" in L.sl_last_error()
    o = sl.make_options(form=3)
    d.n_nodes = 4
    assert L.sl_autotune(arr, 1, ctypes.byref(o), ctypes.byref(t)) == sl.SL_EINVAL


def test_adjacency_argument_errors_before_device_work(L):
    tris = np.array([0, 1, 2], np.int32)
    nnz = ctypes.c_int64(-1)
    assert L.sl_build_adjacency(tris.ctypes.data, 1, 0, None, None, 0, None, None, None, ctypes.byref(nnz)) == \
        sl.SL_EINVAL
    assert b"n_nodes" in L.sl_last_error()
    assert L.sl_build_adjacency(tris.ctypes.data, -1, 3, None, None, 0, None, None, None, ctypes.byref(nnz)) == \
        sl.SL_EINVAL
    assert L.sl_build_adjacency(None, 1, 3, None, None, 0, None, None, None, ctypes.byref(nnz)) == sl.SL_EINVAL
    assert L.sl_build_adjacency(tris.ctypes.data, 1, 3, None, None, 0, None, None, None, None) == sl.SL_EINVAL
    out = np.zeros(8, np.int32)
    assert L.sl_build_adjacency(tris.ctypes.data, 1, 3, None, out.ctypes.data, 8, None, None, None,
                                ctypes.byref(nnz)) == sl.SL_EINVAL
    assert b"null output" in L.sl_last_error()
    assert nnz.value == -1


STRUCTS = {"Options": "sl_options", "Report": "sl_report", "MeshDesc": "sl_mesh_desc",
           "BatchReport": "sl_batch_report", "Tuning": "sl_tuning", "ServerConfig": "sl_server_config",
           "RequestTimes": "sl_request_times", "ServerStats": "sl_server_stats"}


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding marshals has the header's size and field
    offsets (a C program built from include/smartlap.h prints them)."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "smartlap.h"', "int main(void) {"]
    want = {}
    for py, c in STRUCTS.items():
        cls = getattr(sl, py)
        lines.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (py, c))
        want[py] = ctypes.sizeof(cls)
        for name, _ in cls._fields_:
            lines.append('printf("%%s %%zu\\n", "%s.%s", offsetof(%s, %s));' % (py, name, c, name))
            want[py + "." + name] = getattr(cls, name).offset
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True,
                                                    check=True).stdout.splitlines())
    assert {k: int(v) for k, v in got.items()} == want
