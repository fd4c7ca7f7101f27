"""GPU parity of the lane-group kernel (SL_KERNEL_LANES): W work-items of a
wave per free node, their minima folded with DPP moves inside the group.
Against the oracle, bit for bit: accept flags of every sweep (one bit per
group, gathered from the wave's ballot), accepted counts, displacement
maxima and coordinates, for every width, both layouts, both accept rules,
both forms, every valence class (the kernel's LDS row per group is sized
by the mesh's largest valence), ragged node counts, through one-call
smoothing, handles, batches and the server, and with the width autotuned."""
import sys

import numpy as np
import pytest

import meshgen
import oracle
import paper_1502_00355_amd as sl
from test_gpu_parity import _many_stars, _ring_star, assert_parity, run_gpu

pytestmark = pytest.mark.gpu
LANES = sl.KERNELS["lanes"]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    sl.lib()
    yield


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("width", [4, 8, 16])
@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("accept", ["ge", "gt"])
def test_lanes_parity(width, layout, accept):
    """2,025 free nodes: several work-groups for every width and a ragged last one."""
    m = meshgen.make_grid(47, "random", 0.4, 5)
    X, rep, ref, ndiff = assert_parity(m, 8, accept=accept, layout=layout, kernel="lanes", lane_width=width)
    assert ndiff == 0 and rep.kernel_used == LANES


@pytest.mark.parametrize("width", [4, 8, 16])
@pytest.mark.parametrize("k", [3, 8, 9, 16, 17, 32, 33, 100, 127])
def test_lanes_valence_classes(width, k):
    """One free node of valence k: more slots than lanes, up to the valence limit."""
    X, rep, ref, ndiff = assert_parity(_ring_star(k, k), 3, kernel="lanes", lane_width=width)
    assert ndiff == 0 and rep.kernel_used == LANES


@pytest.mark.parametrize("k", [7, 20, 40])
def test_lanes_many_stars(k):
    """600 free nodes of valence k in one mesh (row lengths 8, 32 and 128)."""
    for width in (4, 16):
        X, rep, ref, ndiff = assert_parity(_many_stars(600, k, 5), 4, kernel="lanes", lane_width=width)
        assert ndiff == 0


@pytest.mark.parametrize("width", [4, 8, 16])
def test_lanes_form_b(width):
    """Coloured, in place, one launch per colour class (class sizes are not
    multiples of the group count)."""
    for m in (meshgen.make_grid(61, "random", 0.4, 12), meshgen.make_delaunay(3000, 13)):
        X, rep, ref, ndiff = assert_parity(m, 6, form="colored", kernel="lanes", lane_width=width)
        assert ndiff == 0 and rep.kernel_used == LANES and rep.n_colors > 0


def test_lanes_delaunay_and_tolerance():
    """A 20K-point Delaunay mesh (valence above 8 and 16), both forms; then
    runs that stop on their tolerance."""
    m = meshgen.make_delaunay(20000, 14)
    for form in ("jacobi", "colored"):
        X, rep, ref, ndiff = assert_parity(m, 10, form=form, kernel="lanes")
        assert ndiff == 0
    g = meshgen.make_grid(40, "random", 0.4, 15)
    for form in ("jacobi", "colored"):
        X, rep, ref, ndiff = assert_parity(g, 5000, tol=1e-9, form=form, kernel="lanes", lane_width=4)
        assert ndiff == 0 and 0 < rep.iterations_run < 5000


def test_lanes_permuted_and_fixed_nodes():
    """Relabelled nodes, no reordering, and interior nodes held fixed."""
    m = meshgen.permute_mesh(meshgen.make_grid(50, "unionjack", 0.3, 16), 17)
    b = m.copy()
    rng = np.random.Generator(np.random.PCG64(18))
    free = np.flatnonzero(b.boundary == 0)
    b.boundary = b.boundary.copy()
    b.boundary[rng.choice(free, size=len(free) // 5, replace=False)] = 1
    for mesh in (m, b):
        X, rep, ref, ndiff = assert_parity(mesh, 7, reorder="none", kernel="lanes", lane_width=16)
        assert ndiff == 0


def test_lanes_handles_batch_and_server():
    """The same kernel behind mesh handles (alone and batched), a batch and
    a server: every result is the oracle's."""
    import torch
    meshes = [meshgen.make_grid(30, "random", 0.4, 20), meshgen.make_delaunay(2500, 21), _many_stars(100, 20, 22)]
    for form in ("jacobi", "colored"):
        note("lanes handles/batch/server, %s" % form)
        hs = [sl.Mesh(m, form=form, kernel="lanes", lane_width=8) for m in meshes]
        try:
            for h in hs:
                h.smooth_async(3)
            sl.smooth_batch_async(hs, 4)
            torch.cuda.synchronize()
            for m, h in zip(meshes, hs):
                X, rep = h.download()
                ref = oracle.smooth(m, 7, threads=oracle.max_threads(), form=form)
                assert (X == ref.coords).all(), m.name
                assert rep.kernel_used == LANES and rep.accepted_total == int(ref.accepted.sum())
        finally:
            for h in hs:
                h.close()
        outs, reps, br = sl.batch_smooth(meshes, 6, form=form, kernel="lanes", lane_width=16)
        for m, X, rep in zip(meshes, outs, reps):
            ref = oracle.smooth(m, 6, threads=oracle.max_threads(), form=form)
            assert (X == ref.coords).all(), m.name
            assert rep.kernel_used == LANES
        with sl.Server(form=form, kernel="lanes", lane_width=4) as srv:
            ids = [srv.submit(m, 5) for m in meshes]
            for m, rid in zip(meshes, ids):
                r = srv.wait(rid, timeout=100.0)
                assert r.status == sl.SL_OK, r.message
                ref = oracle.smooth(m, 5, threads=oracle.max_threads(), form=form)
                assert (r.coords == ref.coords).all(), m.name


def test_lanes_autotune():
    """The tuner times widths 4, 8 and 16 and makes the fastest the
    device's automatic width; the result does not change with it."""
    m = meshgen.make_grid(300, "random", 0.4, 23)
    try:
        t = sl.autotune([m], kernel="lanes")
        assert t.lane_width in (4, 8, 16) and t.tile_nodes == 0 and t.block_size == 0
        d = t.as_dict()
        assert sorted(c[1] for c in d["candidates"]) == [4, 8, 16] and all(c[0] == 0 for c in d["candidates"])
        assert all(c[2] > 0 for c in d["candidates"])
        X, rep, ref, ndiff = assert_parity(m, 5, kernel="lanes")
        assert ndiff == 0 and rep.kernel_used == LANES
    finally:
        sl.autotune_reset()


def test_lanes_refuses_single_precision():
    m = meshgen.make_grid(12, "random", 0.4, 24)
    with pytest.raises(sl.SmartlapError) as e:
        run_gpu(m, 2, kernel="lanes", precision="f32")
    assert e.value.status == sl.SL_EINVAL
