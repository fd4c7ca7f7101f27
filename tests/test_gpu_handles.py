"""GPU tests of mesh handles (sl_mesh_* in the C ABI): a mesh set up once and
smoothed over several calls, alone or batched, against the FP64 oracle run
in one piece.  Bar as in the parity tests: flags and coordinates bit-exact
(coordinates within 1e-12 is the stated tolerance; bit-exact is expected
and asserted)."""
import copy
import sys
import time

import numpy as np
import pytest

import meshgen
import oracle
import paper_1502_00355_amd as sl

pytestmark = pytest.mark.gpu


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


def ref(m, iters, tol=0.0, **kw):
    return oracle.smooth(m, iters, tol=tol, threads=oracle.max_threads(), want_flags=False, **kw)


def moved(m, coords):
    """The same mesh with its positions replaced (the oracle's sweep depends
    on the positions only, so this continues a run)."""
    c = copy.copy(m)
    c.coords = np.ascontiguousarray(coords)
    return c


def _many_stars(count, k, seed):
    """count disjoint ring stars of valence k in one mesh (jittered ring
    radii): the free nodes are the centres, each with k neighbour entries."""
    coords, tris, off = [], [], 0
    for s in range(count):
        rng = np.random.Generator(np.random.PCG64(seed + s))
        ang = np.sort(rng.uniform(0, 2 * np.pi, k))
        ring = np.stack([np.cos(ang), np.sin(ang)], 1) * rng.uniform(0.8, 1.2, (k, 1))
        st = meshgen.star_mesh(rng.uniform(-0.2, 0.2, 2), ring)
        coords.append(st.coords + np.array([3.0 * (s % 40), 3.0 * (s // 40)]))
        tris.append(st.tris + off)
        off += st.n_nodes
    coords = np.concatenate(coords)
    tris = np.concatenate(tris)
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = meshgen.build_adjacency(coords.shape[0], tris)
    return meshgen.Mesh(coords, tris, nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd, "stars%dx%d" % (count, k))


@pytest.mark.parametrize("splits", [(5, 5), (33, 7, 40), (32, 32), (1, 64, 3)])
def test_calls_continue_where_the_last_stopped(splits):
    """k sweeps, then k' more ... equal one run of k + k' + ... sweeps:
    odd counts leave the positions in the other buffer, and counts of 32 or
    more replay captured chunks."""
    m = meshgen.make_grid(60, "random", 0.4, 201)
    note("handle %s splits %s" % (m.name, splits))
    with sl.Mesh(m) as h:
        for k in splits:
            h.smooth_async(k)
        X, rep = h.download()
    r = ref(m, sum(splits))
    assert rep.iterations_run == sum(splits) == r.iterations_run
    assert (X == r.coords).all()
    assert rep.accepted_last == r.accepted[-1] and rep.accepted_total == int(r.accepted.sum())
    assert rep.kernel_used == sl.KERNELS["tile"]


@pytest.mark.parametrize("opts", [{"layout": "soa"}, {"form": "colored"}, {"form": "colored", "kernel": "tile"},
                                  {"precision": "f32"}, {"kernel": "node"}, {"accept": "gt"}, {"reorder": "none"}])
def test_options(opts):
    m = meshgen.permute_mesh(meshgen.make_grid(45, "random", 0.4, 202), 3)
    note("handle options %s" % opts)
    with sl.Mesh(m, **opts) as h:
        h.smooth_async(9)
        h.smooth_async(12)
        X, rep = h.download()
    kw = {}
    if opts.get("form") == "colored":
        kw["form"] = "colored"
    if opts.get("precision") == "f32":
        kw["precision"] = "f32"
    r = ref(m, 21, accept_gt=opts.get("accept") == "gt", **kw)
    assert rep.iterations_run == 21
    assert (X == r.coords).all()
    if opts.get("form") == "colored":
        # automatic Form B: the node kernel; colour-class tiles on request
        assert rep.kernel_used == sl.KERNELS[opts.get("kernel", "node")] and rep.n_colors > 0


def test_form_b_handles_on_class_tiles_and_node_kernel_batched():
    """Form B handles asking for colour-class tiles: a grid and a Delaunay
    mesh on them, and a mesh of stars too dense for tiles on the node kernel,
    smoothed alone and batched; every one equals the oracle's coloured
    sweeps."""
    ms = [meshgen.make_grid(70, "random", 0.4, 31), meshgen.make_delaunay(4000, 32), _many_stars(300, 20, 33)]
    hs = [sl.Mesh(m, form="colored", kernel="tile") for m in ms]
    try:
        kinds = [h.report().kernel_used for h in hs]
        assert kinds == [sl.KERNELS["tile"], sl.KERNELS["tile"], sl.KERNELS["node"]], kinds
        for h in hs:
            h.smooth_async(5)
        sl.smooth_batch_async(hs, 7)
        hs[0].smooth_async(3)
        for m, h, k in zip(ms, hs, (15, 12, 12)):
            X, rep = h.download()
            r = ref(m, k, form="colored")
            assert rep.iterations_run == k and (X == r.coords).all(), m.name
            assert rep.accepted_total == int(r.accepted.sum()), m.name
    finally:
        for h in hs:
            h.close()


def test_async_returns_before_the_work_and_overlaps_a_caller_kernel():
    """With no tolerance the call only queues work: right after it returns
    the stream still has work, and a caller kernel on another stream runs
    meanwhile; the results of both are right afterwards."""
    import torch
    m = meshgen.make_grid(1024, "random", 0.4, 203)
    note("handle async 1024^2")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = torch.randn(4096, 4096, device="cuda", dtype=torch.float32)
    want = (a.double() @ a.double()).float()
    with sl.Mesh(m) as h:
        h.smooth_async(2)                 # graphs and first-use costs out of the way
        h.download()
        t0 = time.perf_counter()
        h.smooth_async(200, stream=s1)
        t_call = time.perf_counter() - t0
        pending = not s1.query()
        with torch.cuda.stream(s2):
            c = a @ a
        s2.synchronize()
        s1.synchronize()
        t_all = time.perf_counter() - t0
        X, rep = h.download()
    assert pending, "the call waited for its sweeps"
    assert t_call < t_all / 4, (t_call, t_all)
    assert torch.allclose(c, want, rtol=1e-3, atol=1e-2)
    r = ref(m, 202)
    assert rep.iterations_run == 202 and (X == r.coords).all()


def test_tolerance_and_continuing():
    m = meshgen.make_grid(40, "random", 0.4, 204)
    full = ref(m, 400)
    moving = np.flatnonzero(full.disp > 0)
    tol = float(np.sqrt(full.disp[moving[len(moving) // 3]])) * 1.0000001
    note("handle tol %g" % tol)
    with sl.Mesh(m) as h:
        h.smooth_async(400, tol=tol)
        X, rep = h.download()
        r = ref(m, 400, tol=tol)
        assert rep.iterations_run == r.iterations_run < 400
        assert (X == r.coords).all()
        # ten more without a tolerance, then to a tighter one
        h.smooth_async(10)
        X2, rep2 = h.download()
        r2 = ref(moved(m, r.coords), 10)
        assert rep2.iterations_run == r.iterations_run + 10 and (X2 == r2.coords).all()
        tol2 = tol / 4
        h.smooth_async(400, tol=tol2)
        X3, rep3 = h.download()
        r3 = ref(moved(m, r2.coords), 400, tol=tol2)
        assert rep3.iterations_run == rep2.iterations_run + r3.iterations_run
        assert (X3 == r3.coords).all()


def _star_cluster(n_stars, ring, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    meshes = []
    for k in range(n_stars):
        ang = np.sort(rng.uniform(0, 2 * np.pi, ring))
        pts = np.stack([np.cos(ang), np.sin(ang)], 1) * rng.uniform(0.8, 1.2, (ring, 1))
        meshes.append(meshgen.star_mesh(rng.uniform(-0.2, 0.2, 2), pts))
    return meshes


def test_batch_of_handles_equals_each_alone():
    """Handles of uneven size, at different sweep counts (some with their
    positions in buffer 1), one too dense for the tile path, swept together:
    each equals the oracle over its own total."""
    import torch
    ms = [meshgen.make_grid(n, "random", 0.35, 300 + n) for n in (17, 64, 129, 200)]
    ms.append(meshgen.make_annulus(30, 48, seed=5))
    ms.append(_many_stars(600, 20, 5))   # 20 entries per node on average: too dense for the tiles
    pre = [0, 1, 3, 32, 7, 2]
    hs = [sl.Mesh(m) for m in ms]
    try:
        for h, k in zip(hs, pre):
            if k:
                h.smooth_async(k)
        s = torch.cuda.Stream()
        br = sl.smooth_batch_async(hs, 11, stream=s)
        assert br.meshes_on_tile_path == sum(h.report().kernel_used == sl.KERNELS["tile"] for h in hs)
        sl.smooth_batch_async(hs, 6, stream=s)
        for m, h, k in zip(ms, hs, pre):
            X, rep = h.download()
            r = ref(m, k + 17)
            assert rep.iterations_run == k + 17
            assert (X == r.coords).all(), m.name
        assert hs[-1].report().kernel_used == sl.KERNELS["node"]
        # a tolerance: each stops on its own
        br = sl.smooth_batch_async(hs[:4], 500, tol=1e-7)
        for m, h, k in zip(ms[:4], hs[:4], pre[:4]):
            X, rep = h.download()
            start = ref(m, k + 17).coords
            r = ref(moved(m, start), 500, tol=1e-7)
            assert rep.iterations_run == k + 17 + r.iterations_run
            assert (X == r.coords).all()
    finally:
        for h in hs:
            h.close()


def test_download_device_and_create_device():
    import torch
    m = meshgen.make_grid(70, "random", 0.4, 205)
    dev = sl.to_device(m, "cuda:0")
    with sl.Mesh.from_device(dev) as h:
        h.smooth_async(13)
        out = torch.empty((m.n_nodes, 2), dtype=torch.float64, device="cuda:0")
        h.download_device(out)
        torch.cuda.synchronize()
        X, rep = h.download()
    assert (out.cpu().numpy() == X).all()
    assert (X == ref(m, 13).coords).all()
    # the caller's arrays were only read
    assert (dev[0].cpu().numpy() == m.coords).all()


def test_handle_errors():
    m = meshgen.make_grid(20, "random", 0.4, 206)
    with pytest.raises(sl.SmartlapError) as e:
        sl.Mesh(m, kernel="resident")
    assert e.value.status == sl.SL_EINVAL
    bad = copy.copy(m)
    bad.tri_idx = m.tri_idx.copy()
    bad.tri_idx[5] = 10 ** 6
    with pytest.raises(sl.SmartlapError) as e:
        sl.Mesh(bad)
    assert e.value.status == sl.SL_EINVAL
    with sl.Mesh(m) as a, sl.Mesh(m, layout="soa") as b:
        with pytest.raises(sl.SmartlapError) as e:
            sl.smooth_batch_async([a, b], 2)
        assert e.value.status == sl.SL_EINVAL
        with pytest.raises(sl.SmartlapError) as e:
            sl.smooth_batch_async([a, a], 2)
        assert e.value.status == sl.SL_EINVAL
        with pytest.raises(sl.SmartlapError) as e:
            a.smooth_async(-1)
        assert e.value.status == sl.SL_EINVAL
        a.smooth_async(3)
        X, rep = a.download()
        assert (X == ref(m, 3).coords).all()


def test_release_cached_memory():
    m = meshgen.make_grid(300, "random", 0.4, 207)
    X0, _, _ = sl.smooth_mesh(m.coords, m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary, 4)
    sl.release_cached_memory()
    X1, _, _ = sl.smooth_mesh(m.coords, m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary, 4)
    assert (X0 == X1).all()
