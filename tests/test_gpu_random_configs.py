"""GPU parity over a seeded sample of the option space.

Each case draws a small mesh (a jittered grid with random or Union-Jack
diagonals, an annulus, a Delaunay triangulation of random points, or a
randomly relabelled copy of one of these, with a share of its free nodes
sometimes marked fixed) and a set of options (form, accept rule, layout,
reorder, kernel, precision, tile shape, node-kernel block size or
lane-group width, sweeps, tolerance), runs it through the C ABI and compares sweep by sweep with the
oracle: accept flags, accepted counts, displacement maxima and coordinates
bit for bit.  The draws are fixed by the case number, so a failure names a
reproducible case.
"""
import sys

import numpy as np
import pytest

import meshgen
import oracle
import paper_1502_00355_amd as sl

pytestmark = pytest.mark.gpu

N_CASES = 200


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    sl.lib()
    yield


def draw_mesh(rng):
    kind = rng.choice(["grid", "unionjack", "annulus", "delaunay"])
    seed = int(rng.integers(1 << 20))
    if kind == "grid":
        m = meshgen.make_grid(int(rng.integers(3, 90)), "random", float(rng.uniform(0.0, 0.45)), seed)
    elif kind == "unionjack":
        m = meshgen.make_grid(int(rng.integers(3, 90)), "unionjack", float(rng.uniform(0.0, 0.45)), seed)
    elif kind == "annulus":
        m = meshgen.make_annulus(int(rng.integers(3, 40)), int(rng.integers(6, 120)), seed=seed)
    else:
        m = meshgen.make_delaunay(int(rng.integers(20, 6000)), seed)
    if rng.uniform() < 0.3:
        m = meshgen.permute_mesh(m, seed + 1)
    if rng.uniform() < 0.2:
        # some interior nodes held fixed as well
        free = np.flatnonzero(m.boundary == 0)
        pick = rng.choice(free, size=len(free) // 5, replace=False) if len(free) else free
        m.boundary = m.boundary.copy()
        m.boundary[pick] = 1
    return m, kind


def draw_options(rng, n_nodes):
    form = "colored" if rng.uniform() < 0.35 else "jacobi"
    o = {"form": form,
         "accept": "gt" if rng.uniform() < 0.3 else "ge",
         "layout": "soa" if rng.uniform() < 0.4 else "aos",
         "reorder": "none" if rng.uniform() < 0.3 else "hilbert"}
    kernels = ["auto", "auto", "node", "tile"] + (["resident"] if n_nodes <= 1500 else [])
    o["kernel"] = str(rng.choice(kernels))
    if o["kernel"] == "node":
        o["block_size"] = int(rng.choice([0, 64, 128, 256]))
        if o["block_size"] in (64, 128):
            # the lane-group kernel instead, its width taken from the same draw
            o["kernel"] = "lanes"
            o["lane_width"] = 4 if o.pop("block_size") == 64 else 16
    if o["kernel"] in ("auto", "tile"):
        sizes = [0, 256, 512] + ([128] if form == "colored" else [])
        o["tile_nodes"] = int(rng.choice(sizes))
        o["tile_wg_per_cu"] = int(rng.integers(0, 9))
    if form == "jacobi" and o["kernel"] in ("auto", "tile") and rng.uniform() < 0.25:
        o["precision"] = "f32"
    return o


@pytest.mark.parametrize("case", range(N_CASES))
def test_random_config(case):
    import torch
    rng = np.random.Generator(np.random.PCG64(7_000_000 + case))
    m, kind = draw_mesh(rng)
    opts = draw_options(rng, m.n_nodes)
    iters = int(rng.integers(1, 25))
    tol = float(10.0 ** rng.uniform(-9, -3)) if rng.uniform() < 0.3 else 0.0
    prec = opts.get("precision", "f64")
    print("case %d: %s %s, %d nodes, %d sweeps, tol %g, %s" % (case, kind, m.name, m.n_nodes, iters, tol, opts),
          flush=True)
    sys.stdout.flush()
    dev = sl.to_device(m, "cuda:0")
    nbytes = (m.n_nodes + 7) // 8
    flags = torch.zeros(iters * nbytes, dtype=torch.uint8, device="cuda:0")
    try:
        rep = sl.smooth_mesh_device(*dev, iterations=iters, tol=tol, flags=flags, **opts)
    except sl.SmartlapError as e:
        # an explicit tile or resident kernel, and single precision, need a
        # mesh that path takes; they refuse others with SL_EINVAL
        assert e.status == sl.SL_EINVAL and (opts["kernel"] in ("tile", "resident") or prec == "f32"), str(e)
        return
    torch.cuda.synchronize()
    X = dev[0].cpu().numpy()
    F = sl.unpack_flags(flags.cpu().numpy().reshape(iters, nbytes), m.n_nodes)
    ref = oracle.smooth(m, iters, tol=tol, accept_gt=(opts["accept"] == "gt"), threads=oracle.max_threads(),
                        form=opts["form"], precision=prec)
    k = ref.iterations_run
    assert rep.iterations_run == k
    assert (F[:k] == (ref.flags == 1)).all(), "flags differ in sweeps %s" % np.flatnonzero(
        (F[:k] != (ref.flags == 1)).any(axis=1))
    assert (F[k:] == 0).all()
    assert np.array_equal(X, ref.coords), float(np.abs(X - ref.coords).max())
    if k:
        assert rep.accepted_last == ref.accepted[-1]
        assert rep.accepted_total == int(ref.accepted.sum())
        assert rep.max_disp_sq_last == ref.disp[-1]


N_BATCHES = 24


@pytest.mark.parametrize("case", range(N_BATCHES))
def test_random_batch(case):
    """Batches of 1-24 random meshes under one random option set: every
    mesh's result, sweep count and accepted counts equal the oracle's."""
    rng = np.random.Generator(np.random.PCG64(8_000_000 + case))
    meshes = [draw_mesh(rng)[0] for _ in range(int(rng.integers(1, 25)))]
    opts = draw_options(rng, max(m.n_nodes for m in meshes))
    opts.pop("tile_nodes", None)          # a batch takes the automatic tile shape
    opts.pop("tile_wg_per_cu", None)
    if opts["kernel"] == "tile":
        opts["kernel"] = "auto"
    iters = int(rng.integers(1, 25))
    tol = float(10.0 ** rng.uniform(-9, -3)) if rng.uniform() < 0.3 else 0.0
    prec = opts.get("precision", "f64")
    print("batch %d: %d meshes (%d nodes), %d sweeps, tol %g, %s" %
          (case, len(meshes), sum(m.n_nodes for m in meshes), iters, tol, opts), flush=True)
    try:
        outs, reps, br = sl.batch_smooth(meshes, iters, tol=tol, **opts)
    except sl.SmartlapError as e:
        assert e.status == sl.SL_EINVAL and (opts["kernel"] == "resident" or prec == "f32"), str(e)
        return
    for m, X, rep in zip(meshes, outs, reps):
        ref = oracle.smooth(m, iters, tol=tol, accept_gt=(opts["accept"] == "gt"), threads=oracle.max_threads(),
                            form=opts["form"], precision=prec)
        assert rep.iterations_run == ref.iterations_run, m.name
        assert np.array_equal(X, ref.coords), (m.name, float(np.abs(X - ref.coords).max()))
        if ref.iterations_run:
            assert rep.accepted_last == ref.accepted[-1], m.name
            assert rep.accepted_total == int(ref.accepted.sum()), m.name


N_HANDLE_CASES = 24


@pytest.mark.parametrize("case", range(N_HANDLE_CASES))
def test_random_handles(case):
    """1-6 mesh handles under one drawn option set: smoothed alone, then
    together, then alone again, each call with its own sweep count and
    tolerance; every handle ends where the oracle does after the same three
    calls, with the same accepted total."""
    import torch
    rng = np.random.Generator(np.random.PCG64(9_000_000 + case))
    meshes = [draw_mesh(rng)[0] for _ in range(int(rng.integers(1, 7)))]
    opts = draw_options(rng, 10 ** 9)                 # no resident kernel: handles do not run it
    opts.pop("tile_wg_per_cu", None)
    calls = [(int(rng.integers(0, 16)), float(10.0 ** rng.uniform(-8, -3)) if rng.uniform() < 0.3 else 0.0)
             for _ in range(3)]
    on_device = bool(rng.uniform() < 0.5)
    prec = opts.get("precision", "f64")
    print("handles %d: %d meshes, calls %s, %s, from device %s" % (case, len(meshes), calls, opts, on_device),
          flush=True)
    hs = []
    try:
        for m in meshes:
            hs.append(sl.Mesh.from_device(sl.to_device(m, "cuda:0"), **opts) if on_device else sl.Mesh(m, **opts))
    except sl.SmartlapError as e:
        assert e.status == sl.SL_EINVAL and (opts["kernel"] == "tile" or prec == "f32"), str(e)
        for h in hs:
            h.close()
        return
    try:
        (k1, t1), (k2, t2), (k3, t3) = calls
        for h in hs:
            h.smooth_async(k1, t1)
        sl.smooth_batch_async(hs, max(k2, 1), t2)
        for h in hs:
            h.smooth_async(k3, t3)
        torch.cuda.synchronize()
        for m, h in zip(meshes, hs):
            X, rep = h.download()
            cur, acc = m, 0
            for k, t in ((k1, t1), (max(k2, 1), t2), (k3, t3)):
                ref = oracle.smooth(cur, k, tol=t, accept_gt=(opts["accept"] == "gt"),
                                    threads=oracle.max_threads(), form=opts["form"], precision=prec)
                acc += int(ref.accepted.sum())
                cur = cur.copy()
                cur.coords = ref.coords
            assert np.array_equal(X, cur.coords), (m.name, float(np.abs(X - cur.coords).max()))
            assert rep.accepted_total == acc, m.name
    finally:
        for h in hs:
            h.close()


N_SERVER_CASES = 8


@pytest.mark.parametrize("case", range(N_SERVER_CASES))
def test_random_server(case):
    """A server with a drawn configuration (HBM budget, active-request cap,
    sweeps per step, setup threads) and option set takes 8-40 random
    requests submitted at once, each with its own sweep count and tolerance;
    every result equals the oracle's for that request alone."""
    rng = np.random.Generator(np.random.PCG64(10_000_000 + case))
    opts = draw_options(rng, 10 ** 9)
    opts.pop("tile_nodes", None)
    opts.pop("tile_wg_per_cu", None)
    if opts["kernel"] == "tile":
        opts["kernel"] = "auto"
    cfg = {"hbm_budget_bytes": int(rng.choice([0, 64 << 20, 256 << 20])),
           "max_active": int(rng.choice([0, 1, 3, 16])),
           "sweeps_per_step": int(rng.choice([0, 1, 3, 8])),
           "setup_threads": int(rng.choice([0, 1, 4]))}
    reqs = []
    for _ in range(int(rng.integers(8, 41))):
        m = draw_mesh(rng)[0]
        reqs.append((m, int(rng.integers(0, 30)), float(10.0 ** rng.uniform(-8, -3)) if rng.uniform() < 0.4 else 0.0))
    prec = opts.get("precision", "f64")
    print("server %d: %s, %s, %d requests" % (case, cfg, opts, len(reqs)), flush=True)
    with sl.Server(**cfg, **opts) as srv:
        ids = [srv.submit(m, k, tol=t) for m, k, t in reqs]
        for (m, k, t), rid in zip(reqs, ids):
            r = srv.wait(rid, timeout=100.0)
            if r.status != sl.SL_OK:
                # single precision needs a mesh the tile path takes
                assert r.status == sl.SL_EINVAL and prec == "f32", r.message
                continue
            ref = oracle.smooth(m, k, tol=t, accept_gt=(opts["accept"] == "gt"), threads=oracle.max_threads(),
                                form=opts["form"], precision=prec)
            assert r.report.iterations_run == ref.iterations_run, m.name
            assert np.array_equal(r.coords, ref.coords), (m.name, float(np.abs(r.coords - ref.coords).max()))
            if ref.iterations_run:
                assert r.report.accepted_total == int(ref.accepted.sum()), m.name
