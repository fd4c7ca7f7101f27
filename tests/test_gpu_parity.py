"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar (Jacobi form): accept/reject flags bit-exact in every sweep, coordinates
within 1e-12 absolute (the arithmetic is the same IEEE sequence on both
sides, so bit-exact is expected and also reported).  Coloured form: the same
colouring on both sides, so the same bar applies; its invariants are checked
too.  Inputs are seeded synthetic meshes from ``meshgen``.
"""
import ctypes
import math
import sys

import numpy as np
import pytest

import meshgen
import oracle
import paper_1502_00355_amd as sl

pytestmark = pytest.mark.gpu
COORD_TOL = 1e-12


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


def run_gpu(m, iters, tol=0.0, want_flags=True, **opts):
    import torch
    dev = sl.to_device(m, "cuda:0")
    nbytes = (m.n_nodes + 7) // 8
    flags = torch.zeros(max(iters, 1) * nbytes, dtype=torch.uint8, device="cuda:0") if want_flags else None
    rep = sl.smooth_mesh_device(*dev, iterations=iters, tol=tol, flags=flags, **opts)
    torch.cuda.synchronize()
    X = dev[0].cpu().numpy()
    F = sl.unpack_flags(flags.cpu().numpy().reshape(max(iters, 1), nbytes), m.n_nodes)[:iters] if want_flags else None
    return X, rep, F


def assert_parity(m, iters, tol=0.0, accept="ge", form="jacobi", threads=None, **opts):
    note("parity %s iters=%d tol=%g accept=%s form=%s %s" % (m.name, iters, tol, accept, form, opts))
    X, rep, F = run_gpu(m, iters, tol, accept=accept, form=form, **opts)
    ref = oracle.smooth(m, iters, tol=tol, accept_gt=(accept == "gt"), threads=threads or oracle.max_threads(),
                        form=form, precision=opts.get("precision", "f64"))
    assert rep.iterations_run == ref.iterations_run
    k = ref.iterations_run
    assert (F[:k] == (ref.flags == 1)).all(), "flags differ in sweeps %s" % np.flatnonzero(
        (F[:k] != (ref.flags == 1)).any(axis=1))
    assert (F[k:] == 0).all()
    err = float(np.abs(X - ref.coords).max())
    assert err <= COORD_TOL, err
    if k:
        assert rep.accepted_last == ref.accepted[-1]
        assert rep.accepted_total == int(ref.accepted.sum())
        assert rep.max_disp_sq_last == ref.disp[-1]
    return X, rep, ref, int(np.count_nonzero(X != ref.coords))


def test_config_small_grid_64():
    """64 x 64 Union-Jack grid, +-0.3h jitter, seed 1, 10 sweeps."""
    m = meshgen.make_grid(64, "unionjack", 0.3, 1)
    X, rep, ref, ndiff = assert_parity(m, 10)
    assert ndiff == 0                      # same IEEE sequence: bit-exact
    assert rep.setup_ms > 0 and rep.sweep_ms > 0


@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("reorder", ["none", "hilbert"])
@pytest.mark.parametrize("kernel,block", [("tile", 0), ("node", 0), ("node", 64), ("node", 128)])
def test_variants_are_bit_identical(layout, reorder, kernel, block):
    m = meshgen.make_grid(47, "random", 0.4, 5)       # 2025 free nodes: several tiles and a ragged tail
    X, rep, ref, ndiff = assert_parity(m, 8, layout=layout, reorder=reorder, block_size=block, kernel=kernel)
    assert ndiff == 0
    assert rep.kernel_used == sl.KERNELS[kernel]


def test_strict_accept_rule():
    m = meshgen.make_grid(40, "random", 0.35, 6)
    assert_parity(m, 6, accept="gt")
    d = meshgen.make_grid(33, "unionjack", 0.0, 0, h=1.0 / 32)      # exact fixed point: all ties
    X, rep, F = run_gpu(d, 3, accept="gt")
    assert (X == d.coords).all() and rep.accepted_total == 0
    X, rep, F = run_gpu(d, 3, accept="ge")
    assert (X == d.coords).all() and rep.accepted_total == 3 * d.n_interior


def _half_jittered_grid():
    """90 x 90 Union-Jack grid of spacing 0.1 (not a binary fraction: a
    centroid of the exact neighbours can miss the node by an ulp) whose left
    half is jittered, so that tiles hold clear decisions, exact ties and ties
    broken only in the last bits side by side."""
    m = meshgen.make_grid(90, "unionjack", 0.0, 0, h=0.1)
    rng = np.random.Generator(np.random.PCG64(5))
    left = (m.boundary == 0) & (m.coords[:, 0] < 4.0)
    m.coords[left] += rng.uniform(-0.03, 0.03, size=(int(left.sum()), 2))
    m.name = "grid90_unionjack_h0.1_half_jittered"
    return m


def _minima_gaps(m):
    """|min new quality - min old quality| per free node for the first sweep,
    from the oracle's quality in stored order and a row-order centroid."""
    X = m.coords
    gaps = []
    for i in np.flatnonzero(m.boundary == 0):
        row = m.nbr_idx[m.nbr_ptr[i]:m.nbr_ptr[i + 1]]
        sx = sy = 0.0
        for j in row:
            sx += X[j, 0]
            sy += X[j, 1]
        c = (sx / len(row), sy / len(row))
        qo = qn = math.inf
        for t in m.tri_idx[m.tri_ptr[i]:m.tri_ptr[i + 1]]:
            P = [tuple(X[v]) for v in m.tris[t]]
            qo = min(qo, oracle.quality(*P[0], *P[1], *P[2]))
            P = [c if v == i else P[k] for k, v in enumerate(m.tris[t])]
            qn = min(qn, oracle.quality(*P[0], *P[1], *P[2]))
        gaps.append(abs(qn - qo))
    return np.array(gaps)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("accept", ["ge", "gt"])
def test_near_ties(accept, precision):
    """Nodes whose old and new worst qualities tie exactly or differ in the
    last bits, beside nodes with clear decisions: the tile kernel decides the
    clear ones from its reciprocal-based first pass and sends tiles with close
    minima through its exact pass; every decision equals the oracle's."""
    m = _half_jittered_grid()
    if precision == "f64" and accept == "ge":
        g = _minima_gaps(m)
        assert (g == 0).sum() > 100 and ((g > 0) & (g < 2.0 ** -36)).sum() > 100 and (g > 1e-3).sum() > 1000
    X, rep, ref, nd = assert_parity(m, 12, accept=accept, precision=precision)
    assert nd == 0 and rep.kernel_used == sl.KERNELS["tile"]


@pytest.mark.parametrize("n", [3, 4, 5, 9, 17, 18, 33])
def test_ragged_sizes(n):
    assert_parity(meshgen.make_grid(n, "random", 0.4, 100 + n), 5)


@pytest.mark.parametrize("side", [128, 129, 130, 512, 513])
def test_scan_chunk_boundaries(side):
    """Sizes where setup's scans (node flags, the node path's rows and fans
    over free nodes, the adjacency builder's counts) end at or one past a
    chunk of the one-launch scan (16,384 values: 128^2 nodes, 130^2 with
    128^2 free), at its limit (262,144 = 512^2) and above it (513^2, the
    three-pass scan): both kernels equal the oracle, and the device
    adjacency equals the generators' builder."""
    m = meshgen.make_grid(side, "random", 0.4, 700 + side)
    X, rep, ref, nd = assert_parity(m, 3)
    assert nd == 0
    Xn, rn, _ = run_gpu(m, 3, kernel="node")
    assert rn.kernel_used == sl.KERNELS["node"] and (Xn == X).all()
    got = sl.build_adjacency(m.n_nodes, m.tris)
    want = (m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.boundary)
    assert all(np.array_equal(np.asarray(g), np.asarray(w)) for g, w in zip(got, want))


def test_annulus_and_permuted():
    assert_parity(meshgen.make_annulus(40, 64, seed=4), 12)
    assert_parity(meshgen.permute_mesh(meshgen.make_grid(50, "random", 0.4, 7), 8), 12)


def test_config_1024_permuted_full():
    """1024 x 1024, random diagonals, +-0.4h, random node permutation, 100
    sweeps; AoS and SoA, reorder on and off: every flag of every sweep."""
    m = meshgen.permute_mesh(meshgen.make_grid(1024, "random", 0.4, 2), 2)
    ref = oracle.smooth(m, 100, threads=oracle.max_threads())
    rf = ref.flags == 1
    for layout, reorder, kernel in (("aos", "hilbert", "tile"), ("soa", "hilbert", "tile"),
                                    ("aos", "none", "tile"), ("aos", "hilbert", "node"), ("soa", "none", "node")):
        note("1024^2 permuted, 100 sweeps, %s %s %s" % (layout, reorder, kernel))
        X, rep, F = run_gpu(m, 100, layout=layout, reorder=reorder, kernel=kernel)
        assert rep.iterations_run == 100
        assert (F == rf).all()
        assert float(np.abs(X - ref.coords).max()) <= COORD_TOL
        assert (X == ref.coords).all()


def _mesh_4096(kind):
    if kind == "grid":
        return meshgen.make_grid(4096, "random", 0.4, 3)
    return meshgen.make_annulus(4096, 4096, seed=4)


@pytest.mark.parametrize("kind", ["grid", "annulus"])
def test_config_4096_full_100_sweeps(kind):
    """Full 16.8M-node size, in the launch configuration the benchmark times
    (AoS, Hilbert, automatic shape), for all 100 timed sweeps: every flag of
    every sweep, the per-sweep accept counts, and all coordinates.  The late
    sweeps are the near-tie regime, where a candidate differs from the
    position by an ulp and the accept decision turns on the last bit of the
    qualities."""
    m = _mesh_4096(kind)
    note("4096^2 %s generated" % kind)
    X, rep, F = run_gpu(m, 100)
    assert rep.kernel_used == sl.KERNELS["tile"]
    note("4096^2 %s: GPU done, oracle running" % kind)
    ref = oracle.smooth(m, 100, threads=oracle.max_threads())
    assert rep.iterations_run == ref.iterations_run == 100
    assert rep.accepted_total == int(ref.accepted.sum())
    bad = [k for k in range(100) if not (F[k] == (ref.flags[k] == 1)).all()]
    assert not bad, "flags differ in sweeps %s" % bad[:10]
    assert (F.sum(axis=1) == ref.accepted).all()
    assert float(np.abs(X - ref.coords).max()) <= COORD_TOL
    assert (X == ref.coords).all()


@pytest.mark.parametrize("kind", ["grid", "annulus"])
def test_config_4096_to_tolerance_1e9(kind):
    """The 16.8M-node meshes run until the largest displacement of a sweep
    is below 1e-9 (cap 100,000): the same sweep count as the oracle and the
    same coordinates, bit for bit."""
    m = _mesh_4096(kind)
    note("4096^2 %s generated" % kind)
    X, rep, _ = run_gpu(m, 100000, 1e-9, want_flags=False)
    note("4096^2 %s: GPU stopped after %d sweeps, oracle running" % (kind, rep.iterations_run))
    ref = oracle.smooth(m, 100000, tol=1e-9, threads=oracle.max_threads(), want_flags=False)
    assert rep.iterations_run == ref.iterations_run < 100000
    assert rep.max_disp_sq_last == ref.disp[-1] < 1e-18
    assert rep.accepted_total == int(ref.accepted.sum())
    assert (X == ref.coords).all()


def test_tolerance_stop():
    m = meshgen.make_grid(30, "random", 0.4, 9)
    ref = oracle.smooth(m, 200, tol=0.0)
    # a tolerance the run reaches part-way through
    tol = math.sqrt(ref.disp[40]) * 1.0000001
    X, rep, ref2, _ = assert_parity(m, 200, tol=tol)
    assert 0 < rep.iterations_run < 200


@pytest.mark.parametrize("iters,tol_at", [(64, None), (77, None), (200, 41), (1000, 5)])
def test_sweep_loop_in_graph_chunks(iters, tol_at):
    """Without flag output the sweep loop runs as replays of a captured
    chunk: whole chunks, a shorter tail, and a tolerance reached inside a
    chunk (the host stops launching, the rest of the chunk returns at once)."""
    m = meshgen.make_grid(40, "random", 0.4, 77)
    tol = 0.0
    if tol_at is not None:
        tol = math.sqrt(oracle.smooth(m, tol_at + 1).disp[tol_at]) * 1.0000001
    note("chunks iters=%d tol=%g" % (iters, tol))
    ref = oracle.smooth(m, iters, tol=tol)
    X, rep, _ = run_gpu(m, iters, tol, want_flags=False)
    assert rep.iterations_run == ref.iterations_run
    if tol_at is not None:
        assert rep.iterations_run < iters
    assert (X == ref.coords).all()
    assert rep.accepted_total == int(ref.accepted.sum())


@pytest.mark.parametrize("tile_nodes,wpc", [(256, 1), (256, 3), (512, 2), (512, 8)])
def test_tile_shapes_are_bit_identical(tile_nodes, wpc):
    m = meshgen.make_grid(300, "random", 0.4, 31)
    X, rep, ref, ndiff = assert_parity(m, 6, kernel="tile", tile_nodes=tile_nodes, tile_wg_per_cu=wpc)
    assert ndiff == 0 and rep.kernel_used == 2 and rep.tile_nodes == tile_nodes


def test_autotune_then_automatic_shape():
    ms = [meshgen.make_grid(n, "random", 0.35, 500 + n) for n in (30, 64, 120, 250)]
    try:
        t = sl.autotune(ms)
        note("autotune %s" % t.as_dict())
        assert t.tile_nodes in (256, 512) and 1 <= t.tile_wg_per_cu <= 8 and t.block_size == 0
        assert t.n_candidates >= 2 and t.sampled_meshes == 4
        assert t.sampled_free_nodes == sum(m.n_interior for m in ms)
        cands = list(t.candidates[: t.n_candidates])
        best = min(c.ns_per_update for c in cands)
        assert all(c.ns_per_update > 0 for c in cands)
        chosen = [c for c in cands if c.tile_nodes == t.tile_nodes and c.wg_per_cu == t.tile_wg_per_cu]
        # the fastest shape, or the default one (512 nodes, 4 per CU) within 1% of it
        assert len(chosen) == 1 and (chosen[0].ns_per_update == best or (
            (t.tile_nodes, t.tile_wg_per_cu) == (512, 4) and chosen[0].ns_per_update <= best * 1.01))
        X, rep, ref, ndiff = assert_parity(ms[3], 5)
        assert ndiff == 0 and rep.tile_nodes == t.tile_nodes
        outs, reps, br = sl.batch_smooth(ms, 5)
        for m, X, r in zip(ms, outs, reps):
            assert r.tile_nodes == t.tile_nodes
            assert (X == oracle.smooth(m, 5).coords).all()
        tc = sl.autotune(ms, form="colored")
        note("autotune colored %s" % tc.as_dict())
        assert tc.block_size in (64, 128, 256) and tc.tile_nodes == 0 and tc.n_candidates == 3
        X, rep, ref, ndiff = assert_parity(ms[2], 4, form="colored")
        assert ndiff == 0
        # a coloured tuning keeps the tile shape
        X, rep, ref, ndiff = assert_parity(ms[1], 3)
        assert rep.tile_nodes == t.tile_nodes
    finally:
        sl.autotune_reset()


def test_zero_iterations_and_all_fixed():
    m = meshgen.make_grid(16, "random", 0.4, 10)
    X, rep, F = run_gpu(m, 0)
    assert (X == m.coords).all() and rep.iterations_run == 0
    b = m.copy()
    b.boundary[:] = 1
    X, rep, F = run_gpu(b, 4)
    assert (X == m.coords).all() and rep.accepted_total == 0 and (F == 0).all()
    t = meshgen.star_mesh((0.1, 0.2), [(1, 0), (0, 1), (-1, 0)])
    assert_parity(t, 3)


def _ring_star(k, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ang = np.sort(rng.uniform(0, 2 * np.pi, k))
    ring = np.stack([np.cos(ang), np.sin(ang)], 1) * rng.uniform(0.8, 1.2, (k, 1))
    return meshgen.star_mesh(rng.uniform(-0.2, 0.2, 2), ring)


@pytest.mark.parametrize("k", [3, 8, 9, 16, 17, 32, 33, 100, 127])
def test_valence_classes(k):
    X, rep, ref, _ = assert_parity(_ring_star(k, k), 3)
    assert rep.kernel_used == sl.KERNELS["tile"]
    assert_parity(_ring_star(k, k), 3, kernel="node")


def _many_stars(count, k, seed):
    """count disjoint ring stars of valence k in one mesh: the free nodes are
    the centres, each with k neighbour entries."""
    coords, tris, off = [], [], 0
    for s in range(count):
        st = _ring_star(k, seed + s)
        coords.append(st.coords + np.array([3.0 * (s % 40), 3.0 * (s // 40)]))
        tris.append(st.tris + off)
        off += st.n_nodes
    coords = np.concatenate(coords)
    tris = np.concatenate(tris)
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = meshgen.build_adjacency(coords.shape[0], tris)
    return meshgen.Mesh(coords, tris, nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd, "stars%dx%d" % (count, k))


def test_tiles_too_dense_fall_back_to_the_node_kernel():
    m = _many_stars(600, 20, 5)            # 512 centres x 20 entries > 16 per node on average
    X, rep, ref, nd = assert_parity(m, 3)
    assert nd == 0 and rep.kernel_used == sl.KERNELS["node"]
    m = _many_stars(600, 7, 5)            # 7 distinct outside neighbours per node > 4: node path
    X, rep, ref, nd = assert_parity(m, 3)
    assert nd == 0 and rep.kernel_used == sl.KERNELS["node"]
    m = _many_stars(600, 3, 5)            # 3 per node: tiles and their halos fit
    X, rep, ref, nd = assert_parity(m, 3)
    assert nd == 0 and rep.kernel_used == sl.KERNELS["tile"]


def test_tile_path_at_every_tile_boundary():
    """Free-node counts around multiples of the tile size, both kernels."""
    for n in (24, 25, 26, 34, 35, 47, 48, 49):
        m = meshgen.make_grid(n, "random", 0.4, 200 + n)
        X, rep, ref, nd = assert_parity(m, 4)
        assert nd == 0 and rep.kernel_used == sl.KERNELS["tile"]


def test_valence_limit_rejected():
    m = _ring_star(128, 1)
    with pytest.raises(sl.SmartlapError) as e:
        run_gpu(m, 1)
    assert e.value.status == sl.SL_ETOPO


def test_input_errors():
    m = meshgen.make_grid(8, "random", 0.3, 11)

    def call(mm):
        """Raw C call on the caller's own coordinate buffer."""
        arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (mm.nbr_ptr, mm.nbr_idx, mm.tri_ptr, mm.tri_idx)]
        tr = np.ascontiguousarray(mm.tris, dtype=np.int32)
        b = np.ascontiguousarray(mm.boundary, dtype=np.uint8)
        rep = sl.Report()
        st = sl.lib().smooth_mesh(mm.coords.ctypes.data, mm.n_nodes, arrs[0].ctypes.data, arrs[1].ctypes.data,
                                  arrs[2].ctypes.data, arrs[3].ctypes.data, tr.ctypes.data, mm.n_tris,
                                  b.ctypes.data, 2, 0.0, None, ctypes.byref(rep))
        if st != sl.SL_OK:
            raise sl.SmartlapError(st, sl.lib().sl_last_error().decode())
        return rep

    cases = []
    a = m.copy(); a.nbr_idx[5] = m.n_nodes + 3; cases.append((a, sl.SL_EINVAL))
    a = m.copy(); a.coords[20, 1] = np.nan; cases.append((a, sl.SL_EINVAL))
    a = m.copy(); a.coords[21, 0] = -np.inf; cases.append((a, sl.SL_EINVAL))
    a = m.copy(); a.coords[22, 0] = 2.0 ** 500; cases.append((a, sl.SL_EINVAL))
    a = m.copy(); a.tri_idx[7] = -1; cases.append((a, sl.SL_EINVAL))
    a = m.copy(); a.nbr_ptr[10] = a.nbr_ptr[11] + 1; cases.append((a, sl.SL_EINVAL))
    a = m.copy(); i = 20; a.nbr_idx[a.nbr_ptr[i]] = i; cases.append((a, sl.SL_ETOPO))
    a = m.copy(); a.tris[3, 1] = a.tris[3, 0]; cases.append((a, sl.SL_ETOPO))
    a = m.copy(); i = 20; a.tri_idx[a.tri_ptr[i]] = a.tri_idx[a.tri_ptr[0]]; cases.append((a, sl.SL_ETOPO))
    for bad, want in cases:
        before = bad.coords.copy()
        with pytest.raises(sl.SmartlapError) as e:
            call(bad)
        assert e.value.status == want, str(e.value)
        assert np.array_equal(bad.coords, before, equal_nan=True)      # untouched on error
    before = m.coords.copy()
    rep = call(m)
    assert rep.iterations_run == 2 and not (m.coords == before).all()


@pytest.mark.parametrize("exp2", [-1040, -1020, -1016, -520, -40, 40, 498])
def test_extreme_coordinate_scales(exp2):
    """The same mesh scaled by a power of two (exact): at 2^-520 squared
    lengths are subnormal, near 2^498 they approach the largest doubles.  At
    2^-1016 the centroid sums stay above the bound of the kernel's
    division-by-count step, at 2^-1020 they fall below it, and at 2^-1040 the
    coordinates themselves are subnormal (every quality is 0).  The device
    follows the oracle at every scale (subnormals are kept by both)."""
    m = meshgen.make_grid(45, "random", 0.4, 88)
    m.coords = m.coords * (2.0 ** exp2) + (2.0 ** exp2) * 0.25
    m.name = "grid45_scaled_2^%d" % exp2
    X, rep, ref, ndiff = assert_parity(m, 6)
    assert ndiff == 0


@pytest.mark.parametrize("n", [1000, 10000, 100000])
def test_delaunay_random_points(n):
    """The paper's kind of mesh: Delaunay triangulations of uniformly random
    points (valence up to about 17), Form A on both layouts and Form B."""
    m = meshgen.make_delaunay(n, 11)
    X, rep, ref, nd = assert_parity(m, 20)
    assert nd == 0 and rep.kernel_used == sl.KERNELS["tile"]
    if n <= 10000:
        X, rep, ref, nd = assert_parity(m, 20, layout="soa")
        assert nd == 0
        X, rep, ref, nd = assert_parity(m, 10, form="colored")
        assert nd == 0


def test_coincident_vertices():
    """Triangles whose three vertices coincide (S == 0, quality 0) and edges
    of zero length: the device follows the oracle."""
    m = meshgen.make_grid(20, "random", 0.3, 41)
    tris = m.tris
    free = m.boundary == 0
    picked = 0
    for t in range(len(tris)):
        a, b, c = tris[t]
        if free[a] and free[b] and free[c]:
            m.coords[b] = m.coords[a]
            m.coords[c] = m.coords[a]
            picked += 1
            if picked == 3:
                break
    m.coords[tris[200][1]] = m.coords[tris[200][0]]      # one zero-length edge
    m.name = "grid20_coincident"
    X, rep, ref, ndiff = assert_parity(m, 8)
    assert ndiff == 0


def test_host_and_device_entry_points_agree():
    m = meshgen.make_grid(60, "random", 0.4, 12)
    Xh, rh, Fh = sl.smooth_mesh(m.coords, m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary, 7,
                                want_flags=True)
    Xd, rd, Fd = run_gpu(m, 7)
    assert (Xh == Xd).all()
    assert (sl.unpack_flags(Fh, m.n_nodes) == Fd).all()
    assert rh.accepted_total == rd.accepted_total


def test_device_entry_point_refuses_misaligned_coords():
    import torch
    m = meshgen.make_grid(12, "random", 0.4, 12)
    dev = list(sl.to_device(m, "cuda:0"))
    buf = torch.zeros(2 * m.n_nodes + 1, dtype=torch.float64, device="cuda:0")
    X = buf[1:].view(m.n_nodes, 2)          # contiguous, 8 bytes past a 16-byte boundary
    X.copy_(dev[0])
    assert X.data_ptr() % 16 == 8
    with pytest.raises(sl.SmartlapError) as e:
        sl.smooth_mesh_device(X, *dev[1:], iterations=3)
    assert "aligned" in str(e.value)
    assert torch.equal(X.cpu(), dev[0].cpu())    # untouched


def test_resume_and_repeat_are_bit_exact():
    m = meshgen.make_grid(64, "random", 0.4, 13)
    X12, _, _ = run_gpu(m, 12)
    X12b, _, _ = run_gpu(m, 12)
    m6 = m.copy()
    m6.coords, _, _ = run_gpu(m, 6)
    X66, _, _ = run_gpu(m6, 6)
    assert (X12 == X12b).all() and (X12 == X66).all()


@pytest.mark.parametrize("kernel", ["auto", "node"])
def test_colored_form_parity_and_invariants(kernel):
    m = meshgen.make_grid(48, "random", 0.4, 14)
    X, rep, ref, ndiff = assert_parity(m, 8, form="colored", kernel=kernel)
    # a mesh this small runs Form B on the resident kernel unless told otherwise
    assert rep.kernel_used == sl.KERNELS["resident" if kernel == "auto" else "node"]
    col, nc = oracle.colors(m)
    assert rep.n_colors == nc
    b = m.boundary.astype(bool)
    assert (X[b] == m.coords[b]).all() and np.isfinite(X).all()
    for layout in ("aos", "soa"):
        for reorder in ("none", "hilbert"):
            X2, _, _ = run_gpu(m, 8, form="colored", layout=layout, reorder=reorder, kernel=kernel)
            assert (X2 == X).all()
    # mesh-wide worst quality never drops over a coloured sweep
    prev = min(oracle.quality(*m.coords[a], *m.coords[c], *m.coords[d]) for a, c, d in m.tris)
    mm = m.copy()
    for _ in range(4):
        mm.coords, _, _ = run_gpu(mm, 1, form="colored")
        cur = min(oracle.quality(*mm.coords[a], *mm.coords[c], *mm.coords[d]) for a, c, d in m.tris)
        assert cur >= prev
        prev = cur


def test_batch_equals_single_and_oracle():
    """Meshes of uneven size (some below one tile, one node-path star, a
    permuted mesh) in one batch: each result equals its own single-mesh run
    and the oracle."""
    ms = [meshgen.make_grid(n, "random", 0.35, 10000 + n) for n in (24, 31, 40, 57, 90)]
    ms.append(meshgen.permute_mesh(meshgen.make_grid(33, "random", 0.4, 7), 3))
    ms.append(_many_stars(600, 20, 5))                # tiles too dense: node path
    ms.append(meshgen.make_annulus(12, 40, seed=9))
    outs, reps, br = sl.batch_smooth(ms, 9)
    assert br.graph_used == 1 and br.meshes_on_tile_path == len(ms) - 1 and br.meshes_resident == 0
    for m, X, rep in zip(ms, outs, reps):
        ref = oracle.smooth(m, 9)
        assert rep.iterations_run == 9 and rep.accepted_total == int(ref.accepted.sum())
        assert (X == ref.coords).all(), m.name
        Xs, rs, _ = run_gpu(m, 9)
        assert (X == Xs).all()


def test_batch_tolerance_and_forms():
    ms = [meshgen.make_grid(n, "random", 0.4, 300 + n) for n in (20, 28, 45)]
    ref = [oracle.smooth(m, 400, tol=3e-4) for m in ms]
    for kernel in ("auto", "resident"):
        outs, reps, br = sl.batch_smooth(ms, 400, tol=3e-4, kernel=kernel)
        assert br.meshes_resident == (len(ms) if kernel == "resident" else 0)
        for m, X, rep, r in zip(ms, outs, reps, ref):
            assert rep.iterations_run == r.iterations_run < 400
            assert rep.accepted_total == int(r.accepted.sum())
            assert (X == r.coords).all()
    for kernel in ("auto", "resident", "node"):
        outs, reps, br = sl.batch_smooth(ms, 5, form="colored", kernel=kernel)
        assert br.meshes_resident == (0 if kernel == "node" else len(ms))
        for m, X in zip(ms, outs):
            assert (X == oracle.smooth(m, 5, form="colored").coords).all()
    outs, reps, br = sl.batch_smooth(ms, 6, accept="gt", layout="soa")
    for m, X in zip(ms, outs):
        assert (X == oracle.smooth(m, 6, accept_gt=True).coords).all()


RESIDENT_MESHES = {
    "grid24": lambda: meshgen.make_grid(24, "random", 0.4, 601),               # one node per work-item
    "grid45_unionjack": lambda: meshgen.make_grid(45, "unionjack", 0.3, 602),  # 2025 nodes: two per work-item
    "annulus12x40": lambda: meshgen.make_annulus(12, 40, seed=603),
    "grid33_permuted": lambda: meshgen.permute_mesh(meshgen.make_grid(33, "random", 0.4, 604), 5),
    "delaunay1000": lambda: meshgen.make_delaunay(1000, 11),
    "star17": lambda: _ring_star(17, 17),
}


@pytest.mark.parametrize("name", sorted(RESIDENT_MESHES))
@pytest.mark.parametrize("layout,accept,form", [("aos", "ge", "jacobi"), ("soa", "gt", "jacobi"),
                                                ("aos", "ge", "colored"), ("soa", "gt", "colored")])
def test_resident_kernel_parity(name, layout, accept, form):
    """Every sweep of a small mesh in one launch, with the mesh in LDS (Form
    A: two buffers; Form B: one, class by class): the flags of every sweep,
    the coordinates and the counts equal the oracle's, and the coordinates
    equal the other kernels' (tile for Form A, node for Form B)."""
    m = RESIDENT_MESHES[name]()
    X, rep, ref, nd = assert_parity(m, 12, accept=accept, layout=layout, form=form, kernel="resident")
    assert nd == 0 and rep.kernel_used == sl.KERNELS["resident"] and rep.tile_nodes == 0
    other = "tile" if form == "jacobi" else "node"
    Xt, rt, _ = run_gpu(m, 12, accept=accept, layout=layout, form=form, kernel=other)
    assert rt.kernel_used == sl.KERNELS[other] and (X == Xt).all()
    if form == "colored":
        assert rep.n_colors == rt.n_colors >= 1


def test_resident_tolerance_zero_sweeps_and_fixed_nodes():
    m = meshgen.make_grid(30, "random", 0.4, 605)
    X, rep, ref, nd = assert_parity(m, 400, tol=3e-4, kernel="resident")
    assert nd == 0 and rep.iterations_run < 400
    X, rep, F = run_gpu(m, 0, kernel="resident")
    assert (X == m.coords).all() and rep.iterations_run == 0 and rep.accepted_total == 0
    b = m.copy()
    b.boundary[:] = 1
    X, rep, F = run_gpu(b, 4, kernel="resident")
    assert (X == m.coords).all() and rep.iterations_run == 4 and rep.accepted_total == 0 and (F == 0).all()
    X, rep, F = run_gpu(b, 50, tol=1e-3, kernel="resident")
    assert rep.iterations_run == 1 and rep.max_disp_sq_last == 0.0


@pytest.mark.parametrize("exp2", [-1040, -1020, -520, 498])
def test_resident_extreme_coordinate_scales(exp2):
    m = meshgen.make_grid(30, "random", 0.4, 606)
    m.coords = m.coords * (2.0 ** exp2) + (2.0 ** exp2) * 0.25
    m.name = "grid30_scaled_2^%d" % exp2
    X, rep, ref, nd = assert_parity(m, 5, kernel="resident")
    assert nd == 0


def test_resident_limits():
    big = meshgen.make_grid(64, "random", 0.4, 607)          # 4096 nodes: both buffers alone take 128 KB
    with pytest.raises(sl.SmartlapError) as e:
        run_gpu(big, 2, kernel="resident")
    assert e.value.status == sl.SL_EINVAL and "resident" in str(e.value)
    small = meshgen.make_grid(20, "random", 0.4, 608)
    for opts in ({"precision": "f32"}, {"precision": "f32", "form": "colored"}):
        with pytest.raises(sl.SmartlapError) as e:
            run_gpu(small, 2, kernel="resident", **opts)
        assert e.value.status == sl.SL_EINVAL
    with pytest.raises(sl.SmartlapError) as e:
        sl.Server(kernel="resident")
    assert e.value.status == sl.SL_EINVAL
    # a batch member too large for it is refused by name
    with pytest.raises(sl.SmartlapError) as e:
        sl.batch_smooth([small, big], 2, kernel="resident")
    assert e.value.status == sl.SL_EINVAL and "mesh 1" in str(e.value)


def test_batch_of_resident_meshes_only():
    """A batch whose meshes all run on the resident kernel: no sweep graph,
    one launch."""
    ms = [meshgen.make_grid(n, "random", 0.35, 620 + n) for n in (5, 12, 24, 31, 45)]
    outs, reps, br = sl.batch_smooth(ms, 11, kernel="resident")
    assert br.meshes_resident == len(ms) and br.graph_used == 0 and br.tiles == 0
    assert all(r.kernel_used == sl.KERNELS["resident"] for r in reps)
    for m, X, rep in zip(ms, outs, reps):
        ref = oracle.smooth(m, 11)
        assert rep.iterations_run == 11 and rep.accepted_total == int(ref.accepted.sum())
        assert rep.accepted_last == ref.accepted[-1] and rep.max_disp_sq_last == ref.disp[-1]
        assert (X == ref.coords).all(), m.name


def test_batch_of_one_with_tolerance():
    m = meshgen.make_grid(50, "random", 0.4, 71)
    ref = oracle.smooth(m, 300, tol=3e-4)
    outs, reps, br = sl.batch_smooth([m], 300, tol=3e-4)
    assert reps[0].iterations_run == ref.iterations_run < 300
    assert (outs[0] == ref.coords).all()


def test_batch_bad_member_then_batches_in_both_precisions():
    """The meshes of a batch share one device block: a member that fails
    validation is named and fails the call, and the batches after it, in
    double and single precision, still give the oracle's results."""
    ms = [meshgen.make_grid(n, "random", 0.4, 640 + n) for n in (18, 26, 37)]
    bad = ms[1].copy()
    bad.nbr_idx[5] = bad.n_nodes + 7                 # a neighbour id out of range
    with pytest.raises(sl.SmartlapError) as e:
        sl.batch_smooth([ms[0], ms[2], bad], 4)
    assert e.value.status == sl.SL_EINVAL and "mesh 2" in str(e.value)
    outs, reps, br = sl.batch_smooth(ms, 7)
    for m, X, rep in zip(ms, outs, reps):
        ref = oracle.smooth(m, 7)
        assert rep.accepted_total == int(ref.accepted.sum()) and (X == ref.coords).all()
    outs, reps, br = sl.batch_smooth(ms[::-1], 7, precision="f32")
    for m, X, rep in zip(ms[::-1], outs, reps):
        ref = oracle.smooth(m, 7, precision="f32")
        assert rep.accepted_total == int(ref.accepted.sum()) and (X == ref.coords).all()


def test_server_mix_equals_single_and_oracle():
    """Requests of different sizes, caps and tolerances, submitted at once
    and while others run: each result equals its oracle run (and therefore
    its own single-mesh run)."""
    import time
    ms = [meshgen.make_grid(n, "random", 0.4, 500 + n) for n in (20, 33, 64, 120, 257)]
    ms.append(meshgen.permute_mesh(meshgen.make_grid(40, "random", 0.4, 8), 9))
    ms.append(_ring_star(24, 3))                                   # node path
    jobs = [(6, 0.0), (11, 0.0), (25, 0.0), (40, 0.0), (9, 0.0), (300, 2e-4), (4, 0.0)]
    with sl.Server(sweeps_per_step=3) as srv:
        ids = []
        for k, (m, (it, tol)) in enumerate(zip(ms, jobs)):
            ids.append(srv.submit(m, it, tol))
            if k == 3:
                time.sleep(0.05)                                  # later arrivals join running steps
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st.completed == len(ms) and st.failed == 0
    for m, (it, tol), r in zip(ms, jobs, res):
        assert r.status == sl.SL_OK, r.message
        ref = oracle.smooth(m, it, tol=tol)
        assert r.report.iterations_run == ref.iterations_run
        assert (r.coords == ref.coords).all(), m.name
        t = r.times
        assert t.submitted_s <= t.admitted_s <= t.started_s <= t.done_s


@pytest.mark.parametrize("kernel,kinds,resident", [("auto", ("node", "node", "resident", "node"), 1),
                                                   ("tile", ("tile", "tile", "tile", "node"), 0)])
def test_batch_form_b_on_class_tiles_resident_and_node(kernel, kinds, resident):
    """A Form B batch: automatically, the small mesh on the resident kernel
    and the others on the node kernel; asking for tiles, meshes on
    colour-class tiles and a mesh too dense for them on the node kernel, in
    one call; every one equals the oracle's coloured sweeps."""
    ms = [meshgen.make_grid(70, "random", 0.4, 41), meshgen.make_delaunay(5000, 42),
          meshgen.make_grid(20, "random", 0.4, 43), _many_stars(300, 20, 44)]
    outs, reps, br = sl.batch_smooth(ms, 9, form="colored", kernel=kernel)
    assert [r.kernel_used for r in reps] == [sl.KERNELS[k] for k in kinds]
    assert br.meshes_resident == resident
    for m, X, rep in zip(ms, outs, reps):
        ref = oracle.smooth(m, 9, form="colored")
        assert (X == ref.coords).all(), m.name
        assert rep.accepted_total == int(ref.accepted.sum()), m.name


@pytest.mark.parametrize("kernel", ["auto", "tile"])
def test_server_form_b_mix(kernel):
    """Form B requests sharing steps, on the node kernel (automatic) or on
    colour-class tiles of both automatic sizes (asked for): each result and
    accepted count equals the oracle's coloured sweeps."""
    ms = [meshgen.make_grid(n, "random", 0.4, 900 + n) for n in (30, 90, 200)]
    ms.append(meshgen.make_delaunay(3000, 91))
    ms.append(_ring_star(24, 5))                                   # one node of valence 24
    jobs = [(7, 0.0), (12, 0.0), (20, 0.0), (400, 1e-6), (5, 0.0)]
    with sl.Server(form="colored", sweeps_per_step=4, kernel=kernel) as srv:
        ids = [srv.submit(m, it, tol) for m, (it, tol) in zip(ms, jobs)]
        res = [srv.wait(i) for i in ids]
    for m, (it, tol), r in zip(ms, jobs, res):
        assert r.status == sl.SL_OK, r.message
        ref = oracle.smooth(m, it, tol=tol, form="colored")
        assert r.report.iterations_run == ref.iterations_run, m.name
        assert (r.coords == ref.coords).all(), m.name
        assert r.report.accepted_total == int(ref.accepted.sum()), m.name
    want = "tile" if kernel == "tile" else "node"
    assert [r.report.kernel_used for r in res] == [sl.KERNELS[want]] * 5


def test_server_cancel_deadline_budget_and_bad_input():
    big = meshgen.make_grid(300, "random", 0.4, 1)
    ok = meshgen.make_grid(30, "random", 0.4, 2)
    bad = ok.copy()
    bad.nbr_idx[3] = ok.n_nodes + 5
    with sl.Server(sweeps_per_step=2, hbm_budget_bytes=64 << 20) as srv:
        a = srv.submit(big, 100000)
        b = srv.submit(ok, 7)
        c = srv.submit(bad, 3)
        d = srv.submit(big, 100000, deadline_s=0.05)
        huge = meshgen.make_grid(1500, "random", 0.4, 3)            # estimated footprint over 64 MiB
        e = srv.submit(huge, 2)
        srv.cancel(a)
        ra, rb, rc, rd, re = (srv.wait(x) for x in (a, b, c, d, e))
    assert ra.status == sl.SL_ECANCELED
    assert rb.status == sl.SL_OK and (rb.coords == oracle.smooth(ok, 7).coords).all()
    assert rc.status == sl.SL_EINVAL
    assert rd.status == sl.SL_ETIMEOUT
    assert re.status == sl.SL_ENOMEM


# ------------------------------------------------------ single precision ----

@pytest.mark.parametrize("make,iters", [
    (lambda: meshgen.make_grid(64, "unionjack", 0.3, 1), 10),
    (lambda: meshgen.make_grid(300, "random", 0.4, 31), 12),
    (lambda: meshgen.make_annulus(40, 90, seed=3), 8),
    (lambda: meshgen.make_delaunay(10000, 11), 15),
])
@pytest.mark.parametrize("layout", ["aos", "soa"])
def test_f32_parity(make, iters, layout):
    """Single precision (the paper's): the same float operations on both
    sides, so flags and coordinates are bit-exact."""
    m = make()
    X, rep, ref, nd = assert_parity(m, iters, precision="f32", layout=layout)
    assert nd == 0 and rep.kernel_used == sl.KERNELS["tile"]
    assert (X.astype(np.float32).astype(np.float64) == X).all()


@pytest.mark.parametrize("tile_nodes,wpc,accept", [(256, 3, "ge"), (512, 2, "gt"), (512, 8, "ge")])
def test_f32_shapes_and_rules(tile_nodes, wpc, accept):
    m = meshgen.permute_mesh(meshgen.make_grid(200, "random", 0.4, 8), 4)
    X, rep, ref, nd = assert_parity(m, 9, precision="f32", accept=accept, tile_nodes=tile_nodes,
                                    tile_wg_per_cu=wpc)
    assert nd == 0 and rep.tile_nodes == tile_nodes


def test_f32_full_1024_and_tolerance():
    m = meshgen.permute_mesh(meshgen.make_grid(1024, "random", 0.4, 2), 2)
    X, rep, ref, nd = assert_parity(m, 30, precision="f32")
    assert nd == 0
    small = meshgen.make_grid(30, "random", 0.4, 9)
    ref = oracle.smooth(small, 300, precision="f32")
    moving = np.flatnonzero(ref.disp > 0)           # in float the mesh reaches an exact fixed point
    tol = math.sqrt(ref.disp[moving[len(moving) // 2]]) * 1.0000001
    X, rep, ref2, nd = assert_parity(small, 300, tol=tol, precision="f32")
    assert nd == 0 and rep.iterations_run < 300


@pytest.mark.parametrize("exp2", [-140, -122, -117, 60])
def test_f32_extreme_coordinate_scales(exp2):
    """Single precision at scales where float centroid sums fall below the
    division-by-count step's bound (2^-122), stay above it (2^-117), or the
    float coordinates are subnormal (2^-140)."""
    m = meshgen.make_grid(45, "random", 0.4, 89)
    m.coords = m.coords * (2.0 ** exp2) + (2.0 ** exp2) * 0.25
    m.name = "grid45_f32_scaled_2^%d" % exp2
    X, rep, ref, nd = assert_parity(m, 6, precision="f32")
    assert nd == 0


def test_f32_refused_outside_the_tile_path():
    m = meshgen.make_grid(20, "random", 0.4, 3)
    for opts in ({"form": "colored"}, {"kernel": "node"}):
        with pytest.raises(sl.SmartlapError) as e:
            run_gpu(m, 2, precision="f32", **opts)
        assert e.value.status == sl.SL_EINVAL
    with pytest.raises(sl.SmartlapError) as e:
        run_gpu(_many_stars(600, 20, 5), 2, precision="f32")    # tiles too dense: node path needed
    assert e.value.status == sl.SL_EINVAL and "single precision" in str(e.value)


def test_f32_batch_and_server():
    ms = [meshgen.make_grid(n, "random", 0.35, 700 + n) for n in (24, 57, 130)]
    outs, reps, br = sl.batch_smooth(ms, 7, precision="f32")
    for m, X in zip(ms, outs):
        assert (X == oracle.smooth(m, 7, precision="f32").coords).all()
    with sl.Server(precision="f32") as S:
        ids = [S.submit(m, 5 + k) for k, m in enumerate(ms)]
        for k, (m, rid) in enumerate(zip(ms, ids)):
            r = S.wait(rid)
            assert r.status == sl.SL_OK
            assert (r.coords == oracle.smooth(m, 5 + k, precision="f32").coords).all()


@pytest.mark.parametrize("exp2", [62, 130])
def test_f32_rejects_coordinates_beyond_2_61(exp2):
    """In single precision a coordinate of magnitude 2^61 or more could make
    a squared length or their sum overflow float; such input is refused, and
    the same mesh in double precision is accepted."""
    m = meshgen.make_grid(20, "random", 0.4, 90)
    m.coords = m.coords.copy()
    m.coords[m.n_nodes // 2] = (2.0 ** exp2, 0.5)
    with pytest.raises(sl.SmartlapError) as e:
        run_gpu(m, 2, precision="f32")
    assert e.value.status == sl.SL_EINVAL and "2^61" in str(e.value)
    X, rep, F = run_gpu(m, 2)
    assert rep.iterations_run == 2


def _trim_incidence(m, node, tri):
    """Copy of m with triangle `tri` removed from node `node`'s incidence row."""
    import copy
    b, e = int(m.tri_ptr[node]), int(m.tri_ptr[node + 1])
    row = m.tri_idx[b:e].tolist()
    k = row.index(tri)
    t = copy.copy(m)
    t.tri_idx = np.concatenate([m.tri_idx[:b + k], m.tri_idx[b + k + 1:]]).astype(np.int32)
    t.tri_ptr = m.tri_ptr.copy()
    t.tri_ptr[node + 1:] -= 1
    t.name = m.name + "_trimmed"
    return t


@pytest.mark.parametrize("which,tri", [("smaller", 61), ("larger", 72)])
def test_inconsistent_incidence_rows_follow_each_row(which, tri):
    """A triangle listed by one free vertex but not by another: every node's
    minima come from its own row, as in the oracle.  The tile path lists a
    triangle once per tile and scores it for all its own vertices, so such a
    mesh runs on the node kernel; results equal the oracle either way, and
    with the rows left whole the tile kernel runs.  The triangles are ones
    whose removal from the row of its smallest (or largest) vertex changes
    that node's first-sweep decision in the oracle."""
    m = meshgen.make_grid(30, "random", 0.4, 91)
    vs = sorted(int(v) for v in m.tris[tri])
    assert all(m.boundary[v] == 0 for v in vs)
    node = vs[0] if which == "smaller" else vs[-1]
    tm = _trim_incidence(m, node, tri)
    assert (oracle.smooth(tm, 1).flags != oracle.smooth(m, 1).flags).any()
    X, rep, ref, nd = assert_parity(tm, 4)
    assert nd == 0 and rep.kernel_used == sl.KERNELS["node"]
    X, rep, ref, nd = assert_parity(tm, 4, kernel="tile")
    assert nd == 0 and rep.kernel_used == sl.KERNELS["node"]
    X, rep, ref, nd = assert_parity(m, 4)
    assert nd == 0 and rep.kernel_used == sl.KERNELS["tile"]
