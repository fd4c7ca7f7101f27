"""GPU parity of Form B (eq. (3): coloured, in place) on colour-class tiles.

The free nodes of each colour class are cut into tiles of consecutive device
labels; one launch per class sweeps its tiles in place (no two nodes of a
class are adjacent, so no tile reads what another writes).  The colouring is
the oracle's, so the bar is the Jacobi form's: accept flags bit-exact in
every sweep, coordinates within 1e-12 (bit-exact expected and asserted).
Class starts fall at any label, so the accept bits of a wave straddle words:
flags are compared for every sweep."""
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


def run_gpu(m, iters, tol=0.0, **opts):
    import torch
    dev = sl.to_device(m, "cuda:0")
    nbytes = (m.n_nodes + 7) // 8
    flags = torch.zeros(max(iters, 1) * nbytes, dtype=torch.uint8, device="cuda:0")
    rep = sl.smooth_mesh_device(*dev, iterations=iters, tol=tol, flags=flags, form="colored", **opts)
    torch.cuda.synchronize()
    F = sl.unpack_flags(flags.cpu().numpy().reshape(max(iters, 1), nbytes), m.n_nodes)[:iters]
    return dev[0].cpu().numpy(), rep, F


def check(m, iters, tol=0.0, accept="ge", kernel="tile", **opts):
    note("form B %s iters=%d tol=%g accept=%s %s" % (m.name, iters, tol, accept, opts))
    X, rep, F = run_gpu(m, iters, tol, accept=accept, kernel=kernel, **opts)
    assert rep.kernel_used == sl.KERNELS[kernel]
    ref = oracle.smooth(m, iters, tol=tol, accept_gt=accept == "gt", form="colored")
    assert rep.n_colors == int(ref.colors.max()) + 1
    assert rep.iterations_run == ref.iterations_run
    k = ref.iterations_run
    bad = np.flatnonzero((F[:k] != (ref.flags == 1)).any(axis=1))
    assert bad.size == 0, "flags differ in sweeps %s" % bad[:10]
    assert (F[k:] == 0).all()
    assert float(np.abs(X - ref.coords).max()) <= COORD_TOL
    assert (X == ref.coords).all()
    if k:
        assert rep.accepted_total == int(ref.accepted.sum())
        assert rep.max_disp_sq_last == ref.disp[-1]
    return X, rep


MESHES = {
    "grid200": lambda: meshgen.make_grid(200, "random", 0.4, 61),
    "unionjack150": lambda: meshgen.make_grid(150, "unionjack", 0.3, 62),
    "annulus": lambda: meshgen.make_annulus(90, 160, seed=63),
    "delaunay20k": lambda: meshgen.make_delaunay(20000, 64),
    "permuted180": lambda: meshgen.permute_mesh(meshgen.make_grid(180, "random", 0.35, 65), 65),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_form_b_class_tiles_equal_the_oracle(name):
    m = MESHES[name]()
    X, rep = check(m, 12)
    # the node kernel runs the same sweeps
    Xn, repn, _ = run_gpu(m, 12, kernel="node")
    assert repn.kernel_used == sl.KERNELS["node"]
    assert (Xn == X).all()


@pytest.mark.parametrize("layout,reorder,accept,tile_nodes", [
    ("soa", "hilbert", "ge", 0), ("aos", "none", "ge", 0), ("aos", "hilbert", "gt", 0),
    ("aos", "hilbert", "ge", 512), ("soa", "none", "gt", 256), ("aos", "hilbert", "ge", 128)])
def test_form_b_class_tiles_options(layout, reorder, accept, tile_nodes):
    m = meshgen.permute_mesh(meshgen.make_grid(130, "random", 0.4, 66), 66)
    X, rep = check(m, 9, accept=accept, layout=layout, reorder=reorder, tile_nodes=tile_nodes)
    assert rep.tile_nodes == (tile_nodes or 256)


def test_form_b_class_tiles_tolerance_and_graph_chunks():
    """Tolerance stops inside and across the 32-sweep graph chunks."""
    m = meshgen.make_grid(120, "random", 0.4, 67)
    ref = oracle.smooth(m, 300, form="colored", want_flags=False)
    # this mesh reaches a zero displacement after 52 coloured sweeps
    for stop in (5, 33, 50):
        assert ref.disp[stop] > 0.0
        tol = float(np.sqrt(ref.disp[stop])) * 1.0000001
        X, rep = check(m, 300, tol=tol)
        assert rep.iterations_run <= stop + 1
    check(m, 96)


def test_form_b_class_tiles_1024_permuted():
    """The permuted 1024^2 grid (1.04M free nodes), 30 sweeps: every flag."""
    m = meshgen.permute_mesh(meshgen.make_grid(1024, "random", 0.4, 2), 2)
    check(m, 30)


def test_form_b_small_class_tiles_on_a_large_mesh():
    """128-node class tiles on a 1200 x 1200 grid: its largest class has
    more tiles than a launch has work-groups (at most 2,048), so the groups
    take several tiles each and fold once per launch."""
    m = meshgen.make_grid(1200, "random", 0.4, 70)
    X, rep = check(m, 3, tile_nodes=128)
    assert rep.tile_nodes == 128


@pytest.mark.parametrize("side", [1024, 2100])
def test_form_b_node_kernel_grouped_and_ungrouped_fans(side):
    """Form B's automatic choice, the node kernel: on the 1024 x 1024 grid
    with each node's fan grouped by stored position, on the 2100 x 2100 grid
    (4.4M free nodes, above the grouping's limit) in incidence order."""
    m = meshgen.make_grid(side, "random", 0.4, 71)
    X, rep = check(m, 3, kernel="node")


def test_form_b_class_tiles_invariants():
    """Boundary fixed, connectivity untouched, and the mesh-wide worst
    quality never drops over a coloured sweep."""
    m = meshgen.make_grid(110, "random", 0.4, 68)
    conn = [a.copy() for a in (m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary)]
    b = m.boundary.astype(bool)

    def worst(c):
        t = m.tris
        return min(oracle.quality(*c[a], *c[p], *c[q]) for a, p, q in t[::7])

    mm = m.copy()
    prev = worst(mm.coords)
    for _ in range(5):
        X, rep, _ = run_gpu(mm, 1, kernel="tile")
        assert rep.kernel_used == sl.KERNELS["tile"]
        assert (X[b] == m.coords[b]).all() and np.isfinite(X).all()
        mm.coords = X
        cur = worst(X)
        assert cur >= prev
        prev = cur
    for a, c in zip(conn, (m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary)):
        assert (a == c).all()


def test_form_b_class_tiles_follow_each_incidence_row():
    """A triangle missing from one of its free vertices' incidence rows: on
    colour-class tiles each triangle is scored for the node whose row lists
    it, as the oracle does (Form A sends such a mesh to the node path)."""
    m = meshgen.make_grid(90, "random", 0.4, 69)
    i = int(np.flatnonzero(m.boundary == 0)[len(m.boundary) // 3])
    row = m.tri_idx[m.tri_ptr[i]:m.tri_ptr[i + 1]]
    keep = np.ones(len(m.tri_idx), bool)
    keep[m.tri_ptr[i] + len(row) - 1] = False          # drop i's last incidence
    mm = m.copy()
    mm.tri_idx = m.tri_idx[keep]
    mm.tri_ptr = m.tri_ptr.copy()
    mm.tri_ptr[i + 1:] -= 1
    check(mm, 6)


@pytest.mark.parametrize("points", [5000, 50000])
def test_delaunay_to_convergence_both_forms(points):
    """Delaunay meshes of uniform random points (the paper's mesh kind) run to
    tol 1e-9 in both forms: the same sweep counts as the oracle and the same
    coordinates, bit for bit; Form B takes fewer sweeps than Form A."""
    import torch
    m = meshgen.make_delaunay(points, 11)
    its = {}
    for form in ("jacobi", "colored"):
        dev = sl.to_device(m, "cuda:0")
        rep = sl.smooth_mesh_device(*dev, iterations=100000, tol=1e-9, form=form)
        torch.cuda.synchronize()
        ref = oracle.smooth(m, 100000, tol=1e-9, form=form, want_flags=False, threads=oracle.max_threads())
        note("delaunay %d %s: %d sweeps (oracle %d)" % (points, form, rep.iterations_run, ref.iterations_run))
        assert rep.iterations_run == ref.iterations_run < 100000
        assert rep.max_disp_sq_last == ref.disp[-1]
        assert rep.accepted_total == int(ref.accepted.sum())
        assert (dev[0].cpu().numpy() == ref.coords).all()
        its[form] = rep.iterations_run
    assert its["colored"] < its["jacobi"]
