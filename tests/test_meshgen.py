"""Input generators: sizes, orientation, adjacency and boundary rule.

The adjacency rows follow the paper's neighbour-finding rule (Sec. 3.3.2) and
the boundary mask its recorded-twice rule (Sec. 3.3.3); both are checked here
against brute-force scans and against the geometric boundary.
"""
import numpy as np
import pytest

import meshgen
from oracle.exact import incidence


def _cross(m, X=None):
    X = m.coords if X is None else X
    p0, p1, p2 = X[m.tris[:, 0]], X[m.tris[:, 1]], X[m.tris[:, 2]]
    a, b = p1 - p0, p2 - p0
    return a[:, 0] * b[:, 1] - b[:, 0] * a[:, 1]


@pytest.mark.parametrize("n", [2, 3, 5, 64])
@pytest.mark.parametrize("diag", ["unionjack", "random", "slash", "backslash"])
def test_grid_counts(n, diag):
    m = meshgen.make_grid(n, diag, 0.0, 7)
    assert m.n_nodes == n * n
    assert m.n_tris == 2 * (n - 1) ** 2
    assert m.n_interior == max(n - 2, 0) ** 2
    E = 2 * n * (n - 1) + (n - 1) ** 2
    assert len(m.nbr_idx) == 2 * E
    assert m.tri_ptr[-1] == 3 * m.n_tris
    assert (_cross(m) > 0).all()


def test_config_sizes_small():
    m = meshgen.make_grid(64, "unionjack", 0.3, 1)
    assert (m.n_nodes, m.n_tris, m.n_interior, len(m.nbr_idx)) == (4096, 7938, 3844, 24066)
    d = np.diff(m.nbr_ptr)[m.boundary == 0]
    assert set(np.unique(d)) == {4, 8}          # Union-Jack valence alternates 8 / 4


def test_annulus_counts_and_orientation():
    a = meshgen.make_annulus(16, 24, diag="random", jitter=0.4, seed=4)
    assert a.n_nodes == 16 * 24
    assert a.n_tris == 2 * 15 * 24
    assert a.n_interior == 14 * 24
    a0 = meshgen.make_annulus(16, 24, diag="random", jitter=0.0, seed=4)
    assert (_cross(a0) > 0).all()               # (r, theta) map keeps parameter-CCW triangles CCW
    r = np.hypot(a.coords[:, 0], a.coords[:, 1])
    bnd = a.boundary.astype(bool)
    assert np.allclose(np.sort(np.unique(np.round(r[bnd], 12))), [0.3, 1.0])


def test_jitter_bounds_and_boundary_untouched():
    n = 33
    h = 1.0 / (n - 1)
    m0 = meshgen.make_grid(n, "random", 0.0, 5)
    m = meshgen.make_grid(n, "random", 0.4, 5)
    assert (m.tris == m0.tris).all()
    b = m.boundary.astype(bool)
    assert (m.coords[b] == m0.coords[b]).all()
    d = np.abs(m.coords[~b] - m0.coords[~b])
    assert d.max() <= 0.4 * h and d.max() > 0.3 * h
    # +-0.4h jitter already inverts a few triangles (they start with q < 0)
    assert 0 < np.count_nonzero(_cross(m) <= 0) < 0.01 * m.n_tris


def _first_appearance_rows(n, tris):
    rows = [[] for _ in range(n)]
    for a, b, c in tris:
        for v, us in ((a, (b, c)), (b, (a, c)), (c, (a, b))):
            for u in us:
                if u not in rows[v]:
                    rows[v].append(u)
    return rows


@pytest.mark.parametrize("seed", [0, 1])
def test_adjacency_matches_bruteforce(seed):
    m = meshgen.permute_mesh(meshgen.make_grid(9, "random", 0.3, seed), seed + 10)
    rows = _first_appearance_rows(m.n_nodes, m.tris.tolist())
    nbrs, inc = incidence(m.n_nodes, m.tris.tolist())
    for v in range(m.n_nodes):
        row = m.nbr_idx[m.nbr_ptr[v]:m.nbr_ptr[v + 1]].tolist()
        assert row == rows[v]
        assert set(row) == nbrs[v]
        assert m.tri_idx[m.tri_ptr[v]:m.tri_ptr[v + 1]].tolist() == inc[v]


def test_boundary_rule_equals_geometric_boundary():
    n = 17
    m = meshgen.make_grid(n, "random", 0.3, 3)
    j, i = np.divmod(np.arange(n * n), n)
    geo = (i == 0) | (i == n - 1) | (j == 0) | (j == n - 1)
    assert (m.boundary.astype(bool) == geo).all()
    mp = meshgen.permute_mesh(m, 4)
    assert mp.n_interior == m.n_interior


def test_interior_rows_are_closed_fans():
    m = meshgen.make_grid(20, "random", 0.4, 9)
    for v in np.flatnonzero(m.boundary == 0):
        assert m.nbr_ptr[v + 1] - m.nbr_ptr[v] == m.tri_ptr[v + 1] - m.tri_ptr[v]


def test_seeds_reproducible_and_distinct():
    a = meshgen.make_grid(16, "random", 0.4, 2)
    b = meshgen.make_grid(16, "random", 0.4, 2)
    c = meshgen.make_grid(16, "random", 0.4, 3)
    assert (a.coords == b.coords).all() and (a.tris == b.tris).all()
    assert not (a.coords == c.coords).all()


def test_relabel_keep_rows_is_a_relabelling():
    m = meshgen.make_grid(8, "random", 0.3, 1)
    perm = np.random.Generator(np.random.PCG64(5)).permutation(m.n_nodes)
    r = meshgen.relabel_keep_rows(m, perm)
    for v in range(m.n_nodes):
        w = perm[v]
        assert (r.coords[w] == m.coords[v]).all()
        assert r.nbr_idx[r.nbr_ptr[w]:r.nbr_ptr[w + 1]].tolist() == perm[m.nbr_idx[m.nbr_ptr[v]:m.nbr_ptr[v + 1]]].tolist()
        assert r.tri_idx[r.tri_ptr[w]:r.tri_ptr[w + 1]].tolist() == m.tri_idx[m.tri_ptr[v]:m.tri_ptr[v + 1]].tolist()


def test_batch_sides_range():
    s = meshgen.batch_sides(10000, 24, 450, 10000)
    assert s.min() >= 24 and s.max() <= 450
    assert abs(np.mean(s.astype(float) ** 2) - 34444) / 34444 < 0.05
