"""Pins for the adjacency oracle (paper Sec. 3.3.2 finding of neighbours,
Sec. 3.3.3 determining of constraints).

Hand-worked cases fix the recording order, the first-appearance rule and the
recorded-twice boundary rule; on generated meshes the oracle must agree with
the generators' independent C builder and with the geometric boundary.
"""
import numpy as np
import pytest

import meshgen
from oracle.adjacency import adjacency


def rows(ptr, idx):
    return [list(idx[ptr[v]:ptr[v + 1]]) for v in range(len(ptr) - 1)]


def test_single_triangle_recording_order():
    # (v1, v2, v3) = (5, 2, 9): v1 gets v2, v3; v2 gets v1, v3; v3 gets v1, v2
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = adjacency(10, [[5, 2, 9]])
    r = rows(nbr_ptr, nbr_idx)
    assert r[5] == [2, 9] and r[2] == [5, 9] and r[9] == [5, 2]
    assert all(r[v] == [] for v in (0, 1, 3, 4, 6, 7, 8))
    assert rows(tri_ptr, tri_idx)[5] == [0] and rows(tri_ptr, tri_idx)[0] == []
    assert bnd.tolist() == [1] * 10          # every edge seen once; isolated nodes are boundary


def test_two_triangles_first_appearance():
    # t0 = (0, 1, 2), t1 = (2, 1, 3): node 1 is the second vertex of both
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = adjacency(4, [[0, 1, 2], [2, 1, 3]])
    r = rows(nbr_ptr, nbr_idx)
    assert r[0] == [1, 2]
    assert r[1] == [0, 2, 3]        # t0 gives 0, 2; t1 gives 2 (again), 3
    assert r[2] == [0, 1, 3]        # t0 gives 0, 1; t1 (first vertex) gives 1 (again), 3
    assert r[3] == [2, 1]
    assert rows(tri_ptr, tri_idx) == [[0], [0, 1], [0, 1], [1]]
    assert bnd.tolist() == [1, 1, 1, 1]


def test_closed_star_interior_and_rim():
    tris = [[0, i, i % 6 + 1] for i in range(1, 7)]
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = adjacency(7, tris)
    r = rows(nbr_ptr, nbr_idx)
    assert r[0] == [1, 2, 3, 4, 5, 6]
    assert r[1] == [0, 2, 6]        # from (0,1,2) then (0,6,1)
    assert r[6] == [0, 5, 1]        # from (0,5,6) then (0,6,1)
    assert bnd.tolist() == [0, 1, 1, 1, 1, 1, 1]
    assert rows(tri_ptr, tri_idx)[0] == [0, 1, 2, 3, 4, 5]
    assert rows(tri_ptr, tri_idx)[1] == [0, 5]


def test_edge_in_three_triangles_is_boundary():
    # the edge (0, 1) lies in three triangles: node 0 sees 1 three times
    tris = [[0, 1, 2], [1, 0, 3], [0, 1, 4], [0, 2, 5], [0, 5, 3], [0, 4, 6]]
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = adjacency(7, tris)
    assert bnd[0] == 1


@pytest.mark.parametrize("make", [
    lambda: meshgen.make_grid(9, "unionjack", 0.0, 0),
    lambda: meshgen.make_grid(13, "random", 0.3, 4),
    lambda: meshgen.make_annulus(6, 11, seed=2),
    lambda: meshgen.permute_mesh(meshgen.make_grid(11, "random", 0.4, 5), 7),
])
def test_agrees_with_the_generator_builder(make):
    m = make()
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = adjacency(m.n_nodes, m.tris)
    assert np.array_equal(nbr_ptr, m.nbr_ptr) and np.array_equal(nbr_idx, m.nbr_idx)
    assert np.array_equal(tri_ptr, m.tri_ptr) and np.array_equal(tri_idx, m.tri_idx)
    assert np.array_equal(bnd, m.boundary)


def test_grid_boundary_is_the_geometric_boundary():
    n = 12
    m = meshgen.make_grid(n, "random", 0.0, 3)
    bnd = adjacency(m.n_nodes, m.tris)[4]
    j, i = np.divmod(np.arange(n * n), n)
    geo = ((i == 0) | (j == 0) | (i == n - 1) | (j == n - 1)).astype(np.uint8)
    assert np.array_equal(bnd, geo)
