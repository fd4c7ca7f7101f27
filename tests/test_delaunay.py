"""The Delaunay generator behind the random-point workloads (the paper's test
meshes are Delaunay meshes of uniformly distributed points, Sec. 4).

Checked with exact integer arithmetic in Python on the lattice coordinates:
every triangle counter-clockwise, the empty-circumcircle property against
every point, the triangle count of a triangulation of the convex hull
(2n - h - 2), edges shared by at most two triangles, and the boundary mask
equal to the convex hull (collinear hull points included)."""
import numpy as np
import pytest

import meshgen


def orient(p, q, r):
    return (q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0])


def incircle(a, b, c, d):
    m = [[a[0] - d[0], a[1] - d[1]], [b[0] - d[0], b[1] - d[1]], [c[0] - d[0], c[1] - d[1]]]
    lift = [r[0] * r[0] + r[1] * r[1] for r in m]
    return (m[0][0] * (m[1][1] * lift[2] - lift[1] * m[2][1])
            - m[0][1] * (m[1][0] * lift[2] - lift[1] * m[2][0])
            + lift[0] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def hull_with_collinear(pts):
    """Indices of the points on the convex hull boundary (monotone chain,
    collinear boundary points kept)."""
    idx = sorted(range(len(pts)), key=lambda i: (pts[i][0], pts[i][1]))

    def chain(seq):
        h = []
        for i in seq:
            while len(h) >= 2 and orient(pts[h[-2]], pts[h[-1]], pts[i]) < 0:
                h.pop()
            h.append(i)
        return h
    return set(chain(idx)) | set(chain(idx[::-1]))


def check(xi, yi, tris, strict_empty=True):
    pts = list(zip((int(v) for v in xi), (int(v) for v in yi)))
    n = len(pts)
    assert tris.min() >= 0 and tris.max() < n
    for a, b, c in tris:
        assert orient(pts[a], pts[b], pts[c]) > 0
    for a, b, c in tris:
        for d in range(n):
            if d in (a, b, c):
                continue
            v = incircle(pts[a], pts[b], pts[c], pts[d])
            assert v <= 0, (a, b, c, d)
    edges = {}
    for a, b, c in tris:
        for u, v in ((a, b), (b, c), (c, a)):
            edges[(min(u, v), max(u, v))] = edges.get((min(u, v), max(u, v)), 0) + 1
    assert max(edges.values()) <= 2
    hull = hull_with_collinear(pts)
    assert len(tris) == 2 * n - len(hull) - 2
    on_boundary = {u for (u, v), c in edges.items() if c == 1} | {v for (u, v), c in edges.items() if c == 1}
    assert on_boundary == hull


def test_square_with_centre():
    xi = np.array([0, 2, 2, 0, 1])
    yi = np.array([0, 0, 2, 2, 1])
    tris = meshgen.delaunay_triangles(xi, yi)
    assert len(tris) == 4 and all(4 in t for t in tris.tolist())
    check(xi, yi, tris)


@pytest.mark.parametrize("n,seed", [(3, 1), (10, 2), (60, 3), (150, 4)])
def test_random_points_exact(n, seed):
    xi, yi = meshgen.random_lattice_points(n, seed)
    check(xi, yi, meshgen.delaunay_triangles(xi, yi))


def test_cocircular_and_collinear_lattice():
    # a 6 x 5 block of lattice points: every cell is cocircular, every side collinear
    j, i = np.divmod(np.arange(30), 6)
    tris = meshgen.delaunay_triangles(i, j)
    assert len(tris) == 2 * 5 * 4
    check(i, j, tris)


def test_degenerate_inputs_rejected():
    with pytest.raises(ValueError):
        meshgen.delaunay_triangles(np.arange(7), np.arange(7) * 2)        # all collinear
    with pytest.raises(ValueError):
        meshgen.delaunay_triangles(np.array([0, 1, 0, 1]), np.array([0, 0, 1, 0]))   # duplicate


def test_make_delaunay_mesh():
    m = meshgen.make_delaunay(2000, 7)
    assert m.n_nodes == 2000
    h = int(m.boundary.sum())
    assert m.n_tris == 2 * 2000 - h - 2
    m2 = meshgen.make_delaunay(2000, 7)
    assert np.array_equal(m.tris, m2.tris) and np.array_equal(m.coords, m2.coords)
    # coordinates are the lattice points scaled by 2^-20, exactly
    lat = m.coords * (2.0 ** meshgen.LATTICE_BITS)
    assert np.array_equal(lat, np.rint(lat)) and lat.min() >= 0 and lat.max() < 2 ** meshgen.LATTICE_BITS
    # counter-clockwise in the floating-point coordinates too (the lattice scaling is exact)
    p = m.coords[m.tris]
    cr = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 1, 1] - p[:, 0, 1]) * (p[:, 2, 0] - p[:, 0, 0])
    assert (cr > 0).all()
