"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here checks the oracle against something other than itself:
closed forms, exact rational arithmetic, invariants of the method, or
special cases with a known answer.  None retypes the oracle's formula.
"""
import hashlib
import json
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import meshgen
import oracle
from oracle.exact import exact_sweep

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "stars.json")
getcontext().prec = 60
TWO_SQRT3 = Decimal(12).sqrt()
ULP1 = math.ulp(1.0)


def exact_q(p0, p1, p2) -> Decimal:
    """4*sqrt(3)*A / sum(l^2) from the textbook definition: area by the
    shoelace formula, squared lengths by Pythagoras, exact rationals."""
    P = [(Fraction(float(x)), Fraction(float(y))) for x, y in (p0, p1, p2)]
    A2 = sum(P[k][0] * P[(k + 1) % 3][1] - P[(k + 1) % 3][0] * P[k][1] for k in range(3))  # 2*area
    L = sum((P[(k + 1) % 3][0] - P[k][0]) ** 2 + (P[(k + 1) % 3][1] - P[k][1]) ** 2 for k in range(3))
    if L == 0:
        return Decimal(0)
    r = A2 / L
    return TWO_SQRT3 * Decimal(r.numerator) / Decimal(r.denominator)


# ---------------------------------------------------------------- quality --

def test_quality_equilateral_is_one():
    q = oracle.quality(0.0, 0.0, 1.0, 0.0, 0.5, math.sqrt(3.0) / 2)
    assert abs(q - 1.0) <= ULP1


def test_quality_right_isosceles_is_sqrt3_over_2():
    # cr = 1 and S = 4 are exact, so q = fl(2*sqrt(3))/4 = fl(sqrt(3))/2 exactly
    assert oracle.quality(0.0, 0.0, 1.0, 0.0, 0.0, 1.0) == math.sqrt(3.0) / 2


def test_quality_orientation_sign_and_swap():
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(200):
        p = rng.uniform(-1, 1, size=(3, 2))
        q = oracle.quality(*p[0], *p[1], *p[2])
        # swapping v1 and v2 negates the cross product exactly; S is the same
        # sum grouped differently, so the magnitude agrees up to rounding
        qs = oracle.quality(*p[0], *p[2], *p[1])
        assert np.sign(qs) == -np.sign(q)
        assert abs(qs + q) <= 4 * ULP1 * abs(q)
        assert q <= 1.0 + 4 * ULP1                 # 4 sqrt(3) A <= sum l^2
        cw = (p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[2, 0] - p[0, 0]) * (p[1, 1] - p[0, 1]) < 0
        assert (q < 0) == cw


def test_quality_degenerate():
    assert oracle.quality(0.0, 0.0, 1.0, 1.0, 2.0, 2.0) == 0.0    # collinear: zero area
    assert oracle.quality(0.5, 0.5, 0.5, 0.5, 0.5, 0.5) == 0.0    # coincident: S == 0 -> 0


def test_quality_power_of_two_scaling_is_exact():
    rng = np.random.Generator(np.random.PCG64(12))
    for _ in range(100):
        p = rng.uniform(-1, 1, size=(3, 2))
        q = oracle.quality(*p.ravel())
        for s in (2.0 ** -20, 0.5, 8.0, 2.0 ** 30):
            assert oracle.quality(*(p * s).ravel()) == q


def test_quality_matches_textbook_definition():
    """Against 4*sqrt(3)*A/sum(l^2) in exact arithmetic: a dropped or doubled
    edge term, a swapped coordinate or a wrong constant fails this."""
    rng = np.random.Generator(np.random.PCG64(13))
    for _ in range(300):
        p = rng.uniform(-3, 3, size=(3, 2))
        q = oracle.quality(*p.ravel())
        e = exact_q(*p)
        tol = Decimal(16) * Decimal(2) ** -53 * max(Decimal(1), abs(e)) + Decimal(2) ** -60
        # cancellation in cr for near-collinear triangles: scale by the terms
        terms = abs(Decimal(float(p[1, 0] - p[0, 0]) * float(p[2, 1] - p[0, 1]))) + \
            abs(Decimal(float(p[2, 0] - p[0, 0]) * float(p[1, 1] - p[0, 1])))
        S = sum(float(np.sum((p[(k + 1) % 3] - p[k]) ** 2)) for k in range(3))
        tol += Decimal(8) * Decimal(2) ** -53 * TWO_SQRT3 * terms / Decimal(S)
        assert abs(Decimal(q) - e) <= tol, (p, q, e)


def test_quality_rotation_of_vertex_order():
    """Rotating the stored order is the same triangle: equal up to rounding."""
    rng = np.random.Generator(np.random.PCG64(14))
    for _ in range(200):
        p = rng.uniform(-1, 1, size=(3, 2))
        q0 = oracle.quality(*p[0], *p[1], *p[2])
        q1 = oracle.quality(*p[1], *p[2], *p[0])
        assert abs(q0 - q1) <= 64 * ULP1 * (1 + abs(q0)) / max(abs(q0), 1e-3)


# ------------------------------------------------------------ star golden --

def _golden():
    with open(GOLDEN) as f:
        return {c["name"]: c for c in json.load(f)["cases"]}


@pytest.mark.parametrize("name", ["square_star", "arm_star_inverting", "arm_star_no_inversion"])
def test_star_golden(name):
    c = _golden()[name]
    m = meshgen.star_mesh(c["center"], c["ring"])
    assert m.tris.tolist() == c["tris"]
    assert m.boundary.tolist() == [0] + [1] * len(c["ring"])
    X0 = m.coords.copy()
    qo = min(oracle.quality(*X0[a], *X0[b], *X0[t]) for a, b, t in m.tris)
    cen = [float(Fraction(s)) for s in c["centroid"]]
    X1 = X0.copy()
    X1[0] = cen
    qn = min(oracle.quality(*X1[a], *X1[b], *X1[t]) for a, b, t in m.tris)
    assert abs(Decimal(qo) - Decimal(c["q_old_min"])) <= Decimal(4) * Decimal(2) ** -53
    assert abs(Decimal(qn) - Decimal(c["q_new_min"])) <= Decimal(4) * Decimal(2) ** -53
    for gt, key in ((False, "accept_ge"), (True, "accept_gt")):
        r = oracle.smooth(m, 1, accept_gt=gt)
        assert r.flags[0, 0] == int(c[key])
        assert (r.flags[0, 1:] == 2).all()
        if c[key]:
            assert r.coords[0].tolist() == cen          # centroid is exactly representable here
        else:
            assert r.coords[0].tolist() == c["center"]
        assert (r.coords[1:] == X0[1:]).all()


def test_square_star_second_sweep_and_tie_rule():
    c = _golden()["square_star"]
    m = meshgen.star_mesh(c["center"], c["ring"])
    ge = oracle.smooth(m, 3)
    gt = oracle.smooth(m, 3, accept_gt=True)
    assert ge.coords[0].tolist() == [0.0, 0.0] and gt.coords[0].tolist() == [0.0, 0.0]
    # at the fixed point the candidate equals the position: a tie
    assert ge.flags[:, 0].tolist() == [1, 1, 1]
    assert gt.flags[:, 0].tolist() == [1, 0, 0]
    assert ge.disp.tolist() == [0.3 * 0.3 + 0.2 * 0.2, 0.0, 0.0]
    assert ge.accepted.tolist() == [1, 1, 1] and gt.accepted.tolist() == [1, 0, 0]


def test_tolerance_stop_rule():
    c = _golden()["square_star"]
    m = meshgen.star_mesh(c["center"], c["ring"])
    # first sweep moves by sqrt(0.13) ~ 0.36, the second by 0
    assert oracle.smooth(m, 10, tol=0.5).iterations_run == 1
    assert oracle.smooth(m, 10, tol=0.3).iterations_run == 2
    assert oracle.smooth(m, 10, tol=0.0).iterations_run == 10
    assert oracle.smooth(m, 0).iterations_run == 0


# ------------------------------------------------------- grid fixed points --

@pytest.mark.parametrize("diag", ["unionjack", "slash"])
def test_dyadic_regular_grid_is_exact_fixed_point(diag):
    """h = 1/64: every sum is exact, each free node is the centroid of its
    symmetric neighbourhood, so the candidate equals the position."""
    m = meshgen.make_grid(65, diag, 0.0, 0, h=1.0 / 64)
    ge = oracle.smooth(m, 3)
    gt = oracle.smooth(m, 3, accept_gt=True)
    assert (ge.coords == m.coords).all() and (gt.coords == m.coords).all()
    free = m.boundary == 0
    assert (ge.flags[:, free] == 1).all()
    assert (gt.flags[:, free] == 0).all()
    assert (ge.disp == 0).all()


def test_nondyadic_regular_grid_moves_by_rounding_only():
    m = meshgen.make_grid(64, "unionjack", 0.0, 0)
    r = oracle.smooth(m, 2)
    assert np.abs(r.coords - m.coords).max() <= 8 * math.ulp(1.0)
    assert r.disp.max() <= (8 * math.ulp(1.0)) ** 2 * 2


def test_random_diagonal_grid_smart_rejects_unbalanced_moves():
    """Unjittered random diagonals: a node with unbalanced diagonal neighbours
    has its centroid off its position (plain Laplacian would move it), but all
    its triangles are right isosceles and any move lowers the worst one, so
    Smart Laplacian rejects it; balanced nodes tie and are accepted (GE)."""
    m = meshgen.make_grid(17, "random", 0.0, 3, h=1.0 / 16)
    r = oracle.smooth(m, 1)
    moved = 0
    for i in np.flatnonzero(m.boundary == 0):
        nb = m.nbr_idx[m.nbr_ptr[i]:m.nbr_ptr[i + 1]]
        c = m.coords[nb].sum(axis=0) / len(nb)      # dyadic grid: exact
        if (c != m.coords[i]).any():
            moved += 1
            assert r.flags[0, i] == 0
        else:
            assert r.flags[0, i] == 1
    assert moved > 10
    assert r.disp[0] == 0.0 and (r.coords == m.coords).all()


# -------------------------------------------------------------- invariants --

def _hash(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_boundary_fixed_and_connectivity_unchanged():
    m = meshgen.make_grid(40, "random", 0.4, 21)
    before = _hash(m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary)
    r = oracle.smooth(m, 25)
    assert _hash(m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary) == before
    b = m.boundary.astype(bool)
    assert (r.coords[b] == m.coords[b]).all()
    assert np.isfinite(r.coords).all()
    assert (r.flags[:, b] == 2).all()


def test_jacobi_is_independent_of_node_labels():
    """Form A reads only pass-q positions, so any relabelling that keeps rows
    and triangle vertex order gives bit-identical positions and flags."""
    m = meshgen.make_grid(30, "random", 0.4, 22)
    perm = np.random.Generator(np.random.PCG64(3)).permutation(m.n_nodes)
    mr = meshgen.relabel_keep_rows(m, perm)
    a = oracle.smooth(m, 12)
    b = oracle.smooth(mr, 12)
    assert (b.coords[perm] == a.coords).all()
    assert (b.flags[:, perm] == a.flags).all()
    assert (a.disp == b.disp).all()


def test_resume_is_bit_exact():
    m = meshgen.make_grid(30, "random", 0.4, 23)
    full = oracle.smooth(m, 40)
    half = oracle.smooth(m, 20)
    m2 = m.copy()
    m2.coords = half.coords
    rest = oracle.smooth(m2, 20)
    assert (rest.coords == full.coords).all()
    assert (np.concatenate([half.flags, rest.flags]) == full.flags).all()


def test_threads_are_bit_identical():
    m = meshgen.make_grid(60, "random", 0.4, 24)
    a = oracle.smooth(m, 8, threads=1)
    b = oracle.smooth(m, 8, threads=max(2, oracle.max_threads()))
    assert (a.coords == b.coords).all() and (a.flags == b.flags).all() and (a.disp == b.disp).all()


def test_decisions_are_consistent_with_patch_minima():
    """Decision-time invariant: an accepted node does not lower the worst
    quality of its incident triangles (evaluated on pass-q positions); a
    rejected node would have lowered it."""
    m = meshgen.make_grid(20, "random", 0.4, 25)
    X = m.coords.copy()
    for _ in range(3):
        Xn, fl, _, _ = oracle.sweep(m, X)
        for i in np.flatnonzero(m.boundary == 0):
            ts = m.tri_idx[m.tri_ptr[i]:m.tri_ptr[i + 1]]
            nb = m.nbr_idx[m.nbr_ptr[i]:m.nbr_ptr[i + 1]]
            c = X[nb].sum(axis=0) / len(nb)         # order-free check: exact-enough centroid
            Y = X.copy()
            Y[i] = c
            qo = min(oracle.quality(*X[m.tris[t, 0]], *X[m.tris[t, 1]], *X[m.tris[t, 2]]) for t in ts)
            qn = min(oracle.quality(*Y[m.tris[t, 0]], *Y[m.tris[t, 1]], *Y[m.tris[t, 2]]) for t in ts)
            if abs(qn - qo) > 1e-9:
                assert fl[i] == (1 if qn > qo else 0)
            if fl[i] == 1:
                assert np.abs(Xn[i] - c).max() <= 1e-15
            else:
                assert (Xn[i] == X[i]).all()
        X = Xn


# ---------------------------------------------------------- exact brute force --

@pytest.mark.parametrize("n,seed", [(3, 1), (4, 2), (5, 3), (6, 4), (8, 5)])
def test_exact_rational_brute_force(n, seed):
    """Each sweep checked against exact rational arithmetic from the same
    pass-q positions: decisions must agree wherever the exact relative margin
    exceeds 1e-12; accepted positions lie within the rounding bound of the
    exact centroid; rejected nodes do not move."""
    m = meshgen.make_grid(n, "random", 0.4, seed)
    X = m.coords.copy()
    u = 2.0 ** -53
    checked = 0
    for _ in range(3):
        Xn, fl, _, _ = oracle.sweep(m, X)
        ex = exact_sweep(X, m.tris.tolist(), m.boundary.tolist())
        for i, d in ex.items():
            if d.rel_margin > Fraction(1, 10 ** 12):
                assert fl[i] == int(d.accept_ge), (i, float(d.rel_margin))
                checked += 1
            if fl[i] == 1:
                nb = m.nbr_idx[m.nbr_ptr[i]:m.nbr_ptr[i + 1]]
                k = len(nb)
                bound = (k + 1) * u * float(np.abs(X[nb]).sum(axis=0).max()) / k + 2 * u
                for ax in range(2):
                    assert abs(Fraction(float(Xn[i, ax])) - d.centroid[ax]) <= Fraction(bound)
            else:
                assert (Xn[i] == X[i]).all()
        X = Xn
    assert checked > 0


def test_exact_brute_force_gt_rule():
    m = meshgen.make_grid(6, "random", 0.4, 6)
    Xn, fl, _, _ = oracle.sweep(m, m.coords, accept_gt=True)
    ex = exact_sweep(m.coords, m.tris.tolist(), m.boundary.tolist())
    for i, d in ex.items():
        if d.rel_margin > Fraction(1, 10 ** 12):
            assert fl[i] == int(d.accept_gt)


# ------------------------------------------------------------- Form B ------

def _mesh_min(m, X):
    return min(oracle.quality(*X[a], *X[b], *X[c]) for a, b, c in m.tris)


def test_coloring_is_proper_and_greedy():
    m = meshgen.make_grid(25, "random", 0.4, 31)
    col, nc = oracle.colors(m)
    free = m.boundary == 0
    assert (col[~free] == -1).all() and (col[free] >= 0).all() and nc == col.max() + 1
    order = sorted(np.flatnonzero(free), key=lambda v: -oracle.priority(int(v)))
    rank = {int(v): k for k, v in enumerate(order)}
    for v in np.flatnonzero(free):
        nb = [int(u) for u in m.nbr_idx[m.nbr_ptr[v]:m.nbr_ptr[v + 1]] if free[u]]
        assert all(col[u] != col[v] for u in nb)
        earlier = {int(col[u]) for u in nb if rank[u] < rank[int(v)]}
        assert col[v] == min(set(range(nc + 1)) - earlier)
    assert nc <= 9


def test_splitmix64_published_vector():
    # SplitMix64 output for state increments starting from seed 0: the first
    # output of the generator seeded with 0 is 0xE220A8397B1DCDAF.
    assert oracle.priority(0) == 0xE220A8397B1DCDAF


def test_colored_equals_jacobi_when_free_nodes_are_independent():
    """Form A is Form B with N_{q+1} = 0 (eq. (3)): with no two free nodes
    adjacent there is nothing to read from pass q+1."""
    c = _golden()["arm_star_no_inversion"]
    for mm in (meshgen.make_grid(3, "random", 0.4, 1), meshgen.star_mesh(c["center"], c["ring"]),
               meshgen.star_mesh((0.3, -0.2), [(1, 0), (0, 1), (-1, 0), (0, -1)])):
        a = oracle.smooth(mm, 4)
        b = oracle.smooth(mm, 4, form="colored")
        assert (a.coords == b.coords).all() and (a.flags == b.flags).all()


def test_colored_invariants():
    m = meshgen.make_grid(30, "random", 0.4, 32)
    X = m.coords.copy()
    prev = _mesh_min(m, X)
    mm = m.copy()
    for _ in range(6):
        mm.coords = X
        r = oracle.smooth(mm, 1, form="colored")
        Xn = r.coords
        b = m.boundary.astype(bool)
        assert (Xn[b] == m.coords[b]).all() and np.isfinite(Xn).all()
        cur = _mesh_min(m, Xn)
        assert cur >= prev                          # exact: no triangle has two movers per class
        prev = cur
        X = Xn
    j = oracle.smooth(m, 6)
    assert not (j.coords == X).all()                # the two forms differ on a real mesh


# ------------------------------------------------------ single precision ----

def f32(x):
    return float(np.float32(x))


def test_quality32_closed_forms():
    k32 = np.float32(2.0) * np.sqrt(np.float32(3.0))          # float nearest 2*sqrt(3)
    # right isosceles (0,0),(1,0),(0,1): cr = 1, S = 4, q = K/4 exactly
    assert oracle.quality32(0, 0, 1, 0, 0, 1) == float(k32 / np.float32(4))
    q = oracle.quality32(0, 0, 1, 0, 0.5, f32(math.sqrt(3) / 2))
    assert abs(q - 1.0) <= 4 * 2.0 ** -24
    assert oracle.quality32(0, 0, 1, 0, 0, 1) == -oracle.quality32(0, 0, 0, 1, 1, 0)
    assert oracle.quality32(1, 1, 1, 1, 1, 1) == 0.0
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(200):
        p = [f32(v) for v in rng.uniform(-1, 1, 6)]
        exact = float(exact_q((p[0], p[1]), (p[2], p[3]), (p[4], p[5])))
        q32 = oracle.quality32(*p)
        # a few float roundings of terms no larger than S: absolute error a few ulps of 1
        assert abs(q32 - exact) <= 64 * 2.0 ** -24 * max(1.0, abs(exact)), (p, q32, exact)


def test_f32_dyadic_grids_are_fixed_points():
    for diag in ("unionjack", "slash"):
        m = meshgen.make_grid(9, diag, 0.0, 0, h=0.125)
        r = oracle.smooth(m, 3, precision="f32")
        assert (r.coords == m.coords).all()
        assert (r.flags[:, m.boundary == 0] == 1).all()
        r = oracle.smooth(m, 2, precision="f32", accept_gt=True)
        assert (r.flags[:, m.boundary == 0] == 0).all()


@pytest.mark.parametrize("n,seed", [(6, 31), (8, 32)])
def test_f32_exact_rational_brute_force(n, seed):
    """One single-precision sweep from float positions against exact rational
    arithmetic: decisions agree wherever the exact relative margin exceeds
    1e-4, accepted positions lie within the float rounding bound of the
    exact centroid, results are floats."""
    m = meshgen.make_grid(n, "random", 0.4, seed)
    m.coords = m.coords.astype(np.float32).astype(np.float64)
    r = oracle.smooth(m, 1, precision="f32")
    ex = exact_sweep(m.coords, m.tris.tolist(), m.boundary.tolist())
    u = 2.0 ** -24
    checked = 0
    for i, d in ex.items():
        if d.rel_margin > Fraction(1, 10 ** 4):
            assert r.flags[0, i] == int(d.accept_ge), (i, float(d.rel_margin))
            checked += 1
        if r.flags[0, i] == 1:
            nb = m.nbr_idx[m.nbr_ptr[i]:m.nbr_ptr[i + 1]]
            k = len(nb)
            bound = (k + 1) * u * float(np.abs(m.coords[nb]).sum(axis=0).max()) / k + 2 * u
            for ax in range(2):
                assert abs(Fraction(float(r.coords[i, ax])) - d.centroid[ax]) <= Fraction(bound)
        else:
            assert (r.coords[i] == m.coords[i]).all()
    assert checked > 0.8 * len(ex)
    assert (r.coords.astype(np.float32).astype(np.float64) == r.coords).all()


def test_f32_tracks_f64():
    """Same decisions as FP64 in the first sweep except at near-ties, and
    positions within float resolution of the FP64 run over a few sweeps."""
    m = meshgen.make_grid(40, "random", 0.4, 12)
    a = oracle.smooth(m, 1, precision="f32")
    b = oracle.smooth(m, 1)
    assert (a.flags != b.flags).sum() <= 3
    a = oracle.smooth(m, 5, precision="f32")
    b = oracle.smooth(m, 5)
    assert np.abs(a.coords - b.coords).max() < 1e-3
    with pytest.raises(ValueError):
        oracle.smooth(m, 1, precision="f32", form="colored")


def test_f32_centroid_sums_in_float_in_row_order():
    """Neighbour x-coordinates 1, 2^-24, 2^-24, 2^-24 in row order: in float
    each addition of 2^-24 to 1 is a tie that rounds back to 1, so the sum is
    exactly 1 and the centroid's x exactly 0.25 (in double the small terms
    survive).  The move is accepted, so the node lands on it."""
    t = 2.0 ** -24
    ring = np.array([[1.0, 0.25], [t, 0.75], [t, 0.25], [t, -0.25]])
    m = meshgen.star_mesh(np.array([0.1, 0.25]), ring)
    assert m.nbr_idx[m.nbr_ptr[0]:m.nbr_ptr[1]].tolist() == [1, 2, 3, 4]
    r = oracle.smooth(m, 1, precision="f32")
    assert r.flags[0, 0] == 1 and r.coords[0].tolist() == [0.25, 0.25]
    r64 = oracle.smooth(m, 1)
    assert r64.flags[0, 0] == 1 and r64.coords[0, 0] == (1 + 3 * t) / 4


def test_f64_centroid_sums_in_row_order():
    """Neighbour x-coordinates 1, 2^-53, 2^-53, 2^-53 in row order: each
    addition of 2^-53 (half an ulp of 1) to 1 is a tie that rounds back to 1,
    so the row-order sum is exactly 1 and the centroid's x exactly 0.25.
    Summed in reverse, sorted or pairwise, the small terms first combine and
    survive (1 + 2^-51 or 1 + 2^-52), so any other order moves the node
    somewhere else.  The exact rational decision accepts with a wide margin,
    so the node lands on the rounded centroid."""
    t = 2.0 ** -53
    ring = np.array([[1.0, 0.25], [t, 0.75], [t, 0.25], [t, -0.25]])
    m = meshgen.star_mesh(np.array([0.1, 0.25]), ring)
    assert m.nbr_idx[m.nbr_ptr[0]:m.nbr_ptr[1]].tolist() == [1, 2, 3, 4]
    d = exact_sweep(m.coords, m.tris, m.boundary)[0]
    assert d.accept_ge and d.rel_margin > Fraction(1, 100)
    # the other orders give other sums (plain float arithmetic, no oracle)
    assert ((t + t) + t) + 1.0 == 1.0 + 2.0 ** -51
    assert (1.0 + t) + (t + t) == 1.0 + 2.0 ** -52
    r = oracle.smooth(m, 1)
    assert r.flags[0, 0] == 1 and r.coords[0].tolist() == [0.25, 0.25]
