"""ORACLE -- test infrastructure only.

Exact rational brute force of one Jacobi Smart Laplacian sweep for tiny
meshes (paper Sec. 2.1 and eq. (2)).  Every double is converted to the exact
rational it represents; sums, products and quotients are exact.  Neighbours
and incident triangles are found by scanning every triangle for every node,
not from any CSR array, so this path shares nothing with the FP64 oracle
beyond the mesh itself.

The quality 4*sqrt(3)*A/sum(l^2) is compared through cr/S with cr twice the
signed area and S the sum of squared edge lengths: the factor 2*sqrt(3) is a
positive constant and does not change any comparison.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Tuple


def _ratio(p0, p1, p2) -> Fraction:
    (x0, y0), (x1, y1), (x2, y2) = p0, p1, p2
    cr = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
    S = (x1 - x0) ** 2 + (y1 - y0) ** 2 + (x2 - x1) ** 2 + (y2 - y1) ** 2 + (x2 - x0) ** 2 + (y2 - y0) ** 2
    if S == 0:
        return Fraction(0)
    return Fraction(cr) / S


def incidence(n_nodes: int, tris) -> Tuple[List[set], List[list]]:
    """Neighbour sets and incident-triangle lists by a full scan."""
    nbrs = [set() for _ in range(n_nodes)]
    inc = [[] for _ in range(n_nodes)]
    for t, tri in enumerate(tris):
        tri = [int(v) for v in tri]
        for v in range(n_nodes):
            if v in tri:
                inc[v].append(t)
                for u in tri:
                    if u != v:
                        nbrs[v].add(u)
    return nbrs, inc


class NodeDecision:
    __slots__ = ("centroid", "q_old", "q_new", "accept_ge", "accept_gt", "rel_margin")

    def __init__(self, centroid, q_old, q_new):
        self.centroid = centroid
        self.q_old = q_old
        self.q_new = q_new
        self.accept_ge = q_new >= q_old
        self.accept_gt = q_new > q_old
        den = abs(q_old) if q_old != 0 else Fraction(1)
        self.rel_margin = abs(q_new - q_old) / den


def exact_sweep(coords, tris, boundary) -> Dict[int, NodeDecision]:
    """Exact decisions for every free node, reading positions ``coords``."""
    n = len(coords)
    P = [(Fraction(float(x)), Fraction(float(y))) for x, y in coords]
    nbrs, inc = incidence(n, tris)
    out = {}
    for i in range(n):
        if boundary[i]:
            continue
        nb = sorted(nbrs[i])
        cx = sum(P[j][0] for j in nb) / len(nb)
        cy = sum(P[j][1] for j in nb) / len(nb)
        q_old = None
        q_new = None
        for t in inc[i]:
            tri = [int(v) for v in tris[t]]
            old = [P[v] for v in tri]
            new = [(cx, cy) if v == i else P[v] for v in tri]
            a, b = _ratio(*old), _ratio(*new)
            q_old = a if q_old is None or a < q_old else q_old
            q_new = b if q_new is None or b < q_new else q_new
        out[i] = NodeDecision((cx, cy), q_old, q_new)
    return out
