"""Writes stars.json: exact expected values for the star fixtures.

Uses only ``oracle.exact`` (exact rational arithmetic) and a 60-digit decimal
value of 2*sqrt(3).  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys
from decimal import Decimal, getcontext
from fractions import Fraction

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.exact import exact_sweep  # noqa: E402

getcontext().prec = 60
TWO_SQRT3 = Decimal(12).sqrt()

CASES = [
    {
        "name": "square_star",
        "cite": "Sec. 2.1 (Smart Laplacian: centroid, then accept iff incident quality improves); eq. (2)",
        "why": "one free node, centroid of the 4-ring is exactly (0,0); the move raises the worst "
               "incident quality, so it is accepted; the second sweep does not move it",
        "center": [0.3, -0.2],
        "ring": [[1, 0], [0, 1], [-1, 0], [0, -1]],
    },
    {
        "name": "arm_star_inverting",
        "cite": "Sec. 2.1 (plain Laplacian can create inverted elements; Smart rejects the move)",
        "why": "the centroid (-1.75, 0) lies outside the kernel of the star: two candidate triangles "
               "invert, the worst quality drops below the current one, the move is rejected",
        "center": [0.0, 0.0],
        "ring": [[1, -1], [1, 1], [-0.25, 0.25], [-6, 0.25], [-6, -0.25], [-0.25, -0.25]],
    },
    {
        "name": "arm_star_no_inversion",
        "cite": "Sec. 2.1; Sec. 3.3.4 (accept iff the min quality of the incident triangles increases)",
        "why": "the centroid (-5/12, 0) inverts nothing but lowers the worst incident quality: rejected",
        "center": [0.0, 0.0],
        "ring": [[1, -1], [1, 1], [-0.25, 0.25], [-2, 0.25], [-2, -0.25], [-0.25, -0.25]],
    },
]


def frac_s(f: Fraction) -> str:
    return "%d/%d" % (f.numerator, f.denominator)


def dec(f: Fraction) -> str:
    return str(TWO_SQRT3 * Decimal(f.numerator) / Decimal(f.denominator))


def main():
    out = []
    for c in CASES:
        k = len(c["ring"])
        coords = [tuple(c["center"])] + [tuple(p) for p in c["ring"]]
        tris = [[0, 1 + q, 1 + (q + 1) % k] for q in range(k)]
        bnd = [0] + [1] * k
        d = exact_sweep(coords, tris, bnd)[0]
        row = dict(c)
        row.update({
            "tris": tris,
            "centroid": [frac_s(d.centroid[0]), frac_s(d.centroid[1])],
            "ratio_old_min": frac_s(d.q_old),
            "ratio_new_min": frac_s(d.q_new),
            "q_old_min": dec(d.q_old),
            "q_new_min": dec(d.q_new),
            "accept_ge": bool(d.accept_ge),
            "accept_gt": bool(d.accept_gt),
        })
        out.append(row)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stars.json")
    with open(path, "w") as f:
        json.dump({"note": "quality q = 2*sqrt(3)*cr/S with cr twice the signed area and S the sum of "
                           "squared edge lengths; ratio_* are the exact cr/S of the worst incident "
                           "triangle; q_* are 2*sqrt(3)*ratio to 60 digits",
                   "cases": out}, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
