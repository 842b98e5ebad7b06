"""Independent exact references for pinning the oracle (tests only).

Pure-Python rational arithmetic (fractions.Fraction) on tiny inputs:
the incircle determinant with a symbolic perturbation of the lifting, and a
brute-force O(n^4) Delaunay triangulation built from it.  Written from the
definitions (empty circumcircle; Simulation of Simplicity, Edelsbrunner and
Mücke 1990), sharing nothing with the oracle's C code, which uses a
different formulation (per-cell half-plane cuts with a 3x3 determinant).
"""
from fractions import Fraction as F
from itertools import combinations


def orient(a, b, c):
    return (F(b[0]) - F(a[0])) * (F(c[1]) - F(a[1])) - (F(b[1]) - F(a[1])) * (F(c[0]) - F(a[0]))


def incircle_sos(pts, ia, ib, ic, idd):
    """Sign of 'd inside circle(a, b, c)' for CCW (a, b, c) under the lifting
    z_m = |p_m|^2 - eps_m with eps decreasing in id (smaller id dominates)."""
    d = pts[idd]
    rows = []
    for i in (ia, ib, ic):
        ax = F(pts[i][0]) - F(d[0])
        ay = F(pts[i][1]) - F(d[1])
        rows.append((ax, ay, ax * ax + ay * ay))
    (ax, ay, az), (bx, by, bz), (cx, cy, cz) = rows
    Ma = bx * cy - by * cx
    Mb = -(ax * cy - ay * cx)
    Mc = ax * by - ay * bx
    det = az * Ma + bz * Mb + cz * Mc
    if det != 0:
        return 1 if det > 0 else -1
    # d det / d eps: lifted entry of row m is |.|^2 - eps_m + eps_d
    coef = {ia: -Ma, ib: -Mb, ic: -Mc, idd: Ma + Mb + Mc}
    for i in sorted(coef):
        if coef[i] != 0:
            return 1 if coef[i] > 0 else -1
    return 0


def delaunay_brute(pts):
    """All Delaunay triangles (sorted id triples) of the perturbed point set."""
    n = len(pts)
    out = set()
    for i, j, k in combinations(range(n), 3):
        o = orient(pts[i], pts[j], pts[k])
        if o == 0:
            continue
        a, b, c = (i, j, k) if o > 0 else (i, k, j)
        if all(incircle_sos(pts, a, b, c, l) < 0 for l in range(n) if l not in (i, j, k)):
            out.add((i, j, k))
    return out


def margin_sign(rows, p):
    """Sign of n3 . v - s3 where v solves rows 1, 2 exactly; rows are
    (nx, ny, s) in p-relative coordinates, given as Fractions."""
    (n1x, n1y, s1), (n2x, n2y, s2), (n3x, n3y, s3) = rows
    det = n1x * n2y - n1y * n2x
    vx = (s1 * n2y - s2 * n1y) / det
    vy = (n1x * s2 - n2x * s1) / det
    m = n3x * vx + n3y * vy - s3
    return (m > 0) - (m < 0)


def circumcentre(pts, tri):
    a, b, c = (tuple(map(F, pts[i])) for i in tri)
    bx, by = b[0] - a[0], b[1] - a[1]
    cx, cy = c[0] - a[0], c[1] - a[1]
    d = 2 * (bx * cy - by * cx)
    ux = (cy * (bx * bx + by * by) - by * (cx * cx + cy * cy)) / d
    uy = (bx * (cx * cx + cy * cy) - cx * (bx * bx + by * by)) / d
    return a[0] + ux, a[1] + uy


def circumcentre_inside(pts, tri, box):
    x, y = circumcentre(pts, tri)
    return F(box[0]) < x < F(box[2]) and F(box[1]) < y < F(box[3])
