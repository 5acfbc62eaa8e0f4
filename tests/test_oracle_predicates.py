"""Pins for the oracle's exact predicates and fixed-order formulas.

Each predicate is compared with a *different* exact characterisation written
with Python rationals:

* orient2d  -> signed shoelace area of the triangle;
* incircle  -> compare the squared distance from the exact circumcenter
               (solved from the perpendicular-bisector equations) with the
               squared circumradius;
* indiametral -> compare the distance to the segment midpoint with half the
               segment length;
* incircle with symbolic perturbation -> the 4x4 lifted determinant with an
               explicit tiny perturbation eps^(id+1).
"""
import math
import random
from fractions import Fraction as F

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def fr(p):
    return (F(p[0]), F(p[1]))


def sgn(x):
    return (x > 0) - (x < 0)


def shoelace(a, b, c):
    a, b, c = fr(a), fr(b), fr(c)
    return sgn(a[0] * b[1] - b[0] * a[1] + b[0] * c[1] - c[0] * b[1] + c[0] * a[1] - a[0] * c[1])


def exact_circumcenter(a, b, c):
    a, b, c = fr(a), fr(b), fr(c)
    # |X-a|^2 = |X-b|^2 and |X-a|^2 = |X-c|^2  ->  2(b-a).X = |b|^2-|a|^2 ...
    a11, a12 = 2 * (b[0] - a[0]), 2 * (b[1] - a[1])
    a21, a22 = 2 * (c[0] - a[0]), 2 * (c[1] - a[1])
    r1 = b[0] ** 2 + b[1] ** 2 - a[0] ** 2 - a[1] ** 2
    r2 = c[0] ** 2 + c[1] ** 2 - a[0] ** 2 - a[1] ** 2
    det = a11 * a22 - a12 * a21
    x = (r1 * a22 - a12 * r2) / det
    y = (a11 * r2 - r1 * a21) / det
    return x, y


def incircle_geo(a, b, c, d):
    """+1 if d strictly inside circumcircle of CCW triangle abc."""
    ox, oy = exact_circumcenter(a, b, c)
    A = fr(a)
    D = fr(d)
    r2 = (A[0] - ox) ** 2 + (A[1] - oy) ** 2
    d2 = (D[0] - ox) ** 2 + (D[1] - oy) ** 2
    return sgn(r2 - d2)


def indiam_geo(a, b, c):
    A, B, Cc = fr(a), fr(b), fr(c)
    mx, my = (A[0] + B[0]) / 2, (A[1] + B[1]) / 2
    r2 = ((B[0] - A[0]) ** 2 + (B[1] - A[1]) ** 2) / 4
    d2 = (Cc[0] - mx) ** 2 + (Cc[1] - my) ** 2
    return sgn(r2 - d2)


def _cases(seed, n):
    rnd = random.Random(seed)
    out = []
    for _ in range(n):
        kind = rnd.randrange(5)
        if kind == 0:  # uniform
            pts = [(rnd.random(), rnd.random()) for _ in range(4)]
        elif kind == 1:  # small integer grid (many exact zeros)
            pts = [(rnd.randrange(4) / 4, rnd.randrange(4) / 4) for _ in range(4)]
        elif kind == 2:  # nearly collinear: rounded points on a line
            t = [rnd.random() for _ in range(4)]
            x0, y0, dx, dy = rnd.random(), rnd.random(), rnd.random(), rnd.random() * 1e-3
            pts = [(x0 + ti * dx, y0 + ti * dy) for ti in t]
        elif kind == 3:  # rounded cocircular points
            cx, cy, r = rnd.random(), rnd.random(), rnd.random() * 0.3 + 1e-3
            ang = sorted(rnd.random() * 2 * math.pi for _ in range(4))
            pts = [(cx + r * math.cos(t), cy + r * math.sin(t)) for t in ang]
        else:  # tiny offsets near degeneracy
            base = (rnd.random(), rnd.random())
            pts = [(base[0] + rnd.randrange(-3, 4) * 2.0 ** -50, base[1] + rnd.randrange(-3, 4) * 2.0 ** -50)
                   for _ in range(4)]
        out.append(pts)
    return out


def test_orient2d_matches_shoelace(orc):
    for pts in _cases(1, 3000):
        a, b, c = pts[:3]
        assert orc.orient2d(a, b, c) == shoelace(a, b, c), (a, b, c)


def test_incircle_matches_circumcenter_distance(orc):
    n = 0
    for pts in _cases(2, 3000):
        a, b, c, d = pts
        o = shoelace(a, b, c)
        if o == 0:
            continue
        if o < 0:
            b, c = c, b
        assert orc.incircle(a, b, c, d) == incircle_geo(a, b, c, d), (a, b, c, d)
        n += 1
    assert n > 1500


def test_indiametral_matches_midpoint_distance(orc):
    for pts in _cases(3, 3000):
        a, b, c = pts[:3]
        if a == b:
            continue
        assert orc.indiametral(a, b, c) == indiam_geo(a, b, c), (a, b, c)


def test_exact_cocircular_integer_points(orc):
    # Pythagorean points on the circle of radius 5 (scaled by 2^-10, exact in FP64)
    s = 2.0 ** -10
    P = [(5 * s, 0.0), (3 * s, 4 * s), (0.0, 5 * s), (-4 * s, 3 * s), (-5 * s, 0.0), (4 * s, -3 * s)]
    for i in range(len(P)):
        for j in range(len(P)):
            for k in range(len(P)):
                for l in range(len(P)):
                    if len({i, j, k, l}) < 4:
                        continue
                    a, b, c = P[i], P[j], P[k]
                    if shoelace(a, b, c) <= 0:
                        continue
                    assert orc.incircle(a, b, c, P[l]) == 0
    assert orc.incircle(P[0], P[1], P[2], (0.0, 0.0)) == 1
    assert orc.incircle(P[0], P[1], P[2], (6 * s, 0.0)) == -1


def lifted_det_eps(pts, ids, eps):
    rows = []
    for (x, y), i in zip(pts, ids):
        X, Y = F(x), F(y)
        rows.append([X, Y, X * X + Y * Y + eps ** (i + 1), F(1)])

    def det(m):
        if len(m) == 1:
            return m[0][0]
        s = F(0)
        for j in range(len(m)):
            minor = [r[:j] + r[j + 1:] for r in m[1:]]
            s += (-1) ** j * m[0][j] * det(minor)
        return s
    return sgn(det(rows))


def test_incircle_sos_matches_explicit_perturbation(orc):
    s = 2.0 ** -10
    P = [(5 * s, 0.0), (3 * s, 4 * s), (0.0, 5 * s), (-4 * s, 3 * s), (-5 * s, 0.0), (4 * s, -3 * s),
         (0.0, 0.0), (2 * s, 0.0)]
    eps = F(1, 2 ** 200)
    rnd = random.Random(7)
    n = 0
    for _ in range(400):
        q = rnd.sample(range(len(P)), 4)
        a, b, c, d = (P[i] for i in q)
        if shoelace(a, b, c) <= 0:
            continue
        ids = rnd.sample(range(6), 4)
        got = orc.incircle_sos(a, b, c, d, *ids)
        want = lifted_det_eps([a, b, c, d], ids, eps)
        assert got == want, (q, ids)
        assert got != 0
        n += 1
    assert n > 100


def test_perm32_is_a_bijection_with_explicit_inverse(orc):
    # inverse of the xor-shift / odd-multiply rounds, written independently
    def inv_xorshift(h, s):
        x = h
        for _ in range(32 // s + 1):
            x = h ^ (x >> s)
        return x & 0xFFFFFFFF

    def inv(h):
        h = inv_xorshift(h, 16)
        h = (h * pow(0xc2b2ae35, -1, 1 << 32)) & 0xFFFFFFFF
        h = inv_xorshift(h, 13)
        h = (h * pow(0x85ebca6b, -1, 1 << 32)) & 0xFFFFFFFF
        h = inv_xorshift(h, 16)
        return (h - 1) & 0xFFFFFFFF

    rnd = random.Random(3)
    vals = [0, 1, 2, 3, 1000, 2 ** 31 - 1] + [rnd.randrange(2 ** 31) for _ in range(2000)]
    outs = set()
    for v in vals:
        h = orc.perm32(v)
        assert h != 0
        assert inv(h) == v
        outs.add(h)
    assert len(outs) == len(set(vals))


def test_midpoint_is_correctly_rounded(orc):
    import workloads
    p = workloads.random_small(11, 40, 6)
    m = orc.build_cdt(p.xy, p.seg)
    orc.refine(m, 2.0)
    a = m.arrays()
    xy = a["xy"]
    nin = p.n_vertices
    checked = 0
    for v in range(nin, m.nV):
        if a["vkind"][v] != 1:
            continue
        # the midpoint's subsegment neighbours: find the two subsegments meeting at v with one parent
        ks = np.nonzero((a["sv"][:, 0] == v) | (a["sv"][:, 1] == v))[0]
        assert len(ks) == 2
        # endpoints of the split subsegment at the time of the split are unknown here; check
        # instead that v lies within rounding of the parent segment's line
        par = a["sparent"][ks[0]]
        s0, s1 = p.seg[par]
        A, B, V = fr(p.xy[s0]), fr(p.xy[s1]), fr(xy[v])
        cross = (B[0] - A[0]) * (V[1] - A[1]) - (B[1] - A[1]) * (V[0] - A[0])
        L = float(((B[0] - A[0]) ** 2 + (B[1] - A[1]) ** 2)) ** 0.5
        assert abs(float(cross)) / L <= 4 * 2.0 ** -53 * 4, v
        checked += 1
    assert checked > 0
