"""Pins for the oracle's quality criteria beyond the radius-edge bound
(Section 4.1: a bad triangle has an angle below theta or an edge longer than
l; a subsegment is encroached by a point in its diametric circle under
Ruppert's algorithm or in its diametric lens under Chew's) and for the
bad-area measure reported in Table 1.

The lens is the region from which a subsegment is seen under more than 120
degrees (two circular arcs through its endpoints meeting it at 60 degrees).
Its test is pinned against exact rational arithmetic and constructed angles;
the refined meshes are checked with independent numpy / rational code.
"""
import math
import random
from fractions import Fraction as F

import numpy as np
import pytest

import workloads


def lens_exact(a, b, p):
    a, b, p = [(F(float(x)), F(float(y))) for x, y in (a, b, p)]
    dax, day = a[0] - p[0], a[1] - p[1]
    dbx, dby = b[0] - p[0], b[1] - p[1]
    dot = dax * dbx + day * dby
    la, lb = dax * dax + day * day, dbx * dbx + dby * dby
    return dot < 0 and 4 * dot * dot > la * lb, (4 * dot * dot - la * lb), la * lb


def circle_exact(a, b, p):
    a, b, p = [(F(float(x)), F(float(y))) for x, y in (a, b, p)]
    return (a[0] - p[0]) * (b[0] - p[0]) + (a[1] - p[1]) * (b[1] - p[1]) < 0


def test_lens_constructed_angles():
    import oracle
    a, b = (-1.0, 0.0), (1.0, 0.0)
    t30 = math.tan(math.radians(30.0))  # apex height at which ab is seen under 120 degrees
    assert oracle.encroaches(1, a, b, (0.0, t30 * 0.999)) == 1
    assert oracle.encroaches(1, a, b, (0.0, -t30 * 0.999)) == 1
    assert oracle.encroaches(1, a, b, (0.0, t30 * 1.001)) == 0
    # 106.3 degrees: inside the circle, outside the lens
    assert oracle.encroaches(0, a, b, (0.0, 0.75)) == 1
    assert oracle.encroaches(1, a, b, (0.0, 0.75)) == 0
    # on the segment (180 degrees) and on the circle (90 degrees, not strictly inside)
    assert oracle.encroaches(1, a, b, (0.3, 0.0)) == 1
    assert oracle.encroaches(0, a, b, (0.0, 1.0)) == 0
    # off-centre point near the lens boundary: the arc through a and b with
    # centre (0, -1/sqrt(3)) and radius 2/sqrt(3)
    x = 0.6
    y = math.sqrt(4.0 / 3.0 - x * x) - 1.0 / math.sqrt(3.0)
    assert oracle.encroaches(1, a, b, (x, y * 0.99)) == 1
    assert oracle.encroaches(1, a, b, (x, y * 1.01)) == 0


def test_lens_random_vs_rational():
    import oracle
    rng = random.Random(7)
    checked = 0
    for _ in range(4000):
        a = (rng.uniform(0, 1), rng.uniform(0, 1))
        b = (rng.uniform(0, 1), rng.uniform(0, 1))
        mx, my = (a[0] + b[0]) / 2, (a[1] + b[1]) / 2
        h = math.hypot(b[0] - a[0], b[1] - a[1])
        p = (mx + rng.uniform(-0.6, 0.6) * h, my + rng.uniform(-0.3, 0.3) * h)
        inside, margin, scale = lens_exact(a, b, p)
        c0, c1 = oracle.encroaches(0, a, b, p), oracle.encroaches(1, a, b, p)
        assert c0 == int(circle_exact(a, b, p))
        assert c1 <= c0  # the lens lies inside the circle
        if scale == 0 or abs(margin) <= scale * F(1, 10**9):
            continue  # within FP64 rounding of the lens boundary
        assert c1 == int(inside), (a, b, p)
        checked += 1
    assert checked > 3500


def _edges_sq(xy, tv):
    p = xy[tv]  # (T, 3, 2)
    d = p - np.roll(p, -1, axis=1)
    return (d * d).sum(axis=2)


def _lens_violations(arr):
    """Apexes inside the lens of the subsegment opposite them, in rational arithmetic."""
    xy, tv, ts = arr["xy"], arr["tv"], arr["ts"]
    bad = 0
    for t in range(tv.shape[0]):
        for i in range(3):
            if ts[t, i] < 0:
                continue
            a, b, c = xy[tv[t, i]], xy[tv[t, (i + 1) % 3]], xy[tv[t, (i + 2) % 3]]
            bad += circle_exact(a, b, c) and lens_exact(a, b, c)[0]
    return bad


def test_length_criterion_c0():
    import oracle
    p = workloads.config0()
    L2 = 0.004
    m0 = oracle.build_cdt(p.xy, p.seg)
    assert oracle.refine(m0, p.ratio_bound_sq) == 0
    m = oracle.build_cdt(p.xy, p.seg)
    assert oracle.refine(m, p.ratio_bound_sq, max_edge_len_sq=L2) == 0
    arr = m.arrays()
    e2 = _edges_sq(arr["xy"], arr["tv"])
    assert e2.max() <= L2  # no edge longer than l
    assert m.check_quality(p.ratio_bound_sq) == 0
    assert m.check_quality(p.ratio_bound_sq, L2) == 0
    assert m.check_local_delaunay() == 0
    assert m.check_encroached() == 0
    assert m.check_topology()[0] == 0
    assert abs(m.area() - 1.0) < 1e-12
    assert m.nV > m0.nV  # the length bound only adds splits here
    # the length bound alone, with the angle bound out of reach
    m2 = oracle.build_cdt(p.xy, p.seg)
    assert oracle.refine(m2, 1e6, max_edge_len_sq=0.01) == 0
    assert _edges_sq(m2.arrays()["xy"], m2.arrays()["tv"]).max() <= 0.01


@pytest.mark.parametrize("name", ["c0", "rand_300"])
def test_chew_lens_mode(name):
    import oracle
    p = workloads.config0() if name == "c0" else workloads.random_small(32, 300, 20)
    m = oracle.build_cdt(p.xy, p.seg)
    assert oracle.refine(m, p.ratio_bound_sq, encroach_mode=1) == 0
    assert m.check_topology()[0] == 0
    assert m.check_local_delaunay() == 0
    assert m.check_quality(p.ratio_bound_sq) == 0
    assert m.check_encroached(1) == 0
    assert _lens_violations(m.arrays()) == 0
    assert abs(m.area() - 1.0) < 1e-12
    r = oracle.build_cdt(p.xy, p.seg)
    assert oracle.refine(r, p.ratio_bound_sq) == 0
    # a smaller encroachment region splits no more subsegments than the circle
    nk = lambda mm: int((mm.arrays()["vkind"] == 1).sum())
    assert nk(m) <= nk(r)


def test_bad_area_bare_square():
    import oracle
    p = workloads.bare_square()
    m = oracle.build_cdt(p.xy, p.seg)
    # two right isosceles triangles, legs 1: (R / l_min)^2 = 1/2, longest edge^2 = 2
    assert m.quality(0.49) == (2, 1.0)
    assert m.quality(0.5) == (0, 0.0)
    assert m.quality(2.0, 1.5) == (2, 1.0)
    assert m.quality(2.0, 2.0) == (0, 0.0)


def test_bad_area_refined():
    import oracle
    p = workloads.config0()
    m = oracle.build_cdt(p.xy, p.seg)
    assert oracle.refine(m, p.ratio_bound_sq) == 0
    assert m.quality(p.ratio_bound_sq) == (0, 0.0)
    # a stricter bound after the fact: compare with R = abc / (4K) in numpy
    B2 = 1.2
    arr = m.arrays()
    q = arr["xy"][arr["tv"]]
    e2 = _edges_sq(arr["xy"], arr["tv"])
    area = 0.5 * ((q[:, 1, 0] - q[:, 0, 0]) * (q[:, 2, 1] - q[:, 0, 1])
                  - (q[:, 1, 1] - q[:, 0, 1]) * (q[:, 2, 0] - q[:, 0, 0]))
    R2 = e2.prod(axis=1) / (16.0 * area * area)
    ratio = R2 / e2.min(axis=1)
    sure = np.abs(ratio / B2 - 1.0) > 1e-9
    n, a = m.quality(B2)
    bad = ratio > B2
    assert n >= int((bad & sure).sum()) and n <= int((bad | ~sure).sum())
    if (~sure).sum() == 0:
        assert n == int(bad.sum())
        assert abs(a - area[bad].sum()) <= 1e-12 * max(1.0, abs(a))
    assert n > 0 and 0.0 < a < 1.0


def spider(deg, n_spokes=4):
    p = workloads.spokes(deg, n_spokes)
    return p.xy, p.seg


def test_concentric_shell_points():
    """Concentric shells: a subsegment with exactly one input endpoint c is cut
    at distance 2^j from c, 2^j the power of two nearest to half its length;
    other subsegments at their midpoint."""
    import oracle
    xy, seg = spider(30)
    m = oracle.build_cdt(xy, seg)
    assert oracle.refine(m, 2.0, max_rounds=4, raise_on_error=False) == -5  # stopped with work left
    arr = m.arrays()
    vk, sv, pxy = arr["vkind"], arr["sv"], arr["xy"]
    n_shell = 0
    for k in range(sv.shape[0]):
        a, b = sv[k]
        x, y, _ = m.split_point(k, 1)
        xm, ym, _ = m.split_point(k, 0)
        assert (xm, ym) == ((pxy[a, 0] + pxy[b, 0]) * 0.5, (pxy[a, 1] + pxy[b, 1]) * 0.5)
        if (vk[a] == 0) == (vk[b] == 0):
            assert (x, y) == (xm, ym)
            continue
        c, o = (a, b) if vk[a] == 0 else (b, a)
        C_, O_, P_ = [(F(float(q[0])), F(float(q[1]))) for q in (pxy[c], pxy[o], (x, y))]
        L2 = (O_[0] - C_[0]) ** 2 + (O_[1] - C_[1]) ** 2
        D2 = (P_[0] - C_[0]) ** 2 + (P_[1] - C_[1]) ** 2
        half = math.sqrt(float(L2)) / 2
        j = round(math.log2(float(D2)) / 2)
        assert abs(float(D2) / 4.0 ** j - 1.0) < 1e-14  # distance 2^j up to rounding
        # nearest power of two to len/2 (ties and near-ties excluded by the draw)
        lo = 2.0 ** math.floor(math.log2(half))
        want = 2 * lo if (2 * lo - half) < (half - lo) else lo
        assert 2.0 ** j == want
        # on the subsegment, strictly inside
        cross = (O_[0] - C_[0]) * (P_[1] - C_[1]) - (O_[1] - C_[1]) * (P_[0] - C_[0])
        assert abs(float(cross)) <= 1e-15 * math.sqrt(float(L2))  # within a few ulp of the line
        assert 0 < float(D2) < float(L2)
        n_shell += 1
    assert n_shell > 0


@pytest.mark.parametrize("deg", [30, 60])
@pytest.mark.parametrize("split_mode", [0, 1])
def test_small_angle_inputs(deg, split_mode):
    """Spokes 30 and 60 degrees apart: both splitting rules terminate with a
    valid mesh and no bad triangle at B = sqrt(2)."""
    import oracle
    xy, seg = spider(deg, n_spokes=4 if deg == 30 else 3)
    m = oracle.build_cdt(xy, seg)
    assert oracle.refine(m, 2.0, split_mode=split_mode) == 0
    assert m.check_topology()[0] == 0
    assert m.check_local_delaunay() == 0
    assert m.check_quality(2.0) == 0
    assert m.check_encroached() == 0
    assert m.quality(2.0) == (0, 0.0)
    assert abs(m.area() - 1.0) < 1e-12


def test_shells_c0():
    import oracle
    p = workloads.config0()
    m = oracle.build_cdt(p.xy, p.seg)
    assert oracle.refine(m, p.ratio_bound_sq, split_mode=1) == 0
    assert m.check_topology()[0] == 0
    assert m.check_local_delaunay() == 0
    assert m.check_quality(p.ratio_bound_sq) == 0
    assert m.check_encroached() == 0
    assert abs(m.area() - 1.0) < 1e-12
