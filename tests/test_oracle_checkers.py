"""The oracle's post-condition checkers must be able to fail.

Every parity and oracle test relies on the checkers returning 0 on a good
mesh; these tests plant one defect at a time, on the CPU, in a copy of a
mesh the oracle produced, and show that the checker for that property fires
(and, where the count has an independent exact characterisation, that it
fires exactly as often as rational arithmetic says it should):

* quality (radius-edge ratio above B, Section 5.1 form of the 2D bound) on
  the initial CDT and on a mesh refined for a looser bound;
* encroachment (a vertex strictly inside a subsegment's diametric circle,
  Section 4.2) on the initial CDT;
* local Delaunay and the brute-force constrained-empty-circle test (the CDT
  definition of Section 4) after one edge flip;
* the subsegment union (every segment is a union of subsegments, Section 4)
  after moving one midpoint off its segment;
* topology / Euler after dropping one triangle.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import workloads


def fr(p):
    return (F(float(p[0])), F(float(p[1])))


def orient(a, b, c):
    v = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
    return (v > 0) - (v < 0)


@pytest.fixture(scope="module")
def c0():
    return workloads.config0()


def test_quality_fires_on_initial_cdt_exact_count(orc, c0):
    """The initial CDT of the 1k-point input has many bad triangles.  The
    checker's count must equal the exact count (circumradius^2 > B^2 *
    shortest edge^2 in rationals: R^2 = |ab|^2 |bc|^2 |ca|^2 / (4 cross^2)),
    up to the triangles that lie within 1e-9 relative of the bound."""
    m = orc.build_cdt(c0.xy, c0.seg)
    a = m.arrays()
    B2 = F(2)
    exact = ambiguous = 0
    for tri in a["tv"]:
        A, B, C = (fr(a["xy"][v]) for v in tri)
        d2 = [(P[0] - Q[0]) ** 2 + (P[1] - Q[1]) ** 2 for P, Q in ((A, B), (B, C), (C, A))]
        cross = (B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0])
        R2 = d2[0] * d2[1] * d2[2] / (4 * cross * cross)
        ratio = R2 / (B2 * min(d2))
        if abs(ratio - 1) < F(1, 10 ** 9):
            ambiguous += 1
        elif ratio > 1:
            exact += 1
    got = m.check_quality(2.0)
    assert exact > 100
    assert exact <= got <= exact + ambiguous


def test_quality_fires_on_mesh_refined_for_looser_bound(orc, c0):
    m = orc.build_cdt(c0.xy, c0.seg)
    orc.refine(m, 4.0)
    assert m.check_quality(4.0) == 0
    assert m.check_quality(2.0) > 0


def test_encroached_fires_on_initial_cdt_exact_count(orc, c0):
    """Apexes strictly inside the diametric circle of the subsegment opposite
    them: (a - c).(b - c) < 0 in rationals, counted per triangle side."""
    m = orc.build_cdt(c0.xy, c0.seg)
    a = m.arrays()
    want = 0
    for t in range(m.nT):
        for i in range(3):
            if a["ts"][t, i] < 0:
                continue
            A = fr(a["xy"][a["tv"][t, i]])
            B = fr(a["xy"][a["tv"][t, (i + 1) % 3]])
            C = fr(a["xy"][a["tv"][t, (i + 2) % 3]])
            if (A[0] - C[0]) * (B[0] - C[0]) + (A[1] - C[1]) * (B[1] - C[1]) < 0:
                want += 1
    assert want > 0
    assert m.check_encroached(0) == want
    orc.refine(m, 2.0)
    assert m.check_encroached(0) == 0


def _flip_one_edge(a):
    """Flips the first interior non-subsegment edge whose quadrilateral is
    strictly convex; returns the two triangle slots."""
    xy, tv, tn, ts = a["xy"], a["tv"], a["tn"], a["ts"]
    for t in range(len(tv)):
        for i in range(3):
            n = tn[t, i]
            if n < 0 or ts[t, i] >= 0 or n < t:
                continue
            u, v, w = tv[t, i], tv[t, (i + 1) % 3], tv[t, (i + 2) % 3]
            j = [q for q in range(3) if tv[n, q] == v and tv[n, (q + 1) % 3] == u][0]
            z = tv[n, (j + 2) % 3]
            P = {k: fr(xy[k]) for k in (u, v, w, z)}
            if orient(P[w], P[u], P[z]) <= 0 or orient(P[w], P[z], P[v]) <= 0:
                continue
            # outside neighbours and subsegment ids of the four quad edges
            wu = (tn[t, (i + 2) % 3], ts[t, (i + 2) % 3])
            vw = (tn[t, (i + 1) % 3], ts[t, (i + 1) % 3])
            uz = (tn[n, (j + 1) % 3], ts[n, (j + 1) % 3])
            zv = (tn[n, (j + 2) % 3], ts[n, (j + 2) % 3])
            tv[t] = (w, u, z)
            tn[t] = (wu[0], uz[0], n)
            ts[t] = (wu[1], uz[1], -1)
            tv[n] = (w, z, v)
            tn[n] = (t, zv[0], vw[0])
            ts[n] = (-1, zv[1], vw[1])
            for (o, _), (x, y), new in ((uz, (u, z), t), (vw, (v, w), n)):
                if o >= 0:
                    for q in range(3):
                        if tv[o, q] == y and tv[o, (q + 1) % 3] == x:
                            tn[o, q] = new
            return t, n
    raise AssertionError("no flippable edge")


def test_local_delaunay_and_bruteforce_fire_after_one_flip(orc, c0):
    m = orc.build_cdt(c0.xy, c0.seg)
    orc.refine(m, 2.0)
    assert m.check_local_delaunay() == 0 and m.check_cdt_bruteforce() == 0
    a = m.arrays()
    _flip_one_edge(a)
    bad = orc.mesh_from_arrays(a, m.m.n_input_v, m.m.n_input_s, c0.xy, c0.seg)
    n, msg = bad.check_topology()
    assert n == 0, msg  # still a valid triangulation: only the Delaunay property broke
    assert bad.check_local_delaunay() >= 2  # the flipped edge, seen from both sides
    assert bad.check_cdt_bruteforce() >= 2


def test_subsegment_union_fires_on_displaced_midpoint(orc, c0):
    m = orc.build_cdt(c0.xy, c0.seg)
    orc.refine(m, 2.0)
    a = m.arrays()
    n, msg = m.check_subsegments()
    assert n == 0, msg
    moved = False
    for v in np.nonzero(a["vkind"] == 1)[0]:
        ks = np.nonzero((a["sv"][:, 0] == v) | (a["sv"][:, 1] == v))[0]
        par = a["sparent"][ks[0]]
        s0, s1 = c0.seg[par]
        d = c0.xy[s1] - c0.xy[s0]
        normal = np.array([-d[1], d[0]]) / np.hypot(d[0], d[1])
        trial = {k: v_.copy() for k, v_ in a.items()}
        trial["xy"][v] = a["xy"][v] + 1e-9 * normal
        cand = orc.mesh_from_arrays(trial, m.m.n_input_v, m.m.n_input_s, c0.xy, c0.seg)
        if cand.check_topology()[0] == 0:  # every triangle still CCW
            n, msg = cand.check_subsegments()
            assert n >= 1 and "off the segment" in msg
            moved = True
            break
    assert moved


def test_topology_fires_on_dropped_triangle(orc, c0):
    m = orc.build_cdt(c0.xy, c0.seg)
    orc.refine(m, 2.0)
    a = m.arrays()
    last = m.nT - 1
    a["tv"], a["ts"] = a["tv"][:last], a["ts"][:last]
    tn = a["tn"][:last].copy()
    tn[tn == last] = -1
    a["tn"] = tn
    bad = orc.mesh_from_arrays(a, m.m.n_input_v, m.m.n_input_s, c0.xy, c0.seg)
    n, msg = bad.check_topology()
    assert n >= 1 and msg


def test_midpoint_formula_is_the_rounded_exact_midpoint(orc):
    """A split point of split_mode 0 is ((ax + bx) * 0.5, (ay + by) * 0.5):
    one rounding of the sum, then an exact halving, which is the correctly
    rounded exact midpoint (Python's Fraction -> float conversion rounds
    correctly), checked bitwise on every subsegment of a refined mesh."""
    p = workloads.random_small(12, 300, 30)
    m = orc.build_cdt(p.xy, p.seg)
    orc.refine(m, 2.0, max_rounds=6)
    a = m.arrays()
    for k in range(m.nS):
        s0, s1 = a["sv"][k]
        mx, my, _ = m.split_point(k, 0)
        A, B = fr(a["xy"][s0]), fr(a["xy"][s1])
        assert mx == float((A[0] + B[0]) / 2) and my == float((A[1] + B[1]) / 2), k
