"""Pins for the oracle's initial CDT and its refinement rounds.

The initial CDT is compared with a brute-force enumeration of constrained
Delaunay triangles on tiny inputs (rational arithmetic, general position).
The refined meshes are checked against what the paper fixes for the output:
a triangulation of the square that contains every input vertex and segment
(Section 4), constrained Delaunay, no triangle above the radius-edge bound,
no encroached subsegment (Ruppert mode), plus Euler's relation and the total
area.  Hand-checkable special cases pin individual rules of a round.
"""
import itertools
import random
from fractions import Fraction as F

import numpy as np
import pytest

import workloads


def fr(p):
    return (F(float(p[0])), F(float(p[1])))


def orient(a, b, c):
    v = (a[0] - c[0]) * (b[1] - c[1]) - (a[1] - c[1]) * (b[0] - c[0])
    return (v > 0) - (v < 0)


def proper_cross(p, q, a, b):
    return orient(p, q, a) * orient(p, q, b) < 0 and orient(a, b, p) * orient(a, b, q) < 0


def in_circle(a, b, c, d):
    rows = [(x[0] - d[0], x[1] - d[1]) for x in (a, b, c)]
    m = [(dx, dy, dx * dx + dy * dy) for dx, dy in rows]
    det = (m[0][0] * (m[1][1] * m[2][2] - m[2][1] * m[1][2])
           - m[0][1] * (m[1][0] * m[2][2] - m[2][0] * m[1][2])
           + m[0][2] * (m[1][0] * m[2][1] - m[2][0] * m[1][1]))
    return (det > 0) - (det < 0)


def brute_cdt(xy, seg):
    P = [fr(p) for p in xy]
    S = [tuple(s) for s in seg.tolist()]
    n = len(P)
    tris = set()
    for i, j, k in itertools.combinations(range(n), 3):
        o = orient(P[i], P[j], P[k])
        if o == 0:
            continue
        a, b, c = (i, j, k) if o > 0 else (i, k, j)
        A, B, Cc = P[a], P[b], P[c]
        # no vertex inside the closed triangle
        if any(v not in (a, b, c) and orient(A, B, P[v]) >= 0 and orient(B, Cc, P[v]) >= 0
               and orient(Cc, A, P[v]) >= 0 for v in range(n)):
            continue
        # no triangle edge crosses a segment
        edges = ((a, b), (b, c), (c, a))
        if any(proper_cross(P[u], P[w], P[s0], P[s1]) for (u, w) in edges for (s0, s1) in S
               if len({u, w, s0, s1}) == 4):
            continue
        # sample points of the open triangle
        g = ((A[0] + B[0] + Cc[0]) / 3, (A[1] + B[1] + Cc[1]) / 3)
        samples = [g]
        for lam in (F(1, 2), F(9, 10), F(99, 100)):
            for V in (A, B, Cc):
                samples.append((g[0] + lam * (V[0] - g[0]), g[1] + lam * (V[1] - g[1])))
            for (U, W) in ((A, B), (B, Cc), (Cc, A)):
                mid = ((U[0] + W[0]) / 2, (U[1] + W[1]) / 2)
                samples.append((g[0] + lam * (mid[0] - g[0]), g[1] + lam * (mid[1] - g[1])))
        ok = True
        for v in range(n):
            if v in (a, b, c) or in_circle(A, B, Cc, P[v]) <= 0:
                continue
            for s in samples:
                if not any(proper_cross(P[v], s, P[s0], P[s1]) for (s0, s1) in S if v not in (s0, s1)):
                    ok = False
                    break
            if not ok:
                break
        if ok:
            r = min(range(3), key=lambda q: (a, b, c)[q])
            t = (a, b, c)[r:] + (a, b, c)[:r]
            tris.add(t)
    return tris


@pytest.mark.parametrize("seed", range(8))
def test_initial_cdt_matches_bruteforce(orc, seed):
    rnd = random.Random(100 + seed)
    n_pts = rnd.randrange(4, 10)
    p = workloads.random_small(200 + seed, n_pts, rnd.randrange(0, 3))
    m = orc.build_cdt(p.xy, p.seg)
    got = {tuple(t) for t in m.arrays()["tv"].tolist()}
    want = brute_cdt(p.xy, p.seg)
    assert got == want
    assert m.check_topology()[0] == 0


def test_initial_cdt_is_canonical(orc):
    p = workloads.config0()
    m = orc.build_cdt(p.xy, p.seg)
    tv = m.arrays()["tv"]
    assert (tv[:, 0] < tv[:, 1]).all() and (tv[:, 0] < tv[:, 2]).all()
    keys = [tuple(t) for t in tv.tolist()]
    assert keys == sorted(keys)
    assert m.check_local_delaunay() == 0
    assert m.check_cdt_bruteforce() == 0


def test_bare_square(orc):
    """Four cocircular corners: the perturbation (smallest id dominant) puts
    vertex 3 inside circle(0,1,2), so the diagonal is (1,3): triangles
    (0,1,3) and (1,2,3).  Both are right isosceles with radius-edge ratio
    1/sqrt(2) < sqrt(2), and no apex is inside a side's diametric circle, so
    refinement inserts nothing."""
    p = workloads.bare_square()
    m = orc.build_cdt(p.xy, p.seg)
    assert {tuple(t) for t in m.arrays()["tv"].tolist()} == {(0, 1, 3), (1, 2, 3)}
    orc.refine(m, 2.0)
    assert (m.nV, m.nT, m.rounds) == (4, 2, 0)


def test_point_near_bottom_edge_splits_it_first(orc):
    """A point at height 1e-3 over the bottom side lies inside that side's
    diametric circle, so round 1 splits subsegment 0 = (0,1) at its midpoint,
    which becomes the first new vertex (id 5)."""
    p = workloads.near_edge_point(1e-3)
    m = orc.build_cdt(p.xy, p.seg)
    rc = orc.refine(m, 2.0, max_rounds=1)
    a = m.arrays()
    assert m.rounds == 1 and rc == -5
    assert tuple(a["xy"][5]) == (0.5, 0.0)
    assert a["vkind"][5] == 1
    assert tuple(a["sv"][0]) == (0, 5)
    assert tuple(a["sv"][4]) == (5, 1) and a["sparent"][4] == 0


def _full_checks(m, B2, brute=False):
    n, msg = m.check_topology()
    assert n == 0, msg
    assert m.check_local_delaunay() == 0
    assert m.check_quality(B2) == 0
    assert m.check_encroached() == 0
    assert abs(m.area() - 1.0) < 1e-12 + m.nT * 4e-16
    n, msg = m.check_subsegments()
    assert n == 0, msg
    if brute:
        assert m.check_cdt_bruteforce() == 0


@pytest.mark.parametrize("case", ["c0", "rand_small_a", "rand_small_b", "knn_small", "circles_small"])
def test_refined_mesh_postconditions(orc, case):
    p = {
        "c0": lambda: workloads.config0(),
        "rand_small_a": lambda: workloads.random_small(31, 60, 5),
        "rand_small_b": lambda: workloads.random_small(32, 300, 20),
        "knn_small": lambda: workloads.random_small(33, 2000, 100, pairing="knn"),
        "circles_small": lambda: workloads.scaled_config2(6, 40, 100, seed=5),
    }[case]()
    m = orc.build_cdt(p.xy, p.seg)
    orc.refine(m, p.ratio_bound_sq)
    assert m.nV > p.n_vertices or case == "none"
    _full_checks(m, p.ratio_bound_sq, brute=m.nV < 5000)
    # every round inserts at least one point and vertex ids are dense
    assert all(s["n_ins_mid"] + s["n_ins_cc"] > 0 for s in m.stats)
    assert sum(s["n_ins_mid"] + s["n_ins_cc"] for s in m.stats) == m.nV - p.n_vertices


@pytest.mark.parametrize("B2", [2.0, 1.6 * 1.6, 4.0])
def test_other_bounds(orc, B2):
    p = workloads.random_small(41, 400, 20)
    m = orc.build_cdt(p.xy, p.seg)
    orc.refine(m, B2)
    _full_checks(m, B2)


def test_deterministic_and_resumable(orc):
    p = workloads.random_small(51, 500, 30)
    m1 = orc.build_cdt(p.xy, p.seg)
    orc.refine(m1, 2.0)
    m2 = orc.build_cdt(p.xy, p.seg)
    rc = orc.refine(m2, 2.0, max_rounds=5)
    assert rc == -5 and m2.rounds == 5
    orc.refine(m2, 2.0)  # resume from the round-5 state
    a1, a2 = m1.arrays(), m2.arrays()
    for k in a1:
        assert np.array_equal(a1[k], a2[k]), k


def test_priority_mode_one(orc):
    p = workloads.random_small(52, 300, 10)
    m = orc.build_cdt(p.xy, p.seg)
    orc.refine(m, 2.0, priority_mode=1)
    _full_checks(m, 2.0)


def test_circumcenter_formula_accuracy(orc):
    """The FP64 circumcenters written into the mesh are within a few ulps
    (relative to the circumradius and the condition of the triangle) of the
    exact rational circumcenter of the triangle they split."""
    from tests.test_oracle_predicates import exact_circumcenter
    p = workloads.random_small(61, 200, 0)
    m = orc.build_cdt(p.xy, p.seg)
    orc.refine(m, 2.0, max_rounds=1)
    a = m.arrays()
    # re-derive round-1 circumcenter winners from the initial mesh
    m0 = orc.build_cdt(p.xy, p.seg)
    t0 = m0.arrays()
    xy0 = t0["xy"]
    new = [v for v in range(p.n_vertices, m.nV) if a["vkind"][v] == 2]
    assert new
    for v in new:
        pv = a["xy"][v]
        best = None
        for tri in t0["tv"]:
            A, B, Cc = xy0[tri[0]], xy0[tri[1]], xy0[tri[2]]
            ox, oy = exact_circumcenter(A, B, Cc)
            d = abs(float(ox) - pv[0]) + abs(float(oy) - pv[1])
            if best is None or d < best[0]:
                r = float((F(A[0]) - ox) ** 2 + (F(A[1]) - oy) ** 2) ** 0.5
                best = (d, r)
        assert best[0] <= 1e-12 * max(best[1], 1.0)


@pytest.mark.parametrize("kind", ["cross", "dup_point", "vertex_on_segment", "hull_uncovered", "repeat_seg"])
def test_invalid_inputs_rejected(orc, kind):
    base = workloads.bare_square()
    xy, seg = base.xy.copy(), base.seg.copy()
    if kind == "cross":
        xy = np.concatenate([xy, [[0.2, 0.2], [0.8, 0.8], [0.2, 0.8], [0.8, 0.2]]])
        seg = np.concatenate([seg, [[4, 5], [6, 7]]])
    elif kind == "dup_point":
        xy = np.concatenate([xy, [[0.3, 0.3], [0.3, 0.3]]])
    elif kind == "vertex_on_segment":
        xy = np.concatenate([xy, [[0.25, 0.25], [0.75, 0.75], [0.5, 0.5]]])
        seg = np.concatenate([seg, [[4, 5]]])
    elif kind == "hull_uncovered":
        seg = seg[:3]
    elif kind == "repeat_seg":
        seg = np.concatenate([seg, [[1, 0]]])
    with pytest.raises(orc.OracleError) as e:
        orc.build_cdt(xy, seg)
    assert e.value.code == -2


@pytest.mark.parametrize("f1,n", [(1, 0), (0, 4), (1, 8)])
def test_prefilters_keep_postconditions(orc, f1, n):
    """The Line 6 / Line 7 filters only drop candidates: the result still
    satisfies every post-condition, and the global maximum key of a round is
    never dropped, so no round stalls."""
    for p in (workloads.config0(), workloads.scaled_config2(6, 40, 100, seed=5)):
        m = orc.build_cdt(p.xy, p.seg)
        orc.refine(m, 2.0, prefilter_f1=f1, cavity_approx_n=n)
        _full_checks(m, 2.0)
        assert all(s["n_ins_mid"] + s["n_ins_cc"] > 0 for s in m.stats)
        if f1:
            assert sum(s["n_f1_drop"] for s in m.stats) > 0
        if n:
            assert sum(s["n_f2_drop"] for s in m.stats) > 0
