"""Pins the round oracle's point count against a classic sequential Ruppert.

The round oracle inserts many points per round, with priority marks and a
dependency test deciding which ones go in (Algorithm 1, Lines 2-9; the
marking and dependency rules of Section 5.2).  A sequential refiner inserts
one point at a time from a priority queue (Ruppert's algorithm with the
encroachment and termination rules of Section 4.2).  Both must satisfy every
post-condition, and they must agree on the number of Steiner points within
10%, the spread the paper reports between its parallel refinement and a
sequential refiner on the same inputs (Table 1: 0.96-1.10 times Triangle's
output points).  The sequential refiner shares only the exact predicates and
the initial CDT with the round oracle, so a dropped or mis-ordered rule in
the round (a lost insertion, a wrong conflict or encroachment decision)
shows up as a count outside the band or as a failed post-condition.
"""
import numpy as np
import pytest

import workloads

BOUNDS = [2.0, 1.6 * 1.6, 4.0]


def _post(m, p, B2):
    n, msg = m.check_topology()
    assert n == 0, msg
    assert m.check_local_delaunay() == 0
    # the sequential refiner computes the ratio with its own FP64 formula; a
    # triangle within rounding of the bound may be judged differently
    assert m.check_quality(B2 * (1 + 1e-9)) == 0
    assert m.check_encroached() == 0
    assert abs(m.area() - 1.0) < 1e-12 + m.nT * 4e-16
    n, msg = m.check_subsegments()
    assert n == 0, msg


def _inputs():
    return {
        "c0_1k": lambda: workloads.config0(),
        "c1_100k": lambda: workloads.scaled_config1(100_000, 5_000),
        "c2_32x200": lambda: workloads.scaled_config2(32, 200, 5_000, seed=2),
    }


_cache = {}


def _pslg(name):
    if name not in _cache:
        _cache[name] = _inputs()[name]()
    return _cache[name]


@pytest.mark.parametrize("B2", BOUNDS)
@pytest.mark.parametrize("case", ["c0_1k", "c1_100k", "c2_32x200"])
def test_round_count_within_10pct_of_sequential_ruppert(orc, case, B2):
    p = _pslg(case)
    cdt = orc.build_cdt(p.xy, p.seg)
    seq = cdt.clone()
    orc.refine(cdt, B2)
    r = orc.ruppert(seq, B2)
    assert r["rc"] == 0 and r["n_unsplittable"] == 0
    _post(seq, p, B2)
    n_round = cdt.nV - p.n_vertices
    n_seq = seq.nV - p.n_vertices
    assert n_seq > 0
    assert abs(n_round - n_seq) <= 0.10 * n_seq, (n_round, n_seq)


def test_sequential_ruppert_special_cases(orc):
    """Bare square: two right isosceles triangles (ratio 1/sqrt 2) and no
    encroached side, so nothing is inserted.  A point 1e-3 above the bottom
    side encroaches it: the first insertion is that side's midpoint
    (0.5, 0), vertex 5, and subsegment 0 = (0, 1) becomes (0, 5) + (5, 1)."""
    p = workloads.bare_square()
    m = orc.build_cdt(p.xy, p.seg)
    orc.ruppert(m, 2.0)
    assert (m.nV, m.nT) == (4, 2)
    p = workloads.near_edge_point(1e-3)
    m = orc.build_cdt(p.xy, p.seg)
    r = orc.ruppert(m, 2.0, max_insertions=1)
    a = m.arrays()
    assert r["rc"] == -5 and m.nV == 6
    assert tuple(a["xy"][5]) == (0.5, 0.0) and a["vkind"][5] == 1
    assert tuple(a["sv"][0]) == (0, 5) and tuple(a["sv"][4]) == (5, 1) and a["sparent"][4] == 0


def test_one_candidate_rounds_match_sequential_count(orc):
    """K = 1 lets one scan candidate per round through (plus the subsegments
    it is redirected to): a sequential refinement in key order, so its count
    sits in the same band around the classic sequential refiner's."""
    p = workloads.config0()
    m = orc.build_cdt(p.xy, p.seg)
    seq = m.clone()
    orc.refine(m, 2.0, cand_cap_K=1)
    orc.ruppert(seq, 2.0)
    n1, ns = m.nV - p.n_vertices, seq.nV - p.n_vertices
    assert abs(n1 - ns) <= 0.10 * ns, (n1, ns)


def test_sequential_refiner_is_deterministic(orc):
    p = workloads.random_small(71, 400, 20)
    outs = []
    for _ in range(2):
        m = orc.build_cdt(p.xy, p.seg)
        orc.ruppert(m, 2.0)
        outs.append(m.arrays())
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k
