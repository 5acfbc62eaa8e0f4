"""The Flip-Flop steps of the GPU path (gdp_ff_core.h: splits, Lawson flips
with six-triangle claims, redundancy detection, removals by ear clipping of
the link, renumbering and compaction), run sequentially on the host, against
the oracle's Flip-Flop round (the CDT of the old vertices and the kept
points, Section 4.3 Line 8) from the same points S.

The kernels run the same functions with device atomics; a sequential run is
one legal schedule of them, so a wrong step (a missed back pointer, a wrong
ear, a lost flag) shows up here, element by element, before any GPU run."""
import numpy as np
import pytest

import workloads
from tests import ffemu
from tests.test_oracle_ff import canon, same

FF = dict(priority_mode=2, insert_mode=1)


class _Arr:
    def __init__(self, a):
        self._a = a

    def arrays(self):
        return self._a


CASES = {
    "rand_300": lambda: workloads.random_small(31, 300, 20),
    "knn_2000": lambda: workloads.random_small(33, 2000, 100, pairing="knn"),
    "circles": lambda: workloads.scaled_config2(6, 40, 100, seed=5),
    "c0": lambda: workloads.config0(),
    "near_edge": lambda: workloads.near_edge_point(1e-3),
}


@pytest.mark.parametrize("kw", [dict(), dict(cand_cap_K=25), dict(encroach_mode=1), dict(max_edge_len_sq=0.004)])
@pytest.mark.parametrize("case", list(CASES))
def test_ff_steps_match_oracle_round_by_round(orc, case, kw):
    p = CASES[case]()
    m = orc.build_cdt(p.xy, p.seg)
    lib = orc.load()
    rounds = 0
    for r in range(200):
        nxt = m.clone()
        rc = orc.refine(nxt, p.ratio_bound_sq, max_rounds=m.rounds + 1, raise_on_error=False, **FF, **kw)
        assert rc in (0, -5), rc
        if not nxt.stats:
            break
        S = ffemu.last_points(lib)
        res, cnt = ffemu.round_from_points(m.arrays(), p.xy.shape[0], S, enc_mode=kw.get("encroach_mode", 0))
        assert cnt["err"] == 0, cnt
        st = nxt.stats[-1]
        assert same(canon(nxt), canon(_Arr(res))), f"round {r}"
        assert cnt["iters"] == st["n_ff_iters"]
        assert cnt["dep"] == st["n_dep_drop"]
        rounds += 1
        m = nxt
        if rc == 0:
            break
    assert rounds > 0


def test_ff_steps_with_a_short_candidate_list(orc):
    """With room for only a few flip candidates per pass, a pass that overflows
    sends its whole input list to the next pass; the result is unchanged."""
    p = CASES["rand_300"]()
    m = orc.build_cdt(p.xy, p.seg)
    lib = orc.load()
    for r in range(6):
        nxt = m.clone()
        orc.refine(nxt, p.ratio_bound_sq, max_rounds=m.rounds + 1, raise_on_error=False, **FF)
        S = ffemu.last_points(lib)
        res, cnt = ffemu.round_from_points(m.arrays(), p.xy.shape[0], S, cand_cap=5)
        assert cnt["err"] == 0, cnt
        assert same(canon(nxt), canon(_Arr(res))), f"round {r}"
        m = nxt


def _key(tri):
    r = int(np.argmin(tri))
    return tuple(int(tri[(r + i) % 3]) for i in range(3))


@pytest.mark.parametrize("case", ["near_edge", "rand_300", "circles"])
def test_ff_steps_chained_from_their_own_layout(orc, case):
    """Each round starts from the previous emulated round's mesh (triangles in
    the slots the flips and the compaction left them in), as on the GPU; the
    oracle's claims are mapped onto those slots by triangle."""
    p = CASES[case]()
    m = orc.build_cdt(p.xy, p.seg)
    lib = orc.load()
    emu = m.arrays()
    for r in range(200):
        nxt = m.clone()
        rc = orc.refine(nxt, p.ratio_bound_sq, max_rounds=m.rounds + 1, raise_on_error=False, **FF)
        if not nxt.stats:
            break
        S = dict(ffemu.last_points(lib))
        otv, etv, etn = np.asarray(m.arrays()["tv"]), np.asarray(emu["tv"]), np.asarray(emu["tn"])
        slot_of = {_key(etv[t]): t for t in range(etv.shape[0])}
        c0, c1, edge = S["c0"].copy(), S["c1"].copy(), S["edge"].copy()
        for i in range(S["n"]):
            if S["cls"][i] != 0:
                continue
            ot = int(S["c0"][i])
            nt = slot_of[_key(otv[ot])]
            c0[i] = nt
            if S["edge"][i] >= 0:
                oe = int(S["edge"][i])
                u, v = otv[ot, oe], otv[ot, (oe + 1) % 3]
                edge[i] = next(j for j in range(3) if etv[nt, j] == u and etv[nt, (j + 1) % 3] == v)
                c1[i] = etn[nt, edge[i]]
        S["c0"], S["c1"], S["edge"] = c0, c1, edge
        res, cnt = ffemu.round_from_points(emu, p.xy.shape[0], S, order_seed=r + 1)
        assert cnt["err"] == 0, (r, cnt)
        assert same(canon(nxt), canon(_Arr(res))), f"round {r}"
        tv, tn = res["tv"], res["tn"]
        for t in range(tv.shape[0]):
            for e in range(3):
                o = tn[t, e]
                if o >= 0:
                    u, v = tv[t, e], tv[t, (e + 1) % 3]
                    assert any(tv[o, j] == v and tv[o, (j + 1) % 3] == u and tn[o, j] == t for j in range(3))
        emu, m = res, nxt
        if rc == 0:
            break
