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
