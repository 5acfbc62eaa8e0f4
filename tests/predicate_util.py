"""Query sets for the predicate tests: the seeded corpus of workloads with
the oracle's answers (the oracle's exact signs are pinned separately against
rational arithmetic)."""
from __future__ import annotations

import numpy as np


def corpus_with_oracle(seed: int = 5, n_per_family: int = 1500):
    """{kind: (queries, oracle signs, family)} for the four predicate kinds;
    incircle queries have their first three points in counter-clockwise
    order (by the oracle's orient2d)."""
    import oracle
    import workloads
    Q, fam = workloads.predicate_corpus(seed, n_per_family)
    inc = []
    for q in Q:
        a, b, c, d = q
        if oracle.orient2d(a, b, c) < 0:
            b, c = c, b
        inc.append(np.concatenate([a, b, c, d]))
    inc = np.asarray(inc)
    tri = np.ascontiguousarray(Q[:, :3, :].reshape(-1, 6))
    out = {
        "incircle": (inc, np.array([oracle.incircle(r[0:2], r[2:4], r[4:6], r[6:8]) for r in inc]), fam),
        "orient2d": (tri, np.array([oracle.orient2d(r[0:2], r[2:4], r[4:6]) for r in tri]), fam),
        "indiametral": (tri, np.array([oracle.indiametral(r[0:2], r[2:4], r[4:6]) for r in tri]), fam),
        "lens": (tri, np.array([oracle.encroaches(1, r[0:2], r[2:4], r[4:6]) for r in tri]), fam),
    }
    return out
