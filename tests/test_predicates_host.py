"""The library's exact predicates, run on the host through the C ABI
(gdp_predicates_eval with no context), against the oracle's exact signs on a
corpus built to reach every stage: floating-point filter, exact orient2d and
diametral dot product, incircle on exact differences (stage B) and on raw
coordinates (stage C).  The device runs the same source; tests/test_gpu_
predicates.py checks it there."""
import numpy as np
import pytest

from tests.predicate_util import corpus_with_oracle


@pytest.fixture(scope="module")
def corpus(orc):
    return corpus_with_oracle()


@pytest.mark.parametrize("kind", ["incircle", "orient2d", "indiametral", "lens"])
def test_host_predicates_equal_oracle(corpus, kind):
    from paper_2007_00324_amd import gdp2d
    q, want, _ = corpus[kind]
    got, counts = gdp2d.gdp_predicates_eval(None, kind, q)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (kind, bad[:5], q[bad[:5]])
    # the corpus holds exact zeros and the exact stages are reached
    if kind == "incircle":
        assert (want == 0).sum() > 100
        assert counts[2] > 100 and counts[3] > 100, counts
    elif kind == "orient2d":
        assert (want == 0).sum() > 100 and counts[0] > 100, counts
    else:
        assert counts[1] > 100, counts


def test_stage_c_taken_only_where_differences_round(corpus):
    """Stage C (raw coordinates) is reached on the large rounded circles,
    whose coordinate differences are not exact; the small circles need only
    stage B."""
    import workloads
    from paper_2007_00324_amd import gdp2d
    q, _, fam = corpus["incircle"]
    names = list(workloads.PREDICATE_FAMILIES)
    _, small = gdp2d.gdp_predicates_eval(None, "incircle", q[fam == names.index("cocircular_small")])
    _, large = gdp2d.gdp_predicates_eval(None, "incircle", q[fam == names.index("cocircular_large")])
    assert small[3] == 0 and small[2] > 0
    assert large[3] > 0


def test_predicates_reject_bad_kind():
    from paper_2007_00324_amd import gdp2d
    lib = gdp2d.load()
    import ctypes as C
    out = np.zeros(1, np.int32)
    pts = np.zeros(8)
    assert lib.gdp_predicates_eval(None, 7, 1, pts.ctypes.data_as(C.POINTER(C.c_double)),
                                   out.ctypes.data_as(C.POINTER(C.c_int32)), None) == -1
