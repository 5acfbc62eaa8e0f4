"""Device exact predicates against the oracle's exact signs, element by
element, on the corpus that reaches every stage (filter, exact orient2d and
diametral dot product, incircle on exact differences and on raw
coordinates); the device's stage counters must show each stage taken.  Also
the refinement's own fallback counters and the zero-copy device views."""
import numpy as np
import pytest

import workloads
from tests.parity_util import gpu_run
from tests.predicate_util import corpus_with_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    return gdp2d.Context(0)


@pytest.fixture(scope="module")
def corpus():
    return corpus_with_oracle()


@pytest.mark.parametrize("kind", ["incircle", "orient2d", "indiametral", "lens"])
def test_device_predicates_equal_oracle(ctx, corpus, kind):
    from paper_2007_00324_amd import gdp2d
    print(f"[predicates] device {kind}", flush=True)
    q, want, _ = corpus[kind]
    got, counts = gdp2d.gdp_predicates_eval(ctx, kind, q)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (kind, bad[:5], q[bad[:5]])
    # the same filter runs on the host: the same queries reach the same stages
    _, host_counts = gdp2d.gdp_predicates_eval(None, kind, q)
    assert counts == host_counts
    if kind == "incircle":
        assert counts[2] > 100 and counts[3] > 100, counts
    elif kind == "orient2d":
        assert counts[0] > 100, counts
    else:
        assert counts[1] > 100, counts


def test_refinement_counts_exact_fallbacks(ctx):
    """Rounded cocircular circle vertices drive the refinement's incircle
    tests into both exact stages; the mesh reports the total."""
    p = workloads.scaled_config2(8, 200, 500, seed=6)
    print(f"[predicates] fallback counters on {p.name}", flush=True)
    gm, rc = gpu_run(ctx, p)
    assert rc == 0
    st = gm.round_stats()
    tot = {k: sum(r[k] for r in st) for k in ("n_exact_orient", "n_exact_dot", "n_exact_incircle_b",
                                               "n_exact_incircle_c", "n_incircle_tests", "n_orient_tests")}
    assert tot["n_exact_incircle_c"] > 0 or tot["n_exact_incircle_b"] > 0, tot
    assert tot["n_incircle_tests"] > tot["n_exact_incircle_b"] + tot["n_exact_incircle_c"]
    assert tot["n_orient_tests"] > 0
    info = gm.info()
    assert info["fallbacks"] == sum(tot[k] for k in ("n_exact_orient", "n_exact_dot", "n_exact_incircle_b",
                                                      "n_exact_incircle_c"))
    # winners' sums: every inserted point has a cavity and a fan of at least 3 edges
    ins = sum(r["n_ins_mid"] + r["n_ins_cc"] for r in st)
    assert sum(r["win_cav_tri"] for r in st) >= ins
    assert sum(r["win_fan_edges"] for r in st) >= 3 * ins
    assert sum(r["win_walk_steps"] for r in st) >= sum(r["n_ins_cc"] for r in st)


def test_device_views_alias_the_mesh(ctx):
    """The zero-copy views hold the same arrays as a download."""
    import torch
    p = workloads.config0()
    print(f"[views] {p.name}", flush=True)
    gm, rc = gpu_run(ctx, p)
    assert rc == 0
    torch.cuda.synchronize()
    v = gm.device_views()
    a = gm.arrays()
    assert v["xy"].is_cuda and v["xy"].dtype == torch.float64
    assert np.array_equal(v["xy"].cpu().numpy().view(np.uint64), np.asarray(a["xy"]).view(np.uint64))
    assert np.array_equal(v["vkind"].cpu().numpy(), a["vkind"])
    assert np.array_equal(v["tri"][:, :3].cpu().numpy(), a["tv"])
    assert np.array_equal(v["nbr"][:, :3].cpu().numpy(), a["tn"])
    assert np.array_equal(v["sub_on_edge"][:, :3].cpu().numpy(), a["ts"])
    assert np.array_equal(v["sub_v"].cpu().numpy(), a["sv"])
    assert np.array_equal(v["sub_parent"].cpu().numpy(), a["sparent"])
    assert np.array_equal(v["sub_pending"].cpu().numpy(), np.asarray(a["spend"]).astype(np.int32))
    # no copy: the view's address is the library's
    assert v["tri"].data_ptr() == gm.device_views()["tri"].data_ptr()
