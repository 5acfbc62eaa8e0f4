"""Flip-Flop insertion on the GPU (insert_mode 1, Section 4.3 Line 8) against
the oracle's Flip-Flop rounds, element by element.

A Flip-Flop round leaves triangles in slots of the flips' choosing, so the
mesh is compared in canonical form: vertices, vertex kinds and subsegments
as stored (their ids are fixed by the rules of the round), triangles as the
sorted list of (rotation from the smallest vertex, subsegment per edge).
The per-round counters of Lines 3-8 must be equal too."""
import numpy as np
import pytest

import workloads
from tests.parity_util import COMMON_STATS, gpu_run, oracle_run
from tests.test_oracle_ff import canon, same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    return gdp2d.Context(0)

FF_STATS = COMMON_STATS + ["n_ff_points", "n_ff_iters"]
FF = dict(priority_mode=2, insert_mode=1)


def _check(ctx, p, **kw):
    print(f"[ff] {p.name} {kw}", flush=True)
    om, orc_rc = oracle_run(p, **FF, **kw)
    gm, gpu_rc = gpu_run(ctx, p, **FF, **kw)
    assert orc_rc == gpu_rc
    a, b = canon(om), canon(gm)
    bad = [k for k in a if not np.array_equal(a[k], b[k])]
    assert not bad, bad
    gs = gm.round_stats()
    assert len(gs) == len(om.stats)
    for r, (s, g) in enumerate(zip(om.stats, gs)):
        d = [f for f in FF_STATS if s[f] != g[f]]
        assert not d, (r, {f: (s[f], g[f]) for f in d})
    # the tn array must describe the same triangulation (canon() ignores it)
    arr = gm.arrays()
    tv, tn = arr["tv"], arr["tn"]
    for t in range(tv.shape[0]):
        for e in range(3):
            o = tn[t, e]
            if o < 0:
                continue
            u, v = tv[t, e], tv[t, (e + 1) % 3]
            assert any(tv[o, j] == v and tv[o, (j + 1) % 3] == u for j in range(3)), (t, e)
    return om, gm


SMALL = {
    "bare_square": lambda: workloads.bare_square(),
    "near_edge": lambda: workloads.near_edge_point(1e-3),
    "c0": lambda: workloads.config0(),
    "rand_60": lambda: workloads.random_small(31, 60, 5),
    "rand_300": lambda: workloads.random_small(32, 300, 20),
    "knn_2000": lambda: workloads.random_small(33, 2000, 100, pairing="knn"),
    "circles_small": lambda: workloads.scaled_config2(6, 40, 100, seed=5),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_ff_parity_small(ctx, name):
    _check(ctx, SMALL[name]())


@pytest.mark.parametrize("kw", [dict(cand_cap_K=7), dict(cand_cap_K=40), dict(encroach_mode=1),
                                dict(max_edge_len_sq=0.004), dict(prefilter_f1=1), dict(cavity_approx_n=4),
                                dict(split_mode=1), dict(max_rounds=5)])
@pytest.mark.parametrize("case", ["c0", "circles_small", "knn_2000"])
def test_ff_parity_options(ctx, case, kw):
    _check(ctx, SMALL[case](), **kw)


def test_ff_parity_resume_after_round_cap(ctx):
    """A refine call stopped by the round cap and resumed gives the mesh of
    one uninterrupted call."""
    from paper_2007_00324_amd import gdp2d
    p = workloads.random_small(44, 800, 40)
    om, _ = oracle_run(p, **FF)
    gm, rc = gpu_run(ctx, p, max_rounds=4, **FF)
    assert rc == -5
    gdp2d.gdp_mesh_refine(ctx, gm, p.ratio_bound_sq, gdp2d.make_params(**FF))
    assert same(canon(om), canon(gm))


def test_ff_parity_medium(ctx):
    _check(ctx, workloads.scaled_config1(20_000, 1_000, seed=3))


def test_ff_parity_circles_medium(ctx):
    _check(ctx, workloads.scaled_config2(24, 150, 2_000, seed=4))


def test_ff_rejects_slot_dependent_keys_and_other_forms(ctx):
    from paper_2007_00324_amd import gdp2d
    p = workloads.random_small(31, 60, 5)
    m = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)
    with pytest.raises(gdp2d.GdpError):
        gdp2d.gdp_mesh_refine(ctx, m, p.ratio_bound_sq, gdp2d.make_params(insert_mode=1))
    # the cavity kernels find a mark's owner from the perm32 half of mode 0/1 keys
    with pytest.raises(gdp2d.GdpError):
        gdp2d.gdp_mesh_refine(ctx, m, p.ratio_bound_sq, gdp2d.make_params(priority_mode=2))
    with pytest.raises(gdp2d.GdpError):
        gdp2d.gdp_refine_batch(ctx, [(p.xy, p.seg)], [p.ratio_bound_sq], gdp2d.make_params(**FF))


def test_ff_parity_rounded_cocircular_polygon(ctx):
    """8,192 rounded cocircular vertices: every interior triangle's circle holds
    the centre, so the first point added there ends with a link of thousands of
    vertices (thousands of flip passes, ties decided by the symbolic
    perturbation)."""
    p = workloads.scaled_config2(1, 8192, 0, seed=7, r_lo=0.40, r_hi=0.45)
    _check(ctx, p, cand_cap_K=8, max_rounds=4)
