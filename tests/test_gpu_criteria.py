"""Parity of the HIP path with the oracle under the other quality criteria of
Section 4.1 (edge-length bound l, diametric-lens encroachment of Chew's
algorithm), on the multi-workgroup kernels and on the single-workgroup
engine, and of the device bad-area measure (Table 1) with the oracle's:
meshes bitwise, counts exactly, the area to 1e-12 relative (sums in
different orders).
"""
import pytest

import workloads
from tests.parity_util import diff_arrays, diff_stats, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

ENGINE_ALL = 1 << 30


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    return gdp2d.Context(0)


CASES = {
    "c0": lambda: workloads.config0(),
    "rand_300": lambda: workloads.random_small(32, 300, 20),
    "knn_2000": lambda: workloads.random_small(33, 2000, 100, pairing="knn"),
    "circles_small": lambda: workloads.scaled_config2(6, 40, 100, seed=5),
    "spokes_30": lambda: workloads.spokes(30),
}
MODES = {
    "length": dict(max_edge_len_sq=0.004),
    "lens": dict(encroach_mode=1),
    "lens_length": dict(encroach_mode=1, max_edge_len_sq=0.002),
    "shells": dict(split_mode=1),
    "shells_lens_length": dict(split_mode=1, encroach_mode=1, max_edge_len_sq=0.002),
}


def _check(ctx, p, mode, **perf):
    kw = MODES[mode]
    print(f"[criteria] {p.name} {mode} {perf}", flush=True)
    om, orc_rc = oracle_run(p, **kw)
    gm, gpu_rc = gpu_run(ctx, p, **kw, **perf)
    assert orc_rc == gpu_rc
    bad = diff_arrays(om.arrays(), gm.arrays())
    assert not bad, bad
    sd = diff_stats(om.stats, gm.round_stats())
    assert not sd, sd
    return om, gm


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("name", list(CASES))
def test_criteria_parity(ctx, name, mode):
    _check(ctx, CASES[name](), mode)


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("engine", [-1, ENGINE_ALL])
def test_criteria_parity_paths(ctx, mode, engine):
    """Every round on the grid kernels, and every round inside one workgroup."""
    _check(ctx, CASES["knn_2000"](), mode, tail_engine_max=engine)


@pytest.mark.parametrize("mode", list(MODES))
def test_bad_area_parity(ctx, mode):
    p = CASES["knn_2000"]()
    om, gm = _check(ctx, p, mode)
    L2 = MODES[mode].get("max_edge_len_sq", 0.0)
    for B2, l2 in [(p.ratio_bound_sq, L2), (1.2, 0.0), (1.0, L2 * 0.5), (0.3, 0.0)]:
        n_o, a_o = om.quality(B2, l2)
        n_g, a_g = gm.quality(B2, l2)
        assert n_g == n_o, (B2, l2)
        assert abs(a_g - a_o) <= 1e-12 * max(1.0, abs(a_o)), (B2, l2, a_g, a_o)
    assert gm.quality(p.ratio_bound_sq, L2) == (0, 0.0)


def test_bad_area_initial_cdt(ctx):
    """The unrefined CDT: many bad triangles; area within rounding of the oracle's."""
    import oracle
    from paper_2007_00324_amd import gdp2d
    p = workloads.random_small(34, 5000, 250, pairing="knn")
    om = oracle.build_cdt(p.xy, p.seg)
    gm = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)
    for B2, l2 in [(2.0, 0.0), (2.0, 1e-4), (4.0, 0.0)]:
        n_o, a_o = om.quality(B2, l2)
        n_g, a_g = gm.quality(B2, l2)
        assert n_g == n_o and n_o > 0
        assert abs(a_g - a_o) <= 1e-12 * max(1.0, abs(a_o))


@pytest.mark.slow
@pytest.mark.parametrize("mode", ["lens", "lens_length"])
def test_criteria_parity_200k(ctx, mode):
    """The 1M-point generator scaled to 200k points: many tiles, both paths."""
    p = workloads.scaled_config1(200_000, 10_000)
    kw = dict(MODES[mode])
    if "max_edge_len_sq" in kw:
        kw["max_edge_len_sq"] = 1e-5
    print(f"[criteria] {p.name} {mode} {kw}", flush=True)
    om, orc_rc = oracle_run(p, **kw)
    gm, gpu_rc = gpu_run(ctx, p, **kw)
    assert orc_rc == gpu_rc == 0
    bad = diff_arrays(om.arrays(), gm.arrays())
    assert not bad, bad
    n_o, a_o = om.quality(p.ratio_bound_sq, kw.get("max_edge_len_sq", 0.0))
    assert gm.quality(p.ratio_bound_sq, kw.get("max_edge_len_sq", 0.0)) == (n_o, a_o) == (0, 0.0)


@pytest.mark.parametrize("engine", [0, -1])
def test_small_angle_stall_parity(ctx, engine):
    """Spokes 15 degrees apart: refinement runs until a round has candidates
    but can insert nothing (GDP_E_STALL on both sides), with identical meshes
    and round counters up to that point."""
    from paper_2007_00324_amd import gdp2d
    p = workloads.spokes(15)
    om, orc_rc = oracle_run(p)
    assert orc_rc == -6
    gm = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)
    with pytest.raises(gdp2d.GdpError) as e:
        gdp2d.gdp_mesh_refine(ctx, gm, p.ratio_bound_sq, gdp2d.make_params(tail_engine_max=engine))
    assert e.value.code == -6
    bad = diff_arrays(om.arrays(), gm.arrays())
    assert not bad, bad
    sd = diff_stats(om.stats, gm.round_stats())
    assert not sd, sd
