"""Parity of the HIP refinement path with the oracle: every array of the final
mesh (vertex coordinates bitwise, triangles, neighbours, subsegment marks,
subsegments, pending flags) and every per-round counter must be identical.
"""
import numpy as np
import pytest

import workloads
from tests.parity_util import diff_arrays, diff_stats, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    return gdp2d.Context(0)


PERF_ONLY = ("reserve_mode", "rounds_per_sync", "block_size", "tail_engine_max", "cavity_thread_cap")


def _check(ctx, p, **kw):
    print(f"[parity] {p.name} {kw}", flush=True)
    om, orc_rc = oracle_run(p, **{k: v for k, v in kw.items() if k not in PERF_ONLY})
    gm, gpu_rc = gpu_run(ctx, p, **kw)
    assert orc_rc == gpu_rc
    a, b = om.arrays(), gm.arrays()
    bad = diff_arrays(a, b)
    assert not bad, bad
    sd = diff_stats(om.stats, gm.round_stats())
    assert not sd, sd
    assert gm.info()["rounds"] == om.rounds
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
def test_parity_small(ctx, name):
    _check(ctx, SMALL[name]())


@pytest.mark.parametrize("name", ["c0", "rand_300", "knn_2000", "circles_small"])
def test_parity_small_grid_only(ctx, name):
    """Every round on the multi-workgroup kernels (the single-workgroup engine off)."""
    _check(ctx, SMALL[name](), tail_engine_max=-1)


ENGINE_ALL = 1 << 30  # every round after the first in the single-workgroup engine


@pytest.mark.parametrize("kw", [dict(), dict(cand_cap_K=7), dict(prefilter_f1=1, cavity_approx_n=4),
                                dict(priority_mode=1), dict(reserve_mode=1), dict(max_rounds=6)])
@pytest.mark.parametrize("case", ["c0", "circles_small", "knn_2000"])
def test_parity_engine(ctx, case, kw):
    """Rounds run whole inside one workgroup give the same mesh and counters."""
    _check(ctx, SMALL[case](), tail_engine_max=ENGINE_ALL, **kw)


@pytest.mark.parametrize("cap", [12, 24, 39])
@pytest.mark.parametrize("case", ["circles_small", "knn_2000", "rand_300"])
def test_parity_cavity_thread_cap(ctx, case, cap):
    """The per-thread cavity capacity only moves cavities between the
    per-thread and the cooperative kernels; the mesh must not change."""
    _check(ctx, SMALL[case](), tail_engine_max=-1, cavity_thread_cap=cap)


@pytest.mark.parametrize("B2", [1.6 * 1.6, 4.0])
def test_parity_other_bounds(ctx, B2):
    p = workloads.random_small(41, 400, 20, bsq=B2)
    _check(ctx, p)


@pytest.mark.parametrize("K", [1, 7, 64])
def test_parity_candidate_cap(ctx, K):
    _check(ctx, workloads.random_small(42, 300, 15), cand_cap_K=K)


@pytest.mark.parametrize("f1,n", [(1, 0), (0, 1), (0, 4), (1, 8), (0, 16)])
@pytest.mark.parametrize("case", ["rand_300", "circles_small", "knn_2000"])
def test_parity_prefilters(ctx, case, f1, n):
    _check(ctx, SMALL[case](), prefilter_f1=f1, cavity_approx_n=n)


def test_parity_priority_mode_one(ctx):
    _check(ctx, workloads.random_small(43, 500, 25), priority_mode=1)


def test_parity_round_cap_and_resume(ctx):
    from paper_2007_00324_amd import gdp2d
    p = workloads.random_small(44, 800, 40)
    om, _ = oracle_run(p)
    gm, rc = gpu_run(ctx, p, max_rounds=4)
    assert rc == -5 and gm.info()["rounds"] == 4
    gdp2d.gdp_mesh_refine(ctx, gm, p.ratio_bound_sq, gdp2d.make_params())
    assert not diff_arrays(om.arrays(), gm.arrays())


def test_parity_block_size_invariance(ctx):
    p = workloads.random_small(45, 600, 30)
    om, _ = oracle_run(p)
    for bs in (64, 128, 512, 1024):
        gm, _ = gpu_run(ctx, p, block_size=bs)
        assert not diff_arrays(om.arrays(), gm.arrays()), bs


@pytest.mark.parametrize("case", ["c0", "circles_small"])
def test_parity_grow_on_demand(ctx, case):
    """Buffers grow only after a round is abandoned for lack of room; the
    rerun of that round must give the same mesh."""
    p = SMALL[case]()
    om, _ = oracle_run(p)
    gm, _ = gpu_run(ctx, p, reserve_mode=1)
    assert not diff_arrays(om.arrays(), gm.arrays())


@pytest.mark.parametrize("rps", [1, 3, 64])
def test_parity_rounds_per_sync(ctx, rps):
    """Rounds queued in groups between host synchronisations give the same mesh."""
    _check(ctx, workloads.random_small(47, 900, 45), rounds_per_sync=rps)


@pytest.mark.parametrize("kw", [dict(reserve_mode=1, rounds_per_sync=8), dict(cand_cap_K=9, rounds_per_sync=5),
                                dict(max_rounds=7, rounds_per_sync=4), dict(prefilter_f1=1, cavity_approx_n=3,
                                                                            rounds_per_sync=16)])
def test_parity_grouped_rounds_with_options(ctx, kw):
    """A round abandoned for lack of room, the candidate cap, the round cap and
    the prefilters inside a group of queued rounds."""
    p = workloads.scaled_config2(6, 40, 100, seed=5)
    print(f"[parity] grouped {kw}", flush=True)
    om, orc_rc = oracle_run(p, **{k: v for k, v in kw.items() if k not in PERF_ONLY})
    gm, gpu_rc = gpu_run(ctx, p, **kw)
    assert orc_rc == gpu_rc
    assert not diff_arrays(om.arrays(), gm.arrays())
    assert not diff_stats(om.stats, gm.round_stats())


def test_parity_from_uploaded_oracle_state(ctx):
    """Phase entry: the oracle's state after 3 rounds, uploaded, refined on the GPU."""
    import oracle
    from paper_2007_00324_amd import gdp2d
    p = workloads.random_small(46, 700, 35)
    m3 = oracle.build_cdt(p.xy, p.seg)
    oracle.refine(m3, 2.0, max_rounds=3)
    full, _ = oracle_run(p)
    g = gdp2d.gdp_mesh_upload(ctx, m3.arrays(), p.n_vertices, p.n_segments, rounds=3)
    gdp2d.gdp_mesh_refine(ctx, g, 2.0, gdp2d.make_params())
    assert not diff_arrays(full.arrays(), g.arrays())


MEDIUM = {"c1_100k": lambda: workloads.scaled_config1(100_000, 5_000),
          "c2_32x200": lambda: workloads.scaled_config2(32, 200, 5_000)}


@pytest.mark.parametrize("case", list(MEDIUM))
def test_parity_medium(ctx, case):
    _check(ctx, MEDIUM[case]())


@pytest.mark.parametrize("case", list(MEDIUM))
def test_parity_medium_engine(ctx, case):
    _check(ctx, MEDIUM[case](), tail_engine_max=ENGINE_ALL)


def test_reruns_identical(ctx):
    p = workloads.scaled_config1(20_000, 1_000, seed=9)
    a, _ = gpu_run(ctx, p)
    b, _ = gpu_run(ctx, p)
    assert not diff_arrays(a.arrays(), b.arrays())
