"""Batched form: many PSLGs refined in one persistent launch.  Each mesh must
be identical to the oracle's and to the plain per-instance path's."""
import numpy as np
import pytest

import workloads
from tests.parity_util import diff_arrays, diff_stats, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    return gdp2d.Context(0)


def _batch(ctx, ps, **kw):
    from paper_2007_00324_amd import gdp2d
    prm = gdp2d.make_params(**kw)
    return gdp2d.gdp_refine_batch(ctx, [(p.xy, p.seg) for p in ps], [p.ratio_bound_sq for p in ps], prm)


def test_batch_matches_oracle(ctx):
    ps = workloads.batch_config3(48, seed=11, n_min=100, n_max=3000)
    print(f"[batch] {len(ps)} instances, {sum(p.n_vertices for p in ps)} vertices", flush=True)
    meshes, st, ms = _batch(ctx, ps)
    assert all(s == 0 for s in st), st
    for p, g in zip(ps, meshes):
        om, rc = oracle_run(p)
        assert rc == 0
        bad = diff_arrays(om.arrays(), g.arrays())
        assert not bad, (p.name, bad)
        assert g.info()["rounds"] == om.rounds
        assert not diff_stats(om.stats[:64], g.round_stats()), p.name


@pytest.mark.parametrize("kw", [dict(cand_cap_K=5), dict(prefilter_f1=1, cavity_approx_n=2), dict(priority_mode=1),
                                dict(max_rounds=5), dict(encroach_mode=1, max_edge_len_sq=0.004)])
def test_batch_options_match_oracle(ctx, kw):
    ps = workloads.batch_config3(12, seed=12, n_min=100, n_max=1500)
    meshes, st, _ = _batch(ctx, ps, **kw)
    for p, g, s in zip(ps, meshes, st):
        om, rc = oracle_run(p, **kw)
        assert s == rc, (p.name, s, rc)
        assert not diff_arrays(om.arrays(), g.arrays()), p.name


def test_batch_equals_plain_path(ctx):
    """Each instance alone (plain loop) and in the batch give the same mesh."""
    from tests.parity_util import gpu_run
    ps = workloads.batch_config3(24, seed=13, n_min=500, n_max=20000)
    meshes, st, _ = _batch(ctx, ps)
    assert all(s == 0 for s in st), st
    for p, g in zip(ps, meshes):
        alone, rc = gpu_run(ctx, p)
        assert rc == 0
        assert not diff_arrays(alone.arrays(), g.arrays()), p.name


def test_batch_member_refined_again(ctx):
    """A batch mesh can leave the batch (round cap first, then refined on its
    own to the end), and the others are unaffected."""
    from paper_2007_00324_amd import gdp2d
    ps = workloads.batch_config3(6, seed=14, n_min=200, n_max=2000)
    meshes, st, _ = _batch(ctx, ps, max_rounds=3)
    assert all(s == -5 for s in st), st
    gdp2d.gdp_mesh_refine(ctx, meshes[2], ps[2].ratio_bound_sq, gdp2d.make_params())
    om, _ = oracle_run(ps[2])
    assert not diff_arrays(om.arrays(), meshes[2].arrays())
    o3, _ = oracle_run(ps[3], max_rounds=3)
    assert not diff_arrays(o3.arrays(), meshes[3].arrays())
    del meshes


def test_batch_invalid_member(ctx):
    """A member with an invalid PSLG gets an error status; the rest refine."""
    ps = workloads.batch_config3(4, seed=15, n_min=100, n_max=500)
    bad = workloads.bare_square()
    xy = np.vstack([bad.xy, [[0.5, 0.5], [0.5, 0.5]]])  # duplicate point
    from paper_2007_00324_amd import gdp2d
    inputs = [(p.xy, p.seg) for p in ps] + [(xy, bad.seg)]
    meshes, st, _ = gdp2d.gdp_refine_batch(ctx, inputs, [p.ratio_bound_sq for p in ps] + [2.0])
    assert st[-1] != 0 and meshes[-1] is None
    assert all(s == 0 for s in st[:-1])
    for p, g in zip(ps, meshes[:-1]):
        om, _ = oracle_run(p)
        assert not diff_arrays(om.arrays(), g.arrays())


@pytest.mark.parametrize("split", [1500, 200])
def test_batch_split_between_engine_and_shared_rounds(ctx, split):
    """Meshes above the split run in shared rounds, the rest in the engine:
    every mesh is still the oracle's (the split is perf only)."""
    from paper_2007_00324_amd import gdp2d
    ps = workloads.batch_config3(24, seed=16, n_min=100, n_max=6000)
    print(f"[batch] split at {split} input vertices", flush=True)
    meshes, st, _ = _batch(ctx, ps, batch_engine_max_v=split)
    assert all(s == 0 for s in st), st
    assert any(p.n_vertices > split for p in ps) and any(p.n_vertices <= split for p in ps)
    for p, g in zip(ps, meshes):
        om, rc = oracle_run(p)
        assert not diff_arrays(om.arrays(), g.arrays()), p.name
        assert g.info()["rounds"] == om.rounds
        assert not diff_stats(om.stats[:64], g.round_stats()), p.name


@pytest.mark.parametrize("dev_min,split", [(1000, 0), (3, 0), (1500, 800)])
def test_batch_line1_on_device(ctx, dev_min, split):
    """Inputs of at least dev_min vertices get their initial CDT from the
    device builder (into the batch's arena), the rest from host threads:
    every mesh is still the oracle's, also with members in shared rounds."""
    ps = workloads.batch_config3(24, seed=17, n_min=100, n_max=4000)
    print(f"[batch] Line 1 on the device from {dev_min} vertices, split {split}", flush=True)
    meshes, st, _ = _batch(ctx, ps, batch_line1_device_min_v=dev_min, batch_engine_max_v=split)
    assert all(s == 0 for s in st), st
    assert any(p.n_vertices >= dev_min for p in ps)
    for p, g in zip(ps, meshes):
        om, rc = oracle_run(p)
        assert not diff_arrays(om.arrays(), g.arrays()), p.name
        assert g.info()["rounds"] == om.rounds


def test_batch_line1_on_device_invalid_member(ctx):
    """An invalid PSLG among device-built members fails alone (GDP_E_INPUT)."""
    from paper_2007_00324_amd import gdp2d
    ps = workloads.batch_config3(4, seed=18, n_min=100, n_max=500)
    sq = workloads.bare_square()
    xy = np.vstack([sq.xy, [[0.25, 0.25], [0.75, 0.75], [0.25, 0.75], [0.75, 0.25]]])
    seg = np.vstack([sq.seg, [[4, 5], [6, 7]]]).astype(np.int32)  # crossing segments
    inputs = [(xy, seg)] + [(p.xy, p.seg) for p in ps]
    meshes, st, _ = gdp2d.gdp_refine_batch(ctx, inputs, [2.0] + [p.ratio_bound_sq for p in ps],
                                           gdp2d.make_params(batch_line1_device_min_v=3))
    assert st[0] == -2 and meshes[0] is None
    assert all(s == 0 for s in st[1:])
    for p, g in zip(ps, meshes[1:]):
        om, _ = oracle_run(p)
        assert not diff_arrays(om.arrays(), g.arrays())


def test_batch_line1_on_device_cocircular(ctx):
    """Device Line 1 in the batch for a rounded-cocircular polygon (large
    builder cavities) next to ordinary inputs built on the host."""
    ps = [workloads.scaled_config2(1, 6000, 0, seed=7, r_lo=0.40, r_hi=0.45)]
    ps += workloads.batch_config3(6, seed=19, n_min=100, n_max=2000)
    meshes, st, _ = _batch(ctx, ps, batch_line1_device_min_v=5000)
    assert all(s == 0 for s in st), st
    for p, g in zip(ps, meshes):
        om, rc = oracle_run(p)
        assert rc == 0
        assert not diff_arrays(om.arrays(), g.arrays()), p.name
