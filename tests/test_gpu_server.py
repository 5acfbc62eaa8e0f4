"""Serving form: jobs arrive while others run (continuous batching).  Each
result must be identical to the oracle's, alone or in a mix."""
import pytest

import workloads
from tests.parity_util import diff_arrays, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

GDP_E_BUSY, GDP_E_NOMEM = -7, -3


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    return gdp2d.Context(0)


def _jobs(count, seed, n_min=200, n_max=3000):
    return workloads.batch_config3(count, seed=seed, n_min=n_min, n_max=n_max)


# shared rounds (the default), a stream per slot, every job in the batched
# single-workgroup engine launches, and small jobs there with the rest shared
PATHS = {"shared": dict(mode=0, engine_max_vertices=0), "slots": dict(mode=1, engine_max_vertices=0),
         "batched": dict(mode=0, engine_max_vertices=1 << 30), "split": dict(mode=0, engine_max_vertices=1500)}


@pytest.mark.parametrize("path", list(PATHS))
def test_server_matches_oracle(ctx, path):
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(20, seed=21)
    srv = gdp2d.Server(ctx, 2 << 30, 8, **PATHS[path])
    ids = [srv.submit(p.xy, p.seg, p.ratio_bound_sq) for p in ps]
    print(f"[server] {len(ids)} jobs submitted", flush=True)
    for p, j in zip(ps, ids):
        m, rc, t = srv.wait(j)
        assert rc == 0 and m is not None, (p.name, rc)
        assert t["submit_ms"] <= t["admit_ms"] <= t["done_ms"]
        om, orc = oracle_run(p)
        assert not diff_arrays(om.arrays(), m.arrays()), p.name
        assert m.info()["rounds"] == om.rounds
    srv.close()


@pytest.mark.parametrize("path", list(PATHS))
def test_server_alone_equals_mix(ctx, path):
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(30, seed=22, n_max=8000)
    x = ps[7]
    alone_srv = gdp2d.Server(ctx, 1 << 30, 4, engine_max_vertices=0)
    m_alone, rc, _ = alone_srv.wait(alone_srv.submit(x.xy, x.seg, x.ratio_bound_sq))
    assert rc == 0
    mix = gdp2d.Server(ctx, 4 << 30, 12, **PATHS[path])
    ids = [mix.submit(p.xy, p.seg, p.ratio_bound_sq) for p in ps]
    got = [mix.wait(j) for j in ids]
    assert all(rc == 0 for _, rc, _ in got)
    assert not diff_arrays(m_alone.arrays(), got[7][0].arrays())
    plain, _ = gpu_run(ctx, x)
    assert not diff_arrays(plain.arrays(), got[7][0].arrays())
    for p, (m, _, _) in zip(ps[:6], got[:6]):
        om, _ = oracle_run(p)
        assert not diff_arrays(om.arrays(), m.arrays()), p.name
    mix.close()
    alone_srv.close()


@pytest.mark.parametrize("path", ["shared", "slots", "batched"])
def test_server_tight_budget_and_slots(ctx, path):
    """Room for about one job at a time: jobs wait for room, all finish."""
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(8, seed=23, n_min=1000, n_max=2000)
    srv = gdp2d.Server(ctx, 8 << 20, 2, **PATHS[path])
    ids = [srv.submit(p.xy, p.seg, p.ratio_bound_sq) for p in ps]
    for p, j in zip(ps, ids):
        m, rc, _ = srv.wait(j)
        assert rc == 0
        om, _ = oracle_run(p)
        assert not diff_arrays(om.arrays(), m.arrays()), p.name
        m.free()  # gives the room back
    srv.close()


def test_server_prepared_job_and_close(ctx):
    """A prepared job that has not arrived is pending; meshes handed out stay
    valid after the server is closed; a job larger than the budget is refused."""
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(3, seed=24)
    srv = gdp2d.Server(ctx, 1 << 30, 4)
    j0 = srv.prepare(ps[0].xy, ps[0].seg, ps[0].ratio_bound_sq)
    m, rc, _ = srv.poll(j0)
    assert m is None and rc == GDP_E_BUSY
    j1 = srv.submit(ps[1].xy, ps[1].seg, ps[1].ratio_bound_sq)
    m1, rc1, _ = srv.wait(j1)
    assert rc1 == 0
    srv.arrive(j0)
    m0, rc0, _ = srv.wait(j0)
    assert rc0 == 0
    j2 = srv.submit(ps[2].xy, ps[2].seg, ps[2].ratio_bound_sq)  # left for close() to finish and free
    srv.close()
    for p, mm in ((ps[0], m0), (ps[1], m1)):
        om, _ = oracle_run(p)
        assert not diff_arrays(om.arrays(), mm.arrays())
    small = gdp2d.Server(ctx, 1 << 20, 1)
    big = workloads.batch_instance(20000, 2.0, 5)
    with pytest.raises(gdp2d.GdpError):
        small.prepare(big.xy, big.seg, 2.0)
    small.close()
    del j2


@pytest.mark.parametrize("kw", [dict(cand_cap_K=5), dict(max_rounds=3), dict(prefilter_f1=1, cavity_approx_n=2),
                                dict(encroach_mode=1, max_edge_len_sq=0.004)])
def test_shared_rounds_options_match_oracle(ctx, kw):
    """Semantic options per job in the shared rounds (each job's own
    parameters in its descriptor), mixed with default jobs."""
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(10, seed=25, n_min=300, n_max=4000)
    srv = gdp2d.Server(ctx, 2 << 30, 6)
    ids = []
    for i, p in enumerate(ps):
        opt = kw if i % 2 == 0 else {}
        ids.append((p, opt, srv.submit(p.xy, p.seg, p.ratio_bound_sq, gdp2d.make_params(**opt))))
    for p, opt, j in ids:
        m, rc, _ = srv.wait(j)
        om, orc = oracle_run(p, **opt)
        assert rc == orc, (p.name, rc, orc)
        assert not diff_arrays(om.arrays(), m.arrays()), (p.name, opt)
    srv.close()


def test_shared_rounds_large_cavity_and_growth(ctx):
    """A polygon of 8,192 rounded cocircular vertices (a cavity far beyond a
    workgroup's local list) beside ordinary jobs, in regions sized for the
    inputs: the shared rounds finish the large cavity in device memory and
    grow the jobs that outgrow their regions."""
    from paper_2007_00324_amd import gdp2d
    circle = workloads.scaled_config2(1, 8192, 0, seed=7, r_lo=0.40, r_hi=0.45)
    dense = workloads.random_small(27, 300, 15)  # with l = 0.01: ~50 times its input vertices
    ps = [circle, dense] + _jobs(5, seed=26, n_min=2000, n_max=20000)
    opts = [dict(cand_cap_K=8, max_rounds=3), dict(max_edge_len_sq=1e-4)] + [{}] * 5
    srv = gdp2d.Server(ctx, 2 << 30, 6)
    ids = [srv.submit(p.xy, p.seg, p.ratio_bound_sq, gdp2d.make_params(**o)) for p, o in zip(ps, opts)]
    for p, o, j in zip(ps, opts, ids):
        m, rc, _ = srv.wait(j)
        om, orc = oracle_run(p, **o)
        assert rc == orc, (p.name, rc, orc)
        assert not diff_arrays(om.arrays(), m.arrays()), p.name
        if p is circle:
            assert sum(r["n_huge_cavities"] for r in m.round_stats()) >= 1
    srv.close()
