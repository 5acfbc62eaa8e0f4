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


ENGINE_PATHS = {"slots": 0, "batched": 1 << 30, "split": 1500}


@pytest.mark.parametrize("path", list(ENGINE_PATHS))
def test_server_matches_oracle(ctx, path):
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(20, seed=21)
    srv = gdp2d.Server(ctx, 2 << 30, 8, engine_max_vertices=ENGINE_PATHS[path])
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


@pytest.mark.parametrize("path", list(ENGINE_PATHS))
def test_server_alone_equals_mix(ctx, path):
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(30, seed=22, n_max=8000)
    x = ps[7]
    alone_srv = gdp2d.Server(ctx, 1 << 30, 4, engine_max_vertices=0)
    m_alone, rc, _ = alone_srv.wait(alone_srv.submit(x.xy, x.seg, x.ratio_bound_sq))
    assert rc == 0
    mix = gdp2d.Server(ctx, 4 << 30, 12, engine_max_vertices=ENGINE_PATHS[path])
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


@pytest.mark.parametrize("path", ["slots", "batched"])
def test_server_tight_budget_and_slots(ctx, path):
    """Room for about one job at a time: jobs wait for room, all finish."""
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(8, seed=23, n_min=1000, n_max=2000)
    srv = gdp2d.Server(ctx, 8 << 20, 2, engine_max_vertices=ENGINE_PATHS[path])
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
