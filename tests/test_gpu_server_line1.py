"""Serving form with Line 1 (the initial CDT, Section 4.3) inside the server:
built after arrival on host threads, or for large jobs by the device builder
directly in the job's region.  Each result must equal the oracle's and the
plain form's, alone or in a mix; invalid PSLGs end their job with
GDP_E_INPUT and leave the others untouched."""
import numpy as np
import pytest

import workloads
from tests.parity_util import diff_arrays, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

GDP_E_INPUT = -2


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    return gdp2d.Context(0)


def _jobs(count, seed, n_min=200, n_max=3000):
    return workloads.batch_config3(count, seed=seed, n_min=n_min, n_max=n_max)


# (host threads, device threshold): host only; large jobs on the device; every
# job on the device; host Line 1 with a stream per slot
LINE1 = {"host": dict(line1=(4, 0)), "device": dict(line1=(2, 1000)), "device_all": dict(line1=(1, 3)),
         "host_slots": dict(mode=1, line1=(3, 1000))}


@pytest.mark.parametrize("path", list(LINE1))
def test_line1_in_server_matches_oracle(ctx, path):
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(16, seed=31)
    srv = gdp2d.Server(ctx, 2 << 30, 6, engine_max_vertices=0, **LINE1[path])
    ids = [srv.submit(p.xy, p.seg, p.ratio_bound_sq) for p in ps]
    print(f"[line1 {path}] {len(ids)} jobs submitted", flush=True)
    for p, j in zip(ps, ids):
        m, rc, t = srv.wait(j)
        assert rc == 0 and m is not None, (p.name, rc)
        assert t["submit_ms"] <= t["line1_ms"] <= t["admit_ms"] <= t["done_ms"], t
        om, orc = oracle_run(p)
        assert not diff_arrays(om.arrays(), m.arrays()), p.name
        assert m.info()["rounds"] == om.rounds
        m.free()
    srv.close()


@pytest.mark.parametrize("path", ["host", "device"])
def test_line1_in_server_alone_equals_mix(ctx, path):
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(24, seed=32, n_max=8000)
    x = max(ps, key=lambda p: p.n_vertices)
    k = ps.index(x)
    alone = gdp2d.Server(ctx, 1 << 30, 2, engine_max_vertices=0, **LINE1[path])
    m_alone, rc, _ = alone.wait(alone.submit(x.xy, x.seg, x.ratio_bound_sq))
    assert rc == 0
    mix = gdp2d.Server(ctx, 4 << 30, 10, engine_max_vertices=0, **LINE1[path])
    ids = [mix.submit(p.xy, p.seg, p.ratio_bound_sq) for p in ps]
    got = [mix.wait(j) for j in ids]
    assert all(rc == 0 for _, rc, _ in got)
    assert not diff_arrays(m_alone.arrays(), got[k][0].arrays())
    plain, _ = gpu_run(ctx, x)
    assert not diff_arrays(plain.arrays(), got[k][0].arrays())
    mix.close()
    alone.close()


def test_line1_device_tight_budget(ctx):
    """Room for about one job at a time: the device Line-1 thread waits for
    room before it builds, and every job still finishes."""
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(6, seed=33, n_min=1000, n_max=2000)
    srv = gdp2d.Server(ctx, 8 << 20, 2, engine_max_vertices=0, line1=(1, 500))
    ids = [srv.submit(p.xy, p.seg, p.ratio_bound_sq) for p in ps]
    for p, j in zip(ps, ids):
        m, rc, _ = srv.wait(j)
        assert rc == 0, (p.name, rc)
        om, _ = oracle_run(p)
        assert not diff_arrays(om.arrays(), m.arrays()), p.name
        m.free()
    srv.close()


def _crossing():
    sq = workloads.bare_square()
    xy = np.vstack([sq.xy, [[0.25, 0.25], [0.75, 0.75], [0.25, 0.75], [0.75, 0.25]]])
    seg = np.vstack([sq.seg, [[4, 5], [6, 7]]]).astype(np.int32)
    return xy, seg


@pytest.mark.parametrize("path", ["host", "device_all"])
def test_line1_in_server_invalid_job(ctx, path):
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(4, seed=34)
    srv = gdp2d.Server(ctx, 1 << 30, 4, engine_max_vertices=0, **LINE1[path])
    xy, seg = _crossing()
    bad = srv.submit(xy, seg, 2.0)
    ids = [srv.submit(p.xy, p.seg, p.ratio_bound_sq) for p in ps]
    m, rc, t = srv.wait(bad)
    assert rc == GDP_E_INPUT and m is None
    assert t["line1_ms"] == t["done_ms"]
    for p, j in zip(ps, ids):
        m, rc, _ = srv.wait(j)
        assert rc == 0
        om, _ = oracle_run(p)
        assert not diff_arrays(om.arrays(), m.arrays()), p.name
        m.free()
    srv.close()


def test_line1_set_before_first_job(ctx):
    from paper_2007_00324_amd import gdp2d
    ps = _jobs(1, seed=35)
    srv = gdp2d.Server(ctx, 1 << 30, 2)
    j = srv.prepare(ps[0].xy, ps[0].seg, ps[0].ratio_bound_sq)
    with pytest.raises(gdp2d.GdpError):
        srv.line1(2, 0)
    srv.arrive(j)
    m, rc, _ = srv.wait(j)
    assert rc == 0
    srv.close()


def test_line1_device_cocircular_jobs(ctx):
    """Line 1 on the device inside the server for rounded-cocircular polygons
    (cavities far beyond the builder's per-thread lists), two of them in a
    row on the same builder workspace, among ordinary jobs."""
    from paper_2007_00324_amd import gdp2d
    ps = [workloads.scaled_config2(1, 6000, 0, seed=s, r_lo=0.40, r_hi=0.45) for s in (7, 8)]
    ps += _jobs(4, seed=36)
    srv = gdp2d.Server(ctx, 2 << 30, 4, engine_max_vertices=0, line1=(2, 5000))
    ids = [srv.submit(p.xy, p.seg, p.ratio_bound_sq) for p in ps]
    print(f"[line1 cocircular] {len(ids)} jobs submitted", flush=True)
    for p, j in zip(ps, ids):
        m, rc, _ = srv.wait(j)
        assert rc == 0 and m is not None, (p.name, rc)
        om, orc = oracle_run(p)
        assert orc == 0
        assert not diff_arrays(om.arrays(), m.arrays()), p.name
        m.free()
    srv.close()
