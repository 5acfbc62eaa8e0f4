"""The allocation-free quality entry point (gdp_mesh_quality_noalloc) against
gdp_mesh_quality: two calls in a row on one device, the second on a smaller
mesh, each result equal bit for bit (same kernels, same partial-sum order);
results land in caller device memory."""
import ctypes as C

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _noalloc(ctx, mesh, bsq, l2):
    import torch
    from paper_2007_00324_amd import gdp2d
    out_n = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    out_a = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    rc = gdp2d.load().gdp_mesh_quality_noalloc(ctx._h, mesh._h, float(bsq), float(l2),
                                               C.c_void_p(out_n.data_ptr()), C.c_void_p(out_a.data_ptr()))
    ctx.check(rc)
    torch.cuda.synchronize()
    return int(out_n.item()), float(out_a.item())


def test_noalloc_quality_equals_allocating_entry():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    ctx = gdp2d.Context(0)
    big = workloads.scaled_config1(200_000, 10_000, seed=5)
    small = workloads.config0()
    print("[no_alloc] initial CDTs of a 200k-point PSLG, then the 1k-point PSLG", flush=True)
    for p, l2 in ((big, 0.0), (small, 1e-3)):
        m = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)   # unrefined: many bad triangles
        want = m.quality(p.ratio_bound_sq, l2)
        got = _noalloc(ctx, m, p.ratio_bound_sq, l2)
        assert want[0] > 0
        assert got[0] == want[0]
        assert np.float64(got[1]).view(np.uint64) == np.float64(want[1]).view(np.uint64)
        m.free()


def test_noalloc_rejects_bad_arguments():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    ctx = gdp2d.Context(0)
    p = workloads.config0()
    m = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)
    lib = gdp2d.load()
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    assert lib.gdp_mesh_quality_noalloc(ctx._h, m._h, -1.0, 0.0, C.c_void_p(out.data_ptr()),
                                        C.c_void_p(out.data_ptr() + 8)) == -1
    assert lib.gdp_mesh_quality_noalloc(ctx._h, m._h, 2.0, 0.0, None, None) == -1
