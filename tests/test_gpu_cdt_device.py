"""Line 1 of Algorithm 1 on the GPU (gdp_mesh_create_device) against the
oracle's CDT and the host builder's: every array equal, element by element
(the CDT is unique under the symbolic perturbation and both sides use the
canonical triangle order).  Inputs cover uniform points with long segments,
kNN segments, rounded-cocircular circles, an exactly cocircular grid, small
input angles and the degenerate squares; invalid PSLGs must fail on both
builders with GDP_E_INPUT.
"""
import numpy as np
import pytest

import workloads
from tests.parity_util import diff_arrays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    return gdp2d.Context(0)


def grid_pslg(k: int = 15):
    """The square plus the (k x k) interior points of the 1/(k+1) grid with
    k + 1 a power of two (exact coordinates: every grid square cocircular)."""
    h = 1.0 / (k + 1)
    g = np.array([(i * h, j * h) for i in range(1, k + 1) for j in range(1, k + 1)])
    xy = np.vstack([workloads.generators.CORNERS, g])
    seg = workloads.generators.BOUNDARY.copy()
    # interior segments: a grid edge, two diagonals that pass no grid point
    extra = np.array([[4, 5], [4, 4 + k + 3], [4 + k, 4 + 2 * k + 1]], dtype=np.int32)
    return xy, np.vstack([seg, extra]).astype(np.int32)


CASES = {
    "bare_square": lambda: (workloads.bare_square().xy, workloads.bare_square().seg),
    "near_edge": lambda: (workloads.near_edge_point().xy, workloads.near_edge_point().seg),
    "c0": lambda: (workloads.config0().xy, workloads.config0().seg),
    "rand_300": lambda: (workloads.random_small(32, 300, 20).xy, workloads.random_small(32, 300, 20).seg),
    "knn_2000": lambda: (lambda p: (p.xy, p.seg))(workloads.random_small(33, 2000, 100, pairing="knn")),
    "circles_small": lambda: (lambda p: (p.xy, p.seg))(workloads.scaled_config2(6, 40, 100, seed=5)),
    "spokes_30": lambda: (lambda p: (p.xy, p.seg))(workloads.spokes(30)),
    "grid_15": lambda: grid_pslg(15),
    "c1_20k": lambda: (lambda p: (p.xy, p.seg))(workloads.scaled_config1(20_000, 1000, seed=7)),
}


def _device_arrays(ctx, xy, seg):
    from paper_2007_00324_amd import gdp2d
    m = gdp2d.gdp_mesh_create_device(ctx, xy, seg)
    return m.arrays()


@pytest.mark.parametrize("name", list(CASES))
def test_device_cdt_equals_oracle_and_host(ctx, name):
    import oracle
    from paper_2007_00324_amd import gdp2d
    xy, seg = CASES[name]()
    print(f"device CDT case {name}: {len(xy)} vertices, {len(seg)} segments", flush=True)
    dev = _device_arrays(ctx, xy, seg)
    host = gdp2d.gdp_mesh_create(ctx, xy, seg).arrays()
    assert not diff_arrays(host, dev), diff_arrays(host, dev)
    orc = oracle.build_cdt(xy, seg).arrays()
    assert not diff_arrays(orc, dev), diff_arrays(orc, dev)


def test_device_cdt_refines_like_host(ctx):
    from paper_2007_00324_amd import gdp2d
    p = workloads.config0()
    a = gdp2d.gdp_mesh_create_device(ctx, p.xy, p.seg)
    b = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)
    prm = gdp2d.make_params()
    gdp2d.gdp_mesh_refine(ctx, a, p.ratio_bound_sq, prm)
    gdp2d.gdp_mesh_refine(ctx, b, p.ratio_bound_sq, prm)
    assert not diff_arrays(b.arrays(), a.arrays())


def _bad_inputs():
    sq = workloads.bare_square()
    c, s = sq.xy, sq.seg
    yield "duplicate", np.vstack([c, [[0.5, 0.5], [0.25, 0.75], [0.5, 0.5]]]), s
    yield "repeated_segment", np.vstack([c, [[0.25, 0.25], [0.75, 0.75]]]), np.vstack([s, [[4, 5], [5, 4]]])
    yield "crossing", np.vstack([c, [[0.25, 0.25], [0.75, 0.75], [0.25, 0.75], [0.75, 0.25]]]), \
        np.vstack([s, [[4, 5], [6, 7]]])
    yield "vertex_on_segment", np.vstack([c, [[0.25, 0.25], [0.5, 0.5], [0.75, 0.75]]]), np.vstack([s, [[4, 6]]])
    yield "hull_not_segment", np.vstack([c, [[0.5, 0.5]]]), s[:3]
    yield "vertex_on_boundary", np.vstack([c, [[0.5, 0.0]]]), s


@pytest.mark.parametrize("case", list(_bad_inputs()), ids=lambda c: c[0])
def test_device_cdt_rejects_invalid(ctx, case):
    from paper_2007_00324_amd import gdp2d
    name, xy, seg = case
    seg = np.asarray(seg, np.int32)
    with pytest.raises(gdp2d.GdpError) as host_err:
        gdp2d.gdp_mesh_create(ctx, xy, seg)
    with pytest.raises(gdp2d.GdpError) as dev_err:
        gdp2d.gdp_mesh_create_device(ctx, xy, seg)
    assert host_err.value.code == dev_err.value.code == -2, (host_err.value, dev_err.value)


@pytest.mark.slow
@pytest.mark.parametrize("name", ["c1_full", "c2_full"])
def test_device_cdt_full_configs(ctx, name):
    from paper_2007_00324_amd import gdp2d
    p = workloads.config1() if name == "c1_full" else workloads.config2()
    print(f"device CDT case {name}", flush=True)
    dev = _device_arrays(ctx, p.xy, p.seg)
    host = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg).arrays()
    assert not diff_arrays(host, dev), diff_arrays(host, dev)


def circle_pslg(n: int, with_center: bool, seed: int):
    """The square plus n points on a circle (rounded cocircular) and uniform
    interior points inside it: large cavities under the perturbation."""
    rng = np.random.default_rng(seed)
    a = np.sort(rng.uniform(0, 2 * np.pi, n))
    pts = np.stack([0.5 + 0.3 * np.cos(a), 0.5 + 0.3 * np.sin(a)], axis=1)
    inner = rng.uniform(0.3, 0.7, (n // 10, 2))
    inner = inner[((inner - 0.5) ** 2).sum(axis=1) < 0.25 ** 2]
    extra = [[0.5, 0.5]] if with_center else []
    xy = np.vstack([workloads.generators.CORNERS, pts, inner] + ([np.array(extra)] if extra else []))
    k = np.arange(n)
    seg = np.stack([4 + k, 4 + (k + 1) % n], axis=1)[::3]  # every third chord of the polygon
    return xy, np.vstack([workloads.generators.BOUNDARY, seg]).astype(np.int32)


def rows_pslg(k: int = 40):
    """Exactly collinear rows of points (dyadic coordinates) with segments
    between row neighbours two apart: collinear and cocircular ties."""
    h = 1.0 / 64
    pts = [(i * h, j * h) for j in range(8, 57, 8) for i in range(4, 4 + k)]
    xy = np.vstack([workloads.generators.CORNERS, np.array(pts)])
    seg = [[4 + r * k + i, 4 + r * k + i + 1] for r in range(7) for i in range(0, k - 1, 3)]
    return xy, np.vstack([workloads.generators.BOUNDARY, np.array(seg)]).astype(np.int32)


MORE = {
    **{f"uniform_s{s}": (lambda s=s: (lambda p: (p.xy, p.seg))(workloads.random_small(100 + s, 3000, 60)))
       for s in range(4)},
    **{f"knn_s{s}": (lambda s=s: (lambda p: (p.xy, p.seg))(workloads.random_small(200 + s, 5000, 400, pairing="knn")))
       for s in range(3)},
    "circles_b": lambda: (lambda p: (p.xy, p.seg))(workloads.scaled_config2(20, 100, 500, seed=9)),
    "spokes_60": lambda: (lambda p: (p.xy, p.seg))(workloads.spokes(60, n_spokes=3)),
    "circle_2000": lambda: circle_pslg(2000, False, 3),
    "circle_2000_center": lambda: circle_pslg(2000, True, 4),
    "rows": lambda: rows_pslg(),
    "knn_constrained_slit": lambda: (lambda p: (p.xy, p.seg))(workloads.random_small(1243, 3000, 600, pairing="knn")),
}


@pytest.mark.parametrize("name", list(MORE))
def test_device_cdt_more_inputs(ctx, name):
    import oracle
    xy, seg = MORE[name]()
    print(f"device CDT case {name}: {len(xy)} vertices, {len(seg)} segments", flush=True)
    dev = _device_arrays(ctx, xy, seg)
    orc = oracle.build_cdt(xy, seg).arrays()
    assert not diff_arrays(orc, dev), diff_arrays(orc, dev)
