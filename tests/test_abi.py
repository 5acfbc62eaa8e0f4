"""CPU checks of the C ABI: the library loads, exports every function that
include/gdp2d.h declares, and its host-side Line 1 (initial CDT) equals the
oracle's canonical CDT on the same inputs (two independent builders)."""
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gdp2d.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gdp_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    from paper_2007_00324_amd import gdp2d
    lib = gdp2d.load()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(gdp2d.exported_symbols())


def test_status_strings():
    from paper_2007_00324_amd import gdp2d
    lib = gdp2d.load()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        assert lib.gdp_status_str(code)


CASES = {
    "bare_square": lambda: workloads.bare_square(),
    "near_edge": lambda: workloads.near_edge_point(),
    "c0": lambda: workloads.config0(),
    "knn_5k": lambda: workloads.random_small(61, 5000, 250, pairing="knn"),
    "c1_like_50k": lambda: workloads.scaled_config1(50_000, 2_500, seed=3),
    "c2_like": lambda: workloads.scaled_config2(16, 100, 2_000, seed=4),
    # a segment whose crossed triangles wrap around a vertex, where the slit
    # edge left between them is itself a segment (its id must survive)
    "knn_constrained_slit": lambda: workloads.random_small(1243, 3000, 600, pairing="knn"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_host_cdt_equals_oracle_cdt(orc, name):
    from paper_2007_00324_amd import gdp2d
    p = CASES[name]()
    tri, nbr, seg = gdp2d.gdp_cdt_host(p.xy, p.seg)
    a = orc.build_cdt(p.xy, p.seg).arrays()
    assert np.array_equal(tri, a["tv"])
    assert np.array_equal(nbr, a["tn"])
    assert np.array_equal(seg, a["ts"])


@pytest.mark.parametrize("kind", ["cross", "dup_point", "vertex_on_segment", "hull_uncovered", "repeat_seg",
                                  "out_of_range"])
def test_host_cdt_rejects_invalid_input(kind):
    from paper_2007_00324_amd import gdp2d
    base = workloads.bare_square()
    xy, seg = base.xy.copy(), base.seg.copy()
    if kind == "cross":
        xy = np.concatenate([xy, [[0.2, 0.2], [0.8, 0.8], [0.2, 0.8], [0.8, 0.2]]])
        seg = np.concatenate([seg, [[4, 5], [6, 7]]])
    elif kind == "dup_point":
        xy = np.concatenate([xy, [[0.3, 0.3], [0.3, 0.3]]])
    elif kind == "vertex_on_segment":
        xy = np.concatenate([xy, [[0.25, 0.25], [0.75, 0.75], [0.5, 0.5]]])
        seg = np.concatenate([seg, [[4, 5]]])
    elif kind == "hull_uncovered":
        seg = seg[:3]
    elif kind == "repeat_seg":
        seg = np.concatenate([seg, [[1, 0]]])
    elif kind == "out_of_range":
        xy = np.concatenate([xy, [[0.5, 1e-40]]])
    with pytest.raises(gdp2d.GdpError) as e:
        gdp2d.gdp_cdt_host(xy, seg)
    assert e.value.code == -2


def test_server_calls_reject_a_missing_server():
    """Argument checks that need no device: a NULL server is GDP_E_ARG."""
    import ctypes as C
    from paper_2007_00324_amd import gdp2d
    lib = gdp2d.load()
    assert lib.gdp_server_line1(None, 4, 0) == -1
    assert lib.gdp_server_mode(None, 0, 0) == -1
    assert lib.gdp_server_engine_jobs(None, 0) == -1
    assert lib.gdp_server_arrive(None, C.c_uint64(1)) == -1
