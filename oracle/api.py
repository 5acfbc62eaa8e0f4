"""ctypes binding of the oracle library (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

ORC_OK, ORC_E_ARG, ORC_E_INPUT, ORC_E_NOMEM, ORC_E_NOTERM, ORC_E_STALL, ORC_E_WALK = 0, -1, -2, -3, -5, -6, -8


class _Mesh(C.Structure):
    _fields_ = [
        ("nV", C.c_int32), ("nT", C.c_int32), ("nS", C.c_int32),
        ("n_input_v", C.c_int32), ("n_input_s", C.c_int32),
        ("capV", C.c_int32), ("capT", C.c_int32), ("capS", C.c_int32),
        ("rounds", C.c_int32),
        ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
        ("vkind", C.POINTER(C.c_int32)),
        ("tv", C.POINTER(C.c_int32)), ("tn", C.POINTER(C.c_int32)), ("ts", C.POINTER(C.c_int32)),
        ("sv", C.POINTER(C.c_int32)), ("sparent", C.POINTER(C.c_int32)),
        ("spend", C.POINTER(C.c_uint8)),
    ]


class _Params(C.Structure):
    _fields_ = [("cand_cap_K", C.c_int32), ("priority_mode", C.c_int32), ("max_rounds", C.c_int32),
                ("prefilter_f1", C.c_int32), ("cavity_approx_n", C.c_int32), ("encroach_mode", C.c_int32),
                ("split_mode", C.c_int32), ("max_edge_len_sq", C.c_double), ("insert_mode", C.c_int32)]


STAT_FIELDS = ["n_enc", "n_bad", "n_kept_mid", "n_kept_cc", "n_blocked", "n_coincident",
               "n_enc_reject", "n_mid_cand", "n_unsplittable", "n_fan_invalid", "n_lost_mark",
               "n_dep_drop", "n_ins_mid", "n_ins_cc", "cav_tri_total", "cav_max", "walk_steps",
               "n_f1_drop", "n_f2_drop", "n_ff_points", "n_ff_iters"]


class _Stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in STAT_FIELDS]


_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .build import build
        build()
    lib = C.CDLL(LIB_PATH)
    P2 = C.POINTER(C.c_double)
    lib.orc_cdt_build.argtypes = [C.c_int32, P2, C.c_int32, C.POINTER(C.c_int32),
                                  C.POINTER(C.POINTER(_Mesh)), C.c_char_p, C.c_int32]
    lib.orc_cdt_build.restype = C.c_int
    lib.orc_refine.argtypes = [C.POINTER(_Mesh), C.c_double, C.POINTER(_Params), C.POINTER(_Stats),
                               C.c_int32, C.POINTER(C.c_int32), C.c_char_p, C.c_int32]
    lib.orc_refine.restype = C.c_int
    lib.orc_mesh_clone.argtypes = [C.POINTER(_Mesh)]
    lib.orc_mesh_clone.restype = C.POINTER(_Mesh)
    lib.orc_mesh_free.argtypes = [C.POINTER(_Mesh)]
    lib.orc_mesh_free.restype = None
    for name in ("orc_orient2d", "orc_indiametral"):
        getattr(lib, name).argtypes = [P2, P2, P2]
        getattr(lib, name).restype = C.c_int
    lib.orc_incircle.argtypes = [P2, P2, P2, P2]
    lib.orc_incircle.restype = C.c_int
    lib.orc_incircle_sos.argtypes = [P2, P2, P2, P2, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    lib.orc_incircle_sos.restype = C.c_int
    lib.orc_exact_counts.argtypes = [C.POINTER(C.c_int64)] * 3
    lib.orc_exact_counts.restype = None
    lib.orc_perm32.argtypes = [C.c_uint32]
    lib.orc_perm32.restype = C.c_uint32
    lib.orc_check_topology.argtypes = [C.POINTER(_Mesh), C.c_char_p, C.c_int32]
    lib.orc_check_topology.restype = C.c_int64
    for name in ("orc_check_local_delaunay", "orc_check_cdt_bruteforce"):
        getattr(lib, name).argtypes = [C.POINTER(_Mesh)]
        getattr(lib, name).restype = C.c_int64
    lib.orc_check_encroached.argtypes = [C.POINTER(_Mesh), C.c_int32]
    lib.orc_check_encroached.restype = C.c_int64
    lib.orc_check_quality.argtypes = [C.POINTER(_Mesh), C.c_double, C.c_double]
    lib.orc_check_quality.restype = C.c_int64
    lib.orc_mesh_quality.argtypes = [C.POINTER(_Mesh), C.c_double, C.c_double, C.POINTER(C.c_int64), P2]
    lib.orc_mesh_quality.restype = None
    lib.orc_encroaches.argtypes = [C.c_int32, P2, P2, P2]
    lib.orc_encroaches.restype = C.c_int
    lib.orc_midpoint.argtypes = [C.POINTER(_Mesh), C.c_int32, P2, P2, C.POINTER(C.c_uint64), C.c_int32, C.c_int32]
    lib.orc_midpoint.restype = None
    lib.orc_check_subsegments.argtypes = [C.POINTER(_Mesh), P2, C.POINTER(C.c_int32), C.c_char_p, C.c_int32]
    lib.orc_check_subsegments.restype = C.c_int64
    PI = C.POINTER(C.c_int32)
    lib.orc_mesh_from_arrays.argtypes = [C.c_int32, C.c_int32, P2, PI, C.c_int32, PI, PI, PI,
                                         C.c_int32, C.c_int32, PI, PI, C.POINTER(C.c_uint8)]
    lib.orc_mesh_from_arrays.restype = C.POINTER(_Mesh)
    lib.orc_ruppert.argtypes = [C.POINTER(_Mesh), C.c_double, C.c_int64, C.POINTER(C.c_int64),
                                C.c_char_p, C.c_int32]
    lib.orc_ruppert.restype = C.c_int
    lib.orc_area_sum.argtypes = [C.POINTER(_Mesh)]
    lib.orc_area_sum.restype = C.c_double
    lib.orc_hull_vertex_count.argtypes = [C.POINTER(_Mesh)]
    lib.orc_hull_vertex_count.restype = C.c_int32
    _lib = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code
        self.msg = msg


def _pt(p):
    a = (C.c_double * 2)(float(p[0]), float(p[1]))
    return a


def orient2d(a, b, c) -> int:
    return load().orc_orient2d(_pt(a), _pt(b), _pt(c))


def incircle(a, b, c, d) -> int:
    return load().orc_incircle(_pt(a), _pt(b), _pt(c), _pt(d))


def encroaches(mode: int, a, b, p) -> int:
    """Subsegment ab encroached by p: diametric circle (mode 0) or lens (mode 1)."""
    return load().orc_encroaches(mode, _pt(a), _pt(b), _pt(p))


def indiametral(a, b, c) -> int:
    return load().orc_indiametral(_pt(a), _pt(b), _pt(c))


def incircle_sos(a, b, c, d, ia, ib, ic, id_) -> int:
    return load().orc_incircle_sos(_pt(a), _pt(b), _pt(c), _pt(d), ia, ib, ic, id_)


def perm32(x: int) -> int:
    return int(load().orc_perm32(x & 0xFFFFFFFF))


def exact_counts():
    o, i, d = C.c_int64(), C.c_int64(), C.c_int64()
    load().orc_exact_counts(C.byref(o), C.byref(i), C.byref(d))
    return o.value, i.value, d.value


class OracleMesh:
    """Owns an oracle mesh; arrays are exposed as numpy copies."""

    def __init__(self, ptr, in_xy=None, in_seg=None):
        self._p = ptr
        self.in_xy = in_xy
        self.in_seg = in_seg
        self.stats: list[dict] = []

    def __del__(self):
        if getattr(self, "_p", None) and _lib is not None:
            _lib.orc_mesh_free(self._p)
            self._p = None

    @property
    def m(self) -> _Mesh:
        return self._p.contents

    def clone(self) -> "OracleMesh":
        return OracleMesh(load().orc_mesh_clone(self._p), self.in_xy, self.in_seg)

    @property
    def nV(self): return self.m.nV

    @property
    def nT(self): return self.m.nT

    @property
    def nS(self): return self.m.nS

    @property
    def rounds(self): return self.m.rounds

    def arrays(self) -> dict:
        m = self.m
        nV, nT, nS = m.nV, m.nT, m.nS
        f = np.ctypeslib.as_array
        return {
            "xy": np.stack([f(m.x, (nV,)).copy(), f(m.y, (nV,)).copy()], axis=1) if nV else np.zeros((0, 2)),
            "vkind": f(m.vkind, (nV,)).copy(),
            "tv": f(m.tv, (nT * 3,)).reshape(nT, 3).copy(),
            "tn": f(m.tn, (nT * 3,)).reshape(nT, 3).copy(),
            "ts": f(m.ts, (nT * 3,)).reshape(nT, 3).copy(),
            "sv": f(m.sv, (nS * 2,)).reshape(nS, 2).copy(),
            "sparent": f(m.sparent, (nS,)).copy(),
            "spend": f(m.spend, (nS,)).copy(),
        }

    # ---- checkers ----
    def check_topology(self):
        buf = C.create_string_buffer(256)
        n = load().orc_check_topology(self._p, buf, 256)
        return n, buf.value.decode()

    def check_local_delaunay(self): return load().orc_check_local_delaunay(self._p)
    def check_quality(self, B2, L2=0.0): return load().orc_check_quality(self._p, B2, L2)
    def check_encroached(self, mode=0): return load().orc_check_encroached(self._p, mode)

    def split_point(self, k: int, split_mode: int = 0):
        """Splitting point and key of subsegment k (midpoint, or concentric shells)."""
        x, y, key = C.c_double(0.0), C.c_double(0.0), C.c_uint64(0)
        load().orc_midpoint(self._p, k, C.byref(x), C.byref(y), C.byref(key), 0, split_mode)
        return x.value, y.value, key.value

    def quality(self, B2, L2=0.0):
        """(bad triangle count, area they cover) under the criteria."""
        n, a = C.c_int64(0), C.c_double(0.0)
        load().orc_mesh_quality(self._p, B2, L2, C.byref(n), C.byref(a))
        return n.value, a.value
    def check_cdt_bruteforce(self): return load().orc_check_cdt_bruteforce(self._p)
    def area(self): return load().orc_area_sum(self._p)
    def hull_count(self): return load().orc_hull_vertex_count(self._p)

    def check_subsegments(self):
        xy = np.ascontiguousarray(self.in_xy, dtype=np.float64)
        seg = np.ascontiguousarray(self.in_seg, dtype=np.int32)
        buf = C.create_string_buffer(256)
        n = load().orc_check_subsegments(self._p, xy.ctypes.data_as(C.POINTER(C.c_double)),
                                         seg.ctypes.data_as(C.POINTER(C.c_int32)), buf, 256)
        return n, buf.value.decode()


def build_cdt(xy: np.ndarray, seg: np.ndarray) -> OracleMesh:
    lib = load()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    seg = np.ascontiguousarray(seg, dtype=np.int32).reshape(-1, 2)
    out = C.POINTER(_Mesh)()
    err = C.create_string_buffer(256)
    rc = lib.orc_cdt_build(xy.shape[0], xy.ctypes.data_as(C.POINTER(C.c_double)), seg.shape[0],
                           seg.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(out), err, 256)
    if rc != ORC_OK:
        raise OracleError(rc, err.value.decode())
    return OracleMesh(out, xy.copy(), seg.copy())


def mesh_from_arrays(arr: dict, n_input_v: int, n_input_s: int, in_xy=None, in_seg=None) -> OracleMesh:
    """An oracle mesh holding the given arrays (the dict form of
    ``OracleMesh.arrays()``), e.g. a deliberately damaged copy for checker
    tests."""
    lib = load()
    xy = np.ascontiguousarray(arr["xy"], dtype=np.float64).reshape(-1, 2)
    vk = np.ascontiguousarray(arr["vkind"], dtype=np.int32)
    tv = np.ascontiguousarray(arr["tv"], dtype=np.int32).reshape(-1, 3)
    tn = np.ascontiguousarray(arr["tn"], dtype=np.int32).reshape(-1, 3)
    ts = np.ascontiguousarray(arr["ts"], dtype=np.int32).reshape(-1, 3)
    sv = np.ascontiguousarray(arr["sv"], dtype=np.int32).reshape(-1, 2)
    sp = np.ascontiguousarray(arr["sparent"], dtype=np.int32)
    pe = np.ascontiguousarray(arr["spend"], dtype=np.uint8)
    PI = C.POINTER(C.c_int32)
    ptr = lib.orc_mesh_from_arrays(xy.shape[0], n_input_v, xy.ctypes.data_as(C.POINTER(C.c_double)),
                                   vk.ctypes.data_as(PI), tv.shape[0], tv.ctypes.data_as(PI),
                                   tn.ctypes.data_as(PI), ts.ctypes.data_as(PI), sv.shape[0], n_input_s,
                                   sv.ctypes.data_as(PI), sp.ctypes.data_as(PI),
                                   pe.ctypes.data_as(C.POINTER(C.c_uint8)))
    if not ptr:
        raise OracleError(ORC_E_NOMEM, "mesh_from_arrays failed")
    return OracleMesh(ptr, in_xy, in_seg)


def ruppert(mesh: OracleMesh, ratio_bound_sq: float, max_insertions: int = 0) -> dict:
    """Classic sequential Ruppert refinement of ``mesh`` in place (the
    point-count reference).  Returns the status and counters."""
    lib = load()
    uns = C.c_int64(0)
    err = C.create_string_buffer(256)
    rc = lib.orc_ruppert(mesh._p, float(ratio_bound_sq), int(max_insertions), C.byref(uns), err, 256)
    if rc not in (ORC_OK, ORC_E_NOTERM):
        raise OracleError(rc, err.value.decode())
    return {"rc": rc, "n_unsplittable": uns.value}


def refine(mesh: OracleMesh, ratio_bound_sq: float, cand_cap_K: int = 0, priority_mode: int = 0,
           max_rounds: int = 0, stats_cap: int = 1 << 16, raise_on_error: bool = True,
           prefilter_f1: int = 0, cavity_approx_n: int = 0, encroach_mode: int = 0,
           max_edge_len_sq: float = 0.0, split_mode: int = 0, insert_mode: int = 0) -> int:
    lib = load()
    prm = _Params(cand_cap_K, priority_mode, max_rounds, prefilter_f1, cavity_approx_n, encroach_mode,
                  split_mode, float(max_edge_len_sq), insert_mode)
    st = (_Stats * stats_cap)()
    ns = C.c_int32(0)
    err = C.create_string_buffer(256)
    rc = lib.orc_refine(mesh._p, float(ratio_bound_sq), C.byref(prm), st, stats_cap, C.byref(ns), err, 256)
    mesh.stats.extend({f: getattr(st[i], f) for f in STAT_FIELDS} for i in range(ns.value))
    if rc != ORC_OK and raise_on_error and rc != ORC_E_NOTERM:
        raise OracleError(rc, err.value.decode())
    return rc
