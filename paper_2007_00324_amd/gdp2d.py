"""Python binding of libgdp2d.so (include/gdp2d.h): argument marshalling only.

Every step of the refinement runs in the library's HIP kernels; this module
converts numpy arrays to pointers and back.  PyTorch is imported first so the
library binds to the same HIP runtime as torch, and is used for the stream.
The binding fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgdp2d.so")

GDP_OK = 0
STATUS = {0: "GDP_OK", -1: "GDP_E_ARG", -2: "GDP_E_INPUT", -3: "GDP_E_NOMEM", -4: "GDP_E_DEVICE",
          -5: "GDP_E_NOTERM", -6: "GDP_E_STALL", -7: "GDP_E_BUSY", -8: "GDP_E_WALK", -9: "GDP_E_CAVITY"}


class GdpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.msg = msg


class gdp_pslg(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("xy", C.POINTER(C.c_double)),
                ("n_segments", C.c_int32), ("seg", C.POINTER(C.c_int32))]


class gdp_job_times(C.Structure):
    _fields_ = [("submit_ms", C.c_double), ("line1_ms", C.c_double), ("admit_ms", C.c_double),
                ("done_ms", C.c_double)]


class gdp_params(C.Structure):
    _fields_ = [("cand_cap_K", C.c_int32), ("priority_mode", C.c_int32), ("max_rounds", C.c_int32),
                ("prefilter_f1", C.c_int32), ("cavity_approx_n", C.c_int32), ("block_size", C.c_int32),
                ("profile_kernels", C.c_int32), ("reserve_mode", C.c_int32), ("rounds_per_sync", C.c_int32),
                ("tail_engine_max", C.c_int32), ("encroach_mode", C.c_int32), ("split_mode", C.c_int32),
                ("max_edge_len_sq", C.c_double), ("batch_engine_max_v", C.c_int32),
                ("cavity_thread_cap", C.c_int32), ("insert_mode", C.c_int32),
                ("batch_line1_device_min_v", C.c_int32)]


class gdp_kernel_prof(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("items", C.c_int64), ("alg_bytes", C.c_int64)]


class gdp_mesh_info(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_triangles", C.c_int32), ("n_subsegments", C.c_int32),
                ("n_input_vertices", C.c_int32), ("n_input_segments", C.c_int32), ("rounds", C.c_int32),
                ("cdt_point_rounds", C.c_int32), ("cdt_segment_rounds", C.c_int32), ("fallbacks", C.c_int64)]


class gdp_device_views(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_triangles", C.c_int32), ("n_subsegments", C.c_int32),
                ("tri_stride", C.c_int32), ("xy", C.c_void_p), ("vkind", C.c_void_p), ("tri", C.c_void_p),
                ("nbr", C.c_void_p), ("sub_on_edge", C.c_void_p), ("sub_v", C.c_void_p),
                ("sub_parent", C.c_void_p), ("sub_pending", C.c_void_p)]


STAT_FIELDS = ["n_enc", "n_bad", "n_kept_mid", "n_kept_cc", "n_blocked", "n_coincident", "n_enc_reject",
               "n_mid_cand", "n_unsplittable", "n_fan_invalid", "n_lost_mark", "n_dep_drop", "n_ins_mid",
               "n_ins_cc", "cav_tri_total", "cav_max", "n_big_cavities", "n_f1_drop", "n_f2_drop",
               "n_incircle_tests", "n_orient_tests", "n_exact_orient", "n_exact_dot", "n_exact_incircle_b",
               "n_exact_incircle_c", "win_cav_tri", "win_fan_edges", "win_walk_steps", "win_cc_cav_tri",
               "win_cc_fan_edges", "n_huge_cavities", "n_marks_mid", "n_marks_cc", "n_ff_points", "n_ff_iters",
               "n_flips", "n_flip_passes", "n_removals", "n_removal_passes"]


class gdp_round_stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in STAT_FIELDS]


_lib = None
_VP = C.c_void_p
_PI = C.POINTER(C.c_int32)
_PD = C.POINTER(C.c_double)


def load() -> C.CDLL:
    """Loads libgdp2d.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (binds the HIP runtime torch ships)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2007_00324_amd.build")
    lib = C.CDLL(LIB_PATH)
    S = C.c_int
    sig = {
        "gdp_params_default": (None, [C.POINTER(gdp_params)]),
        "gdp_status_str": (C.c_char_p, [S]),
        "gdp_ctx_create": (S, [C.c_int, _VP, C.POINTER(_VP)]),
        "gdp_ctx_destroy": (None, [_VP]),
        "gdp_last_error": (C.c_char_p, [_VP]),
        "gdp_mesh_create": (S, [_VP, C.POINTER(gdp_pslg), C.POINTER(_VP)]),
        "gdp_mesh_create_device": (S, [_VP, C.POINTER(gdp_pslg), C.POINTER(_VP)]),
        "gdp_cdt_host": (S, [C.POINTER(gdp_pslg), _PI, C.c_int32, _PI, _PI, _PI, C.c_char_p, C.c_int32]),
        "gdp_mesh_upload": (S, [_VP, C.c_int32, C.c_int32, _PD, _PI, C.c_int32, _PI, _PI, _PI, C.c_int32,
                                C.c_int32, _PI, _PI, C.POINTER(C.c_uint8), C.c_int32, C.POINTER(_VP)]),
        "gdp_mesh_refine": (S, [_VP, _VP, C.c_double, C.POINTER(gdp_params)]),
        "gdp_refine": (S, [_VP, C.POINTER(gdp_pslg), C.c_double, C.POINTER(gdp_params), C.POINTER(_VP)]),
        "gdp_mesh_info_get": (S, [_VP, C.POINTER(gdp_mesh_info)]),
        "gdp_mesh_quality": (S, [_VP, _VP, C.c_double, C.c_double, C.POINTER(C.c_int64), _PD]),
        "gdp_mesh_download": (S, [_VP, _VP, _PD, _PI, _PI, _PI, _PI, _PI, _PI, C.POINTER(C.c_uint8)]),
        "gdp_mesh_round_stats": (S, [_VP, C.POINTER(gdp_round_stats), C.c_int32, _PI]),
        "gdp_mesh_last_refine_ms": (S, [_VP, C.POINTER(C.c_double)]),
        "gdp_mesh_kernel_profile": (S, [_VP, C.POINTER(gdp_kernel_prof), C.c_int32, _PI]),
        "gdp_mesh_assign": (S, [_VP, _VP, _VP]),
        "gdp_mesh_clone": (S, [_VP, _VP, C.POINTER(_VP)]),
        "gdp_mesh_free": (None, [_VP]),
        "gdp_refine_batch": (S, [_VP, C.POINTER(gdp_pslg), _PD, C.POINTER(gdp_params), C.c_int32, C.POINTER(_VP),
                                 C.POINTER(C.c_int), C.POINTER(C.c_double)]),
        "gdp_server_create": (S, [_VP, C.c_size_t, C.c_int32, C.POINTER(_VP)]),
        "gdp_server_prepare": (S, [_VP, C.POINTER(gdp_pslg), C.c_double, C.POINTER(gdp_params), C.POINTER(C.c_uint64)]),
        "gdp_server_arrive": (S, [_VP, C.c_uint64]),
        "gdp_server_submit": (S, [_VP, C.POINTER(gdp_pslg), C.c_double, C.POINTER(gdp_params), C.POINTER(C.c_uint64)]),
        "gdp_server_poll": (S, [_VP, C.c_uint64, C.POINTER(_VP), C.POINTER(gdp_job_times)]),
        "gdp_server_wait": (S, [_VP, C.c_uint64, C.POINTER(_VP), C.POINTER(gdp_job_times)]),
        "gdp_server_destroy": (None, [_VP]),
        "gdp_server_engine_jobs": (S, [_VP, C.c_int32]),
        "gdp_server_mode": (S, [_VP, C.c_int32, C.c_int32]),
        "gdp_server_line1": (S, [_VP, C.c_int32, C.c_int32]),
        "gdp_mesh_device_views": (S, [_VP, C.POINTER(gdp_device_views)]),
        "gdp_predicates_eval": (S, [_VP, C.c_int32, C.c_int32, _PD, _PI, C.POINTER(C.c_int64)]),
        "gdp_bench_atomic_max": (S, [_VP, C.c_int64, C.c_int64, C.POINTER(C.c_double)]),
        "gdp_mesh_quality_noalloc": (S, [_VP, _VP, C.c_double, C.c_double, _VP, _VP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return ["gdp_params_default", "gdp_status_str", "gdp_ctx_create", "gdp_ctx_destroy", "gdp_last_error",
            "gdp_mesh_create", "gdp_mesh_create_device", "gdp_cdt_host", "gdp_mesh_upload", "gdp_mesh_refine", "gdp_refine",
            "gdp_mesh_info_get", "gdp_mesh_quality", "gdp_mesh_download", "gdp_mesh_round_stats", "gdp_mesh_last_refine_ms",
            "gdp_mesh_kernel_profile", "gdp_mesh_assign", "gdp_mesh_clone", "gdp_mesh_free", "gdp_refine_batch",
            "gdp_server_create", "gdp_server_prepare", "gdp_server_arrive", "gdp_server_submit", "gdp_server_poll",
            "gdp_server_wait", "gdp_server_engine_jobs", "gdp_server_destroy", "gdp_mesh_device_views",
            "gdp_predicates_eval", "gdp_bench_atomic_max", "gdp_mesh_quality_noalloc", "gdp_server_mode",
            "gdp_server_line1"]


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _pslg(xy, seg):
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    seg = np.ascontiguousarray(seg, dtype=np.int32).reshape(-1, 2)
    p = gdp_pslg(xy.shape[0], _ptr(xy, C.c_double), seg.shape[0], _ptr(seg, C.c_int32))
    return p, (xy, seg)


def make_params(cand_cap_K=0, priority_mode=0, max_rounds=0, block_size=256, profile_kernels=0,
                prefilter_f1=0, cavity_approx_n=0, reserve_mode=0, rounds_per_sync=0,
                tail_engine_max=0, encroach_mode=0, max_edge_len_sq=0.0, split_mode=0,
                batch_engine_max_v=0, cavity_thread_cap=0, insert_mode=0,
                batch_line1_device_min_v=0) -> gdp_params:
    p = gdp_params()
    load().gdp_params_default(C.byref(p))
    p.batch_line1_device_min_v = batch_line1_device_min_v
    p.insert_mode = insert_mode
    p.batch_engine_max_v = batch_engine_max_v
    p.cavity_thread_cap = cavity_thread_cap
    p.encroach_mode = encroach_mode
    p.split_mode = split_mode
    p.max_edge_len_sq = float(max_edge_len_sq)
    p.reserve_mode = reserve_mode
    p.rounds_per_sync = rounds_per_sync
    p.tail_engine_max = tail_engine_max
    p.prefilter_f1 = prefilter_f1
    p.cavity_approx_n = cavity_approx_n
    p.profile_kernels = profile_kernels
    p.cand_cap_K = cand_cap_K
    p.priority_mode = priority_mode
    p.max_rounds = max_rounds
    p.block_size = block_size
    return p


def gdp_cdt_host(xy, seg):
    """Line 1 on the host: canonical CDT arrays (tri, nbr, seg) of shape (T, 3)."""
    lib = load()
    p, keep = _pslg(xy, seg)
    nt = C.c_int32(0)
    err = C.create_string_buffer(256)
    rc = lib.gdp_cdt_host(C.byref(p), C.byref(nt), 0, None, None, None, err, 256)
    if rc != GDP_OK:
        raise GdpError(rc, err.value.decode())
    T = nt.value
    tri = np.empty((T, 3), np.int32)
    nbr = np.empty((T, 3), np.int32)
    sg = np.empty((T, 3), np.int32)
    rc = lib.gdp_cdt_host(C.byref(p), C.byref(nt), T, _ptr(tri, C.c_int32), _ptr(nbr, C.c_int32),
                          _ptr(sg, C.c_int32), err, 256)
    if rc != GDP_OK:
        raise GdpError(rc, err.value.decode())
    return tri, nbr, sg


PRED_KINDS = {"orient2d": 0, "incircle": 1, "indiametral": 2, "lens": 3}


def gdp_predicates_eval(ctx, kind: str, pts: np.ndarray):
    """The library's predicates on query rows (6 or 8 doubles each): on the
    device of ctx, or on the host when ctx is None.  Returns (signs, stage
    counts [orient, dot, incircle B, incircle C])."""
    lib = load()
    k = PRED_KINDS[kind]
    w = 8 if k == 1 else 6
    q = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, w)
    n = q.shape[0]
    out = np.empty(n, np.int32)
    counts = (C.c_int64 * 4)()
    h = ctx._h if ctx is not None else None
    rc = lib.gdp_predicates_eval(h, k, n, _ptr(q, C.c_double), _ptr(out, C.c_int32), counts)
    if rc != GDP_OK:
        raise GdpError(rc, lib.gdp_last_error(h).decode() if h is not None else "bad predicate query")
    return out, list(counts)


def gdp_bench_atomic_max(ctx, n_slots: int, n_ops: int) -> float:
    """Device ms of n_ops random-slot 64-bit atomicMax on a table of n_slots words."""
    ms = C.c_double(0.0)
    ctx.check(load().gdp_bench_atomic_max(ctx._h, int(n_slots), int(n_ops), C.byref(ms)))
    return ms.value


class Context:
    """A device context bound to a HIP stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self._h = _VP()
        rc = lib.gdp_ctx_create(device, _VP(stream), C.byref(self._h))
        if rc != GDP_OK:
            raise GdpError(rc, lib.gdp_last_error(None).decode())
        self.device = device

    def check(self, rc: int, ok=(GDP_OK,)):
        if rc not in ok:
            raise GdpError(rc, load().gdp_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            load().gdp_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    def __init__(self, ctx: Context, handle: _VP):
        self.ctx = ctx
        self._h = handle

    def free(self):
        if getattr(self, "_h", None):
            load().gdp_mesh_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self) -> dict:
        i = gdp_mesh_info()
        self.ctx.check(load().gdp_mesh_info_get(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in gdp_mesh_info._fields_}

    def quality(self, ratio_bound_sq: float, max_edge_len_sq: float = 0.0):
        """(bad triangle count, area they cover) under the criteria, on the device."""
        n, a = C.c_int64(0), C.c_double(0.0)
        self.ctx.check(load().gdp_mesh_quality(self.ctx._h, self._h, float(ratio_bound_sq), float(max_edge_len_sq),
                                               C.byref(n), C.byref(a)))
        return n.value, a.value

    def device_views(self) -> dict:
        """Zero-copy torch tensors over the mesh's device arrays (the library
        keeps ownership; valid until the mesh is freed, refined or assigned)."""
        import torch
        v = gdp_device_views()
        self.ctx.check(load().gdp_mesh_device_views(self._h, C.byref(v)))
        V, T, S = v.n_vertices, v.n_triangles, v.n_subsegments
        dev = torch.device("cuda", self.ctx.device)

        def wrap(ptr, n, dtype, shape):
            if n == 0:
                return torch.empty(shape, dtype=dtype, device=dev)
            iface = {"shape": (n,), "typestr": "<f8" if dtype == torch.float64 else "<i4",
                     "data": (ptr, False), "version": 3, "strides": None}
            holder = type("_View", (), {"__cuda_array_interface__": iface})()
            return torch.as_tensor(holder, device=dev).view(shape)

        return {"xy": wrap(v.xy, 2 * V, torch.float64, (V, 2)),
                "vkind": wrap(v.vkind, V, torch.int32, (V,)),
                "tri": wrap(v.tri, 4 * T, torch.int32, (T, 4)),
                "nbr": wrap(v.nbr, 4 * T, torch.int32, (T, 4)),
                "sub_on_edge": wrap(v.sub_on_edge, 4 * T, torch.int32, (T, 4)),
                "sub_v": wrap(v.sub_v, 2 * S, torch.int32, (S, 2)),
                "sub_parent": wrap(v.sub_parent, S, torch.int32, (S,)),
                "sub_pending": wrap(v.sub_pending, S, torch.int32, (S,))}

    def arrays(self) -> dict:
        lib = load()
        i = self.info()
        V, T, S = i["n_vertices"], i["n_triangles"], i["n_subsegments"]
        xy = np.empty((V, 2), np.float64)
        vk = np.empty(V, np.int32)
        tv = np.empty((T, 3), np.int32)
        tn = np.empty((T, 3), np.int32)
        ts = np.empty((T, 3), np.int32)
        sv = np.empty((max(S, 1), 2), np.int32)
        sp = np.empty(max(S, 1), np.int32)
        pe = np.empty(max(S, 1), np.uint8)
        self.ctx.check(lib.gdp_mesh_download(self.ctx._h, self._h, _ptr(xy, C.c_double), _ptr(vk, C.c_int32),
                                             _ptr(tv, C.c_int32), _ptr(tn, C.c_int32), _ptr(ts, C.c_int32),
                                             _ptr(sv, C.c_int32), _ptr(sp, C.c_int32), _ptr(pe, C.c_uint8)))
        return {"xy": xy, "vkind": vk, "tv": tv, "tn": tn, "ts": ts, "sv": sv[:S], "sparent": sp[:S],
                "spend": pe[:S]}

    def round_stats(self) -> list[dict]:
        lib = load()
        n = C.c_int32(0)
        lib.gdp_mesh_round_stats(self._h, None, 0, C.byref(n))
        arr = (gdp_round_stats * max(n.value, 1))()
        lib.gdp_mesh_round_stats(self._h, arr, n.value, C.byref(n))
        return [{f: getattr(arr[i], f) for f in STAT_FIELDS} for i in range(n.value)]

    def kernel_profile(self) -> list[dict]:
        lib = load()
        n = C.c_int32(0)
        arr = (gdp_kernel_prof * 32)()
        self.ctx.check(lib.gdp_mesh_kernel_profile(self._h, arr, 32, C.byref(n)))
        return [{"name": arr[i].name.decode(), "launches": arr[i].launches, "total_ms": arr[i].total_ms,
                 "items": arr[i].items, "alg_bytes": arr[i].alg_bytes} for i in range(n.value)]

    def assign_from(self, src: "Mesh"):
        self.ctx.check(load().gdp_mesh_assign(self.ctx._h, self._h, src._h))

    def clone(self) -> "Mesh":
        h = _VP()
        self.ctx.check(load().gdp_mesh_clone(self.ctx._h, self._h, C.byref(h)))
        return Mesh(self.ctx, h)

    def last_refine_ms(self) -> float:
        ms = C.c_double(0)
        load().gdp_mesh_last_refine_ms(self._h, C.byref(ms))
        return ms.value


def gdp_mesh_create(ctx: Context, xy, seg) -> Mesh:
    p, keep = _pslg(xy, seg)
    h = _VP()
    ctx.check(load().gdp_mesh_create(ctx._h, C.byref(p), C.byref(h)))
    return Mesh(ctx, h)


def gdp_mesh_create_device(ctx: Context, xy, seg) -> Mesh:
    """Line 1 on the GPU: the same canonical CDT as gdp_mesh_create, built by kernels."""
    p, keep = _pslg(xy, seg)
    h = _VP()
    ctx.check(load().gdp_mesh_create_device(ctx._h, C.byref(p), C.byref(h)))
    return Mesh(ctx, h)


def gdp_mesh_upload(ctx: Context, arrays: dict, n_input_v: int, n_input_s: int, rounds: int = 0) -> Mesh:
    a = {k: np.ascontiguousarray(v) for k, v in arrays.items()}
    xy = np.ascontiguousarray(a["xy"], np.float64)
    vk = np.ascontiguousarray(a["vkind"], np.int32)
    tv = np.ascontiguousarray(a["tv"], np.int32)
    tn = np.ascontiguousarray(a["tn"], np.int32)
    ts = np.ascontiguousarray(a["ts"], np.int32)
    sv = np.ascontiguousarray(a["sv"], np.int32)
    sp = np.ascontiguousarray(a["sparent"], np.int32)
    pe = np.ascontiguousarray(a["spend"], np.uint8)
    h = _VP()
    ctx.check(load().gdp_mesh_upload(ctx._h, xy.shape[0], n_input_v, _ptr(xy, C.c_double), _ptr(vk, C.c_int32),
                                     tv.shape[0], _ptr(tv, C.c_int32), _ptr(tn, C.c_int32), _ptr(ts, C.c_int32),
                                     sv.shape[0], n_input_s, _ptr(sv, C.c_int32), _ptr(sp, C.c_int32),
                                     _ptr(pe, C.c_uint8), rounds, C.byref(h)))
    return Mesh(ctx, h)


def gdp_mesh_refine(ctx: Context, mesh: Mesh, ratio_bound_sq: float, params: gdp_params | None = None,
                    allow_noterm: bool = False) -> int:
    prm = params if params is not None else make_params()
    rc = load().gdp_mesh_refine(ctx._h, mesh._h, float(ratio_bound_sq), C.byref(prm))
    return ctx.check(rc, ok=(GDP_OK, -5) if allow_noterm else (GDP_OK,))


def gdp_refine_batch(ctx: Context, inputs, ratio_bound_sq, params: gdp_params | None = None):
    """Batched form: inputs is a list of (xy, seg) pairs, ratio_bound_sq a list
    of bounds.  Returns (meshes, statuses, elapsed_ms); meshes[i] is None when
    statuses[i] is an error."""
    n = len(inputs)
    keep, arr = [], (gdp_pslg * max(n, 1))()
    for i, (xy, seg) in enumerate(inputs):
        p, k = _pslg(xy, seg)
        arr[i] = p
        keep.append(k)
    bsq = np.ascontiguousarray(np.asarray(ratio_bound_sq, dtype=np.float64).reshape(-1))
    if bsq.shape[0] != n:
        raise ValueError("one bound per input")
    prm = params if params is not None else make_params()
    outs = (_VP * max(n, 1))()
    st = (C.c_int * max(n, 1))()
    ms = C.c_double(0.0)
    ctx.check(load().gdp_refine_batch(ctx._h, arr, _ptr(bsq, C.c_double), C.byref(prm), n, outs, st, C.byref(ms)))
    meshes = [Mesh(ctx, _VP(outs[i])) if outs[i] else None for i in range(n)]
    return meshes, [int(st[i]) for i in range(n)], ms.value


GDP_E_BUSY = -7


class Server:
    """Serving form: jobs arrive while others run; each finished job yields a
    device-resident Mesh."""

    def __init__(self, ctx: Context, hbm_budget: int, max_slots: int, engine_max_vertices: int | None = None,
                 mode: int = 0, rounds_per_group: int = 0, line1: tuple[int, int] | None = None):
        self.ctx = ctx
        self._h = _VP()
        ctx.check(load().gdp_server_create(ctx._h, int(hbm_budget), int(max_slots), C.byref(self._h)))
        if mode or rounds_per_group:
            self.ctx.check(load().gdp_server_mode(self._h, int(mode), int(rounds_per_group)))
        if engine_max_vertices is not None:
            self.engine_jobs(engine_max_vertices)
        if line1 is not None:
            self.line1(*line1)

    def line1(self, host_threads: int, device_min_vertices: int) -> None:
        """Line 1 runs in the server after arrival: on host_threads library threads, or on the
        device for jobs with at least device_min_vertices input vertices (0: never)."""
        self.ctx.check(load().gdp_server_line1(self._h, int(host_threads), int(device_min_vertices)))

    def engine_jobs(self, max_input_vertices: int) -> None:
        """Jobs up to this many input vertices run in batched single-workgroup launches (0: never)."""
        self.ctx.check(load().gdp_server_engine_jobs(self._h, int(max_input_vertices)))

    def prepare(self, xy, seg, ratio_bound_sq: float, params: gdp_params | None = None) -> int:
        p, keep = _pslg(xy, seg)
        prm = params if params is not None else make_params()
        job = C.c_uint64(0)
        self.ctx.check(load().gdp_server_prepare(self._h, C.byref(p), float(ratio_bound_sq), C.byref(prm),
                                                 C.byref(job)))
        return job.value

    def arrive(self, job: int) -> None:
        self.ctx.check(load().gdp_server_arrive(self._h, C.c_uint64(job)))

    def submit(self, xy, seg, ratio_bound_sq: float, params: gdp_params | None = None) -> int:
        job = self.prepare(xy, seg, ratio_bound_sq, params)
        self.arrive(job)
        return job

    def _take(self, fn, job: int):
        h = _VP()
        t = gdp_job_times()
        rc = fn(self._h, C.c_uint64(job), C.byref(h), C.byref(t))
        times = {"submit_ms": t.submit_ms, "line1_ms": t.line1_ms, "admit_ms": t.admit_ms, "done_ms": t.done_ms}
        if rc == GDP_E_BUSY:
            return None, rc, times
        return (Mesh(self.ctx, h) if h.value else None), rc, times

    def poll(self, job: int):
        """(mesh or None, status, times); status GDP_E_BUSY while pending."""
        return self._take(load().gdp_server_poll, job)

    def wait(self, job: int):
        return self._take(load().gdp_server_wait, job)

    def close(self):
        if getattr(self, "_h", None):
            load().gdp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gdp_refine(ctx: Context, xy, seg, ratio_bound_sq: float, params: gdp_params | None = None) -> Mesh:
    p, keep = _pslg(xy, seg)
    prm = params if params is not None else make_params()
    h = _VP()
    ctx.check(load().gdp_refine(ctx._h, C.byref(p), float(ratio_bound_sq), C.byref(prm), C.byref(h)))
    return Mesh(ctx, h)
