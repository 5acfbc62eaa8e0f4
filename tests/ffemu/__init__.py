"""Sequential host run of the Flip-Flop steps (gdp_ff_core.h), driven from a
point set S that the oracle's Flip-Flop round chose (test infrastructure).

The library is built from ff_emu.cpp with hipcc as plain host code."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CORE = os.path.join(HERE, "..", "..", "paper_2007_00324_amd", "csrc")
LIB = os.path.join(HERE, "libffemu.so")
_lib = None


def build() -> str:
    tmp = f"{LIB}.{os.getpid()}.tmp"  # test workers may build at the same time
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-O2", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-I", CORE, "-o", tmp, os.path.join(HERE, "ff_emu.cpp")]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        srcs = [os.path.join(HERE, "ff_emu.cpp"), os.path.join(HERE, "__init__.py"), os.path.join(CORE, "gdp_ff_core.h"), os.path.join(CORE, "gdp_exact.h")]
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(s) for s in srcs):
            build()
        _lib = C.CDLL(LIB)
        I = C.POINTER(C.c_int32)
        D = C.POINTER(C.c_double)
        _lib.ffemu_round.argtypes = [C.c_int32] * 4 + [D, I, C.c_int32, I, I, I, C.c_int32, I, I, I, C.c_int32,
                                                       C.c_int32, C.c_int32, D, I, I, C.c_int32, I, I,
                                                       C.POINTER(C.c_int64), C.c_int32, C.c_uint64]
        _lib.ffemu_round.restype = C.c_int32
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def last_points(orc_lib):
    orc_lib.orc_ff_last_points.restype = C.c_int64
    orc_lib.orc_ff_last_points.argtypes = [C.c_int64] + [C.c_void_p] * 7
    orc_lib.orc_ff_last_flagged.restype = C.c_int64
    orc_lib.orc_ff_last_flagged.argtypes = [C.c_int64, C.c_void_p]
    n = orc_lib.orc_ff_last_points(0, None, None, None, None, None, None, None)
    xy = np.zeros((max(n, 1), 2))
    cls, idx, c0, c1, edge = (np.zeros(max(n, 1), np.int32) for _ in range(5))
    key = np.zeros(max(n, 1), np.uint64)
    orc_lib.orc_ff_last_points(n, _ptr(xy, C.c_double), _ptr(cls, C.c_int32), _ptr(idx, C.c_int32),
                               _ptr(c0, C.c_int32), _ptr(c1, C.c_int32), _ptr(edge, C.c_int32),
                               _ptr(key, C.c_uint64))
    nf = orc_lib.orc_ff_last_flagged(0, None)
    ks = np.zeros(max(nf, 1), np.int32)
    orc_lib.orc_ff_last_flagged(nf, _ptr(ks, C.c_int32))
    return dict(n=n, xy=xy[:n], cls=cls[:n], id=idx[:n], c0=c0[:n], c1=c1[:n], edge=edge[:n], key=key[:n],
                flagged=ks[:nf])


def round_from_points(arr: dict, n_input_v: int, S: dict, enc_mode: int = 0, cand_cap: int = 0, order_seed: int = 0):
    """Runs Line 8 on mesh arrays `arr` (oracle layout) for the points S.
    Returns (arrays in oracle layout, counters)."""
    lib = load()
    xy = np.ascontiguousarray(arr["xy"], dtype=np.float64)
    nV = xy.shape[0]
    tv3 = np.asarray(arr["tv"], np.int32).reshape(-1, 3)
    tn3 = np.asarray(arr["tn"], np.int32).reshape(-1, 3)
    ts3 = np.asarray(arr["ts"], np.int32).reshape(-1, 3)
    nT = tv3.shape[0]
    sv = np.asarray(arr["sv"], np.int32).reshape(-1, 2)
    nS = sv.shape[0]
    np_ = S["n"]
    capV, capT, capS = nV + np_ + 8, nT + 2 * np_ + 8, nS + np_ + 8
    X = np.zeros((capV, 2)); X[:nV] = xy
    K = np.zeros(capV, np.int32); K[:nV] = np.asarray(arr["vkind"])
    TV = np.zeros((capT, 4), np.int32); TN = np.zeros((capT, 4), np.int32); TS = np.zeros((capT, 4), np.int32)
    TV[:nT, :3] = tv3; TN[:nT, :3] = tn3; TS[:nT, :3] = ts3
    TV[:nT, 3] = (ts3[:, 0] >= 0) * 1 + (ts3[:, 1] >= 0) * 2 + (ts3[:, 2] >= 0) * 4
    SV = np.zeros((capS, 2), np.int32); SV[:nS] = sv
    SP = np.zeros(capS, np.int32); SP[:nS] = np.asarray(arr["sparent"])
    SE = np.zeros(capS, np.int32); SE[:nS] = np.asarray(arr["spend"])
    # directed edge -> (triangle, edge index)
    edge_of = {}
    for t in range(nT):
        for i in range(3):
            edge_of[(int(tv3[t, i]), int(tv3[t, (i + 1) % 3]))] = (t, i)
    pinfo = np.zeros((max(np_, 1), 4), np.int32)
    pab = np.zeros((max(np_, 1), 2), np.int32)
    nmid = int(np.sum(S["cls"] == 1))
    for r in range(np_):
        if S["cls"][r] == 1:
            k = int(S["id"][r])
            a, b = int(sv[k, 0]), int(sv[k, 1])
            s0 = edge_of.get((a, b)); s1 = edge_of.get((b, a))
            pinfo[r] = (1, k, s0[0] * 4 + s0[1] if s0 else -1, s1[0] * 4 + s1[1] if s1 else -1)
            pab[r] = (a, b)
        else:
            pinfo[r] = (0, int(S["edge"][r]), int(S["c0"][r]), int(S["c1"][r]))
    mid_elem = np.ascontiguousarray(S["flagged"], np.int32)
    mid_state = np.zeros(max(len(mid_elem), 1), np.int32)
    out = np.zeros(16, np.int64)
    pxy = np.ascontiguousarray(S["xy"], np.float64).reshape(-1)
    if pxy.size == 0:
        pxy = np.zeros(2)
    rc = lib.ffemu_round(nV, nT, nS, enc_mode, _ptr(X, C.c_double), _ptr(K, C.c_int32), capV,
                         _ptr(TV, C.c_int32), _ptr(TN, C.c_int32), _ptr(TS, C.c_int32), capT,
                         _ptr(SV, C.c_int32), _ptr(SP, C.c_int32), _ptr(SE, C.c_int32), capS,
                         np_, nmid, _ptr(pxy, C.c_double), _ptr(pinfo, C.c_int32), _ptr(pab, C.c_int32),
                         len(mid_elem), _ptr(mid_elem if len(mid_elem) else np.zeros(1, np.int32), C.c_int32),
                         _ptr(mid_state, C.c_int32), _ptr(out, C.c_int64), cand_cap, order_seed)
    nV2, nT2, nS2 = int(out[0]), int(out[1]), int(out[2])
    res = dict(xy=X[:nV2].copy(), vkind=K[:nV2].copy(), tv=TV[:nT2, :3].copy(), tn=TN[:nT2, :3].copy(),
               ts=TS[:nT2, :3].copy(), sv=SV[:nS2].copy(), sparent=SP[:nS2].copy(), spend=SE[:nS2].astype(np.uint8))
    cnt = dict(rc=rc, iters=int(out[3]), flips=int(out[4]), removals=int(out[5]), dep=int(out[6]),
               enc=int(out[7]), flags=int(out[8]), err=int(out[9]), passes=int(out[10]), where=int(out[11]))
    return res, cnt
