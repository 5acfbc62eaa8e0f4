"""Helpers shared by the GPU parity tests: run the oracle and the HIP path on
the same seeded input and compare every array element by element."""
from __future__ import annotations

import numpy as np

COMMON_STATS = ["n_enc", "n_bad", "n_kept_mid", "n_kept_cc", "n_blocked", "n_coincident", "n_enc_reject",
                "n_mid_cand", "n_unsplittable", "n_fan_invalid", "n_lost_mark", "n_dep_drop", "n_ins_mid",
                "n_ins_cc", "cav_tri_total", "cav_max", "n_f1_drop", "n_f2_drop"]


def oracle_run(pslg, cand_cap_K=0, priority_mode=0, max_rounds=0, prefilter_f1=0, cavity_approx_n=0,
               encroach_mode=0, max_edge_len_sq=0.0, split_mode=0, insert_mode=0):
    import oracle
    m = oracle.build_cdt(pslg.xy, pslg.seg)
    rc = oracle.refine(m, pslg.ratio_bound_sq, cand_cap_K=cand_cap_K, priority_mode=priority_mode, raise_on_error=False,
                       max_rounds=max_rounds, prefilter_f1=prefilter_f1, cavity_approx_n=cavity_approx_n,
                       encroach_mode=encroach_mode, max_edge_len_sq=max_edge_len_sq, split_mode=split_mode,
                       insert_mode=insert_mode)
    return m, rc


def gpu_run(ctx, pslg, cand_cap_K=0, priority_mode=0, max_rounds=0, block_size=256, prefilter_f1=0,
            cavity_approx_n=0, reserve_mode=0, rounds_per_sync=0, tail_engine_max=0, encroach_mode=0,
            max_edge_len_sq=0.0, split_mode=0, cavity_thread_cap=0, insert_mode=0):
    from paper_2007_00324_amd import gdp2d
    mesh = gdp2d.gdp_mesh_create(ctx, pslg.xy, pslg.seg)
    prm = gdp2d.make_params(cand_cap_K=cand_cap_K, priority_mode=priority_mode, max_rounds=max_rounds,
                            block_size=block_size, prefilter_f1=prefilter_f1, cavity_approx_n=cavity_approx_n,
                            reserve_mode=reserve_mode, rounds_per_sync=rounds_per_sync,
                            tail_engine_max=tail_engine_max, encroach_mode=encroach_mode,
                            max_edge_len_sq=max_edge_len_sq, split_mode=split_mode,
                            cavity_thread_cap=cavity_thread_cap, insert_mode=insert_mode)
    rc = gdp2d.gdp_mesh_refine(ctx, mesh, pslg.ratio_bound_sq, prm, allow_noterm=True)
    return mesh, rc


def diff_arrays(a: dict, b: dict) -> list[str]:
    """Names of arrays that differ (coordinates compared bitwise)."""
    bad = []
    for k in ["xy", "vkind", "tv", "tn", "ts", "sv", "sparent", "spend"]:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        if x.shape != y.shape:
            bad.append(f"{k}: shape {x.shape} vs {y.shape}")
            continue
        if k == "xy":
            same = np.array_equal(x.view(np.uint64), y.view(np.uint64))
        else:
            same = np.array_equal(x.astype(np.int64), y.astype(np.int64))
        if not same:
            idx = np.argwhere(x != y)
            bad.append(f"{k}: {len(idx)} differences, first at {idx[0].tolist()}")
    return bad


def diff_stats(orc_stats: list[dict], gpu_stats: list[dict]) -> list[str]:
    out = []
    if len(orc_stats) != len(gpu_stats):
        out.append(f"rounds {len(orc_stats)} vs {len(gpu_stats)}")
    for r, (s, g) in enumerate(zip(orc_stats, gpu_stats)):
        for f in COMMON_STATS:
            if s[f] != g[f]:
                out.append(f"round {r + 1} {f}: oracle {s[f]} gpu {g[f]}")
        if len(out) > 20:
            break
    return out


ARRAY_KEYS = ["xy", "vkind", "tv", "tn", "ts", "sv", "sparent", "spend"]


def mesh_digest(a: dict) -> str:
    """SHA-256 over the mesh arrays in a fixed order and dtype (coordinates as
    their IEEE bit patterns), so two meshes compare bit for bit by digest."""
    import hashlib
    h = hashlib.sha256()
    for k in ARRAY_KEYS:
        x = np.asarray(a[k])
        x = x.view(np.uint64) if k == "xy" else x.astype(np.int64)
        h.update(k.encode())
        h.update(np.asarray(x.shape, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(x).tobytes())
    return h.hexdigest()


def batch_instance_with_oracle(args):
    """Worker (a spawned process that never touches the GPU): one instance of
    the batched workload and the digest of the oracle's refined mesh."""
    import workloads
    n, bsq, seed = args
    p = workloads.batch_instance(n, bsq, seed)
    om, rc = oracle_run(p)
    return p.xy, p.seg, p.ratio_bound_sq, rc, mesh_digest(om.arrays()), om.rounds
