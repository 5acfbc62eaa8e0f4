#!/usr/bin/env python3
"""Benchmark of the gfx950 refinement loop (Algorithm 1, Lines 2-9).

One step = one complete refinement of the 1,000,000-point PSLG (uniform /
Gaussian-cluster / jittered-ellipse thirds, 50,000 k-nearest-neighbour
segments, unit-square boundary, B = sqrt(2)) starting from its initial CDT,
which is already resident in device memory (Line 1 runs once on the host and
is not timed, as in the paper's measurements).  Each step copies the resident
initial mesh into a working mesh on the device and refines it to the end.

Prints one JSON line:  value = Steiner points per second; the line also
carries output triangles per second, a roofline object for the dominant
kernel (HIP-event timed in a separate profiled pass) and the oracle's CPU
rate on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "Steiner pts/s + output tris/s, 1M-vertex PSLG B=√2; batched jobs/s vs plain"
HBM_PEAK_GBS = 8000.0
HERE = os.path.dirname(os.path.abspath(__file__))
ROOFLINE_KERNEL = "k_cavity_cc"
# HBM traffic of the roofline kernel measured with rocprofv3 (FETCH_SIZE and
# WRITE_SIZE, scaled by a plain-copy calibration), with the hash of the kernel
# sources it was measured on.
TRAFFIC_FILE = os.path.join(HERE, "profiles", "k_cavity_cc_c1_1M.md")
KERNEL_SOURCES = ["gdp_kernels.hip", "gdp_kernels.h", "gdp_internal.h", "gdp_exact.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_2007_00324_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """Bytes per launch from the committed counter summary, or None if the
    kernel sources changed since it was taken (or there is none)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        line = line.strip().strip("`")
        for key in ("traffic_bytes_per_launch", "kernel_sources_sha256"):
            if line.startswith(key + ":"):
                vals[key] = line.split(":", 1)[1].strip()
    if vals.get("kernel_sources_sha256") != kernel_source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def loop_alg_bytes(tot: dict) -> float:
    """What a sequential Bowyer-Watson insertion of the same points must
    touch, from the winners' sums: per cavity triangle its record (36 B) and
    its mark (16 B); per fan edge the incircle test outside (28 B), the new
    triangle (36 B), the outside neighbour's repair (16 B) and the next
    round's quality test of the new triangle (60 B); per walk step 52 B; per
    inserted vertex 20 B."""
    ins = tot.get("n_ins_mid", 0) + tot.get("n_ins_cc", 0)
    return (52.0 * tot.get("win_cav_tri", 0) + 140.0 * tot.get("win_fan_edges", 0)
            + 52.0 * tot.get("win_walk_steps", 0) + 20.0 * ins)


def atomic_peak(ctx) -> dict:
    """Random-slot 64-bit atomicMax throughput on a table the size of the
    1M-point mesh's mark array (the conflict step's pattern)."""
    from paper_2007_00324_amd import gdp2d
    slots, ops = 6_000_000, 256_000_000
    ms = gdp2d.gdp_bench_atomic_max(ctx, slots, ops)
    return {"bench": f"{ops:,} atomicMax on random slots of a {slots:,}-word table", "ms": ms,
            "gatomic_per_s": ops / (ms / 1000.0) / 1e9}


def host_cpu() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(p, n_points: int, n_segments: int) -> dict:
    """Times the oracle (one thread) on the same workload (p) when n_points is
    its size, else on the same generator at n_points."""
    import oracle
    import workloads
    if n_points != p.n_vertices - 4:
        p = workloads.scaled_config1(n_points, n_segments, seed=1)
    m = oracle.build_cdt(p.xy, p.seg)
    t0 = time.perf_counter()
    oracle.refine(m, p.ratio_bound_sq)
    dt = time.perf_counter() - t0
    steiner = m.nV - p.n_vertices
    return {
        "value": steiner / dt,
        "unit": "Steiner points/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle refinement (initial CDT excluded), one thread, of {p.name}: {p.n_vertices:,} vertices / "
                   f"{p.n_segments:,} segments -> {steiner:,} Steiner points, {m.nT:,} output triangles in {dt:.2f} s"),
        "output_triangles_per_s": m.nT / dt,
        **host_cpu(),
    }


def criteria_leg(ctx, init, work, p) -> dict:
    """The other quality criteria of Section 4.1 on the same resident initial CDT:
    Chew's diametric lenses, concentric-shell subsegment splitting, an edge-length
    bound l, and the angle bound theta = 20
    degrees of Table 1 (B^2 = 1 / (4 sin^2 theta)); each refinement timed alone
    (one warmup, then the median of three), with the bad-area measure of the
    result under its own criteria."""
    import math

    from paper_2007_00324_amd import gdp2d
    theta20 = 1.0 / (4.0 * math.sin(math.radians(20.0)) ** 2)
    modes = [
        ("ruppert_B=sqrt2", p.ratio_bound_sq, dict()),
        ("chew_lens_B=sqrt2", p.ratio_bound_sq, dict(encroach_mode=1)),
        ("concentric_shells_B=sqrt2", p.ratio_bound_sq, dict(split_mode=1)),
        ("ruppert_B=sqrt2_l=0.001", p.ratio_bound_sq, dict(max_edge_len_sq=1e-6)),
        ("ruppert_theta=20deg", theta20, dict()),
        ("chew_lens_theta=20deg_l=0.001", theta20, dict(encroach_mode=1, max_edge_len_sq=1e-6)),
    ]
    rows = []
    n_in = init.info()["n_vertices"]
    for name, bsq, kw in modes:
        prm = gdp2d.make_params(**kw)
        ms = []
        for rep in range(4):
            work.assign_from(init)
            gdp2d.gdp_mesh_refine(ctx, work, bsq, prm)
            if rep:
                ms.append(work.last_refine_ms())
        ms.sort()
        info = work.info()
        steiner = info["n_vertices"] - n_in
        n_bad, bad_area = work.quality(bsq, kw.get("max_edge_len_sq", 0.0))
        row = {"mode": name, "ratio_bound_sq": bsq, **kw, "refine_ms": ms[1], "steiner_points": steiner,
               "output_triangles": info["n_triangles"], "rounds": info["rounds"],
               "steiner_per_s": steiner / (ms[1] / 1000.0), "bad_triangles": n_bad, "bad_area": bad_area}
        log(f"criteria {name}: {ms[1]:.2f} ms, {steiner:,} Steiner points, {info['rounds']} rounds, "
            f"{n_bad} bad triangles covering {bad_area:.3e}")
        rows.append(row)
    return {"workload": "the 1M-point PSLG above, same initial CDT", "timing": "device refine time, median of 3",
            "modes": rows}


def flipflop_leg(ctx, init, work, p) -> dict:
    """Line 8 by Flip-Flop insertion (Section 4.3, with the slot-independent keys
    of priority mode 2) against cavity insertion (default keys) on the same
    resident initial CDT: device refine time (median of 3 after a warmup), time per
    round, and points kept per point added (Flip-Flop adds every point of S
    and takes the redundant ones out again; cavity insertion decides before it
    writes).  The Line 7 filter (n-triangle approximate cavities, Section 4.3)
    runs before Line 8 in two of the rows: it exists to keep dependent points
    from being added only to be removed again."""
    from paper_2007_00324_amd import gdp2d
    rows = []
    n_in = init.info()["n_vertices"]
    ff = dict(priority_mode=2, insert_mode=1)
    for name, kw in [("cavity", dict()), ("flipflop", ff), ("flipflop+F2_n=4", dict(ff, cavity_approx_n=4)),
                     ("flipflop+F2_n=8", dict(ff, cavity_approx_n=8))]:
        prm = gdp2d.make_params(**kw)
        ms = []
        for rep in range(4):
            work.assign_from(init)
            gdp2d.gdp_mesh_refine(ctx, work, p.ratio_bound_sq, prm)
            if rep:
                ms.append(work.last_refine_ms())
        ms.sort()
        info = work.info()
        st = work.round_stats()
        steiner = info["n_vertices"] - n_in
        row = {"insertion": name, "refine_ms": ms[1], "rounds": info["rounds"],
               "ms_per_round": ms[1] / max(1, info["rounds"]), "steiner_points": steiner,
               "steiner_per_s": steiner / (ms[1] / 1000.0), "output_triangles": info["n_triangles"]}
        if name.startswith("flipflop"):
            added = sum(r["n_ff_points"] for r in st)
            row.update({"points_added": added, "kept_per_added": steiner / max(1, added),
                        "flips": sum(r["n_flips"] for r in st), "flip_passes": sum(r["n_flip_passes"] for r in st),
                        "removals": sum(r["n_removals"] for r in st),
                        "removal_passes": sum(r["n_removal_passes"] for r in st),
                        "f2_dropped": sum(r["n_f2_drop"] for r in st),
                        "cdts_examined": sum(r["n_ff_iters"] for r in st)})
        else:
            cands = sum(r["n_kept_cc"] + r["n_mid_cand"] for r in st)
            row.update({"candidates": cands, "kept_per_candidate": steiner / max(1, cands)})
        log(f"flip-flop leg {name}: {ms[1]:.2f} ms, {info['rounds']} rounds, {steiner:,} Steiner points")
        rows.append(row)
    return {"workload": "the 1M-point PSLG above, same initial CDT", "timing": "device refine time, median of 3",
            "rows": rows}


def cdt_leg(ctx, init, p) -> dict:
    """Line 1 of Algorithm 1 on the GPU (gdp_mesh_create_device) against the host
    builder (gdp_mesh_create) on the benchmark PSLG: wall time from the PSLG in host
    memory to the initial CDT resident in device memory, both including the copy of
    their inputs (host: the finished CDT; device: the points and segments); one warmup,
    then the median of three.  The two meshes must be identical element by element."""
    import numpy as np

    from paper_2007_00324_amd import gdp2d
    host_ms, dev_ms = [], []
    info = None
    for rep in range(4):
        t0 = time.perf_counter()
        h = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)
        t1 = time.perf_counter()
        d = gdp2d.gdp_mesh_create_device(ctx, p.xy, p.seg)
        t2 = time.perf_counter()
        if rep:
            host_ms.append(1e3 * (t1 - t0))
            dev_ms.append(1e3 * (t2 - t1))
        if rep == 3:
            a, b = init.arrays(), d.arrays()
            identical = all(np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8))
                            for k in ["xy", "vkind", "tv", "tn", "ts", "sv", "sparent", "spend"])
            info = d.info()
        del h, d
    host_ms.sort()
    dev_ms.sort()
    log(f"initial CDT: host {host_ms[1]:.1f} ms, device {dev_ms[1]:.1f} ms, "
        f"{info['cdt_point_rounds']} + {info['cdt_segment_rounds']} rounds, identical {identical}")
    return {"workload": f"{p.name}: {p.n_vertices:,} vertices / {p.n_segments:,} segments",
            "timing": "wall time, PSLG in host memory to CDT in device memory, median of 3",
            "host_ms": host_ms[1], "device_ms": dev_ms[1], "speedup": host_ms[1] / dev_ms[1],
            "point_rounds": info["cdt_point_rounds"], "segment_rounds": info["cdt_segment_rounds"],
            "triangles": info["n_triangles"], "identical_to_host": identical}


ABLATION_SETTINGS = [
    ("base", dict()),
    ("K=65536", dict(cand_cap_K=65536)),
    ("K=16384", dict(cand_cap_K=16384)),
    ("F1", dict(prefilter_f1=1)),
    ("F2_n=2", dict(cavity_approx_n=2)),
    ("F2_n=4", dict(cavity_approx_n=4)),
    ("F1+F2_n=4", dict(prefilter_f1=1, cavity_approx_n=4)),
    ("no_single_workgroup_rounds", dict(tail_engine_max=-1)),
]
# Rule 3 (the cooperative path for large cavities) on the circles input, whose
# circle interiors make cavities of hundreds of triangles: per-thread slices of
# 12, 24 or 39 (the default) slots before a cavity goes cooperative.
COOP_SETTINGS = [("coop_cap_39", dict(cavity_thread_cap=39)), ("coop_cap_24", dict(cavity_thread_cap=24)),
                 ("coop_cap_12", dict(cavity_thread_cap=12))]
ABLATION_TRAFFIC_FILE = os.path.join(HERE, "profiles", "ablation_traffic.md")


def recorded_setting_traffic() -> dict:
    """HBM bytes per refine of each ablation setting from the committed counter
    summary, if the kernel sources still hash to the recorded value."""
    try:
        with open(ABLATION_TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return {}
    out, sha = {}, None
    for line in text.splitlines():
        line = line.strip().strip("`")
        if line.startswith("kernel_sources_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("setting_traffic:"):
            name, val = line.split(":", 1)[1].rsplit("=", 1)
            out[name.strip()] = float(val)
    return out if sha == kernel_source_hash() else {}


def pmc_sum(fetch_dir: str, write_dir: str, fetch_scale: float, write_scale: float,
            match: str = r"gdp::(k|kf|kg)_") -> dict:
    """HBM bytes of the refinement's own kernels from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by what the
    counter reads for a plain copy of known size."""
    import csv
    import glob
    import re
    mine = re.compile(match)
    tot = {}
    for d, name in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        kib = 0.0
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row.get("Counter_Name") == name and mine.search(row.get("Kernel_Name", "")):
                        kib += float(row["Counter_Value"])
        tot[name] = kib
    b = tot["FETCH_SIZE"] * 1024 * fetch_scale + tot["WRITE_SIZE"] * 1024 * write_scale
    return {"fetch_kib": tot["FETCH_SIZE"], "write_kib": tot["WRITE_SIZE"], "bytes": b}


def ablation_leg(ctx, init, work, p, init2=None, p2=None) -> dict:
    """gDP2d's rules switched on and off on the 1M-point PSLG (the paper leaves this
    study out for 2D), and the cooperative path's capacity on the circles input.
    Per setting: device refine time (median of 3), Steiner points, rounds, and the
    Rule 2 quantities: alpha = insertions / candidates given to threads (effective
    concurrency without a filter), beta = the same with it, and l / L = the filter
    kernels' share of the profiled time.  Rule 2 predicts a gain iff
    (L + l) / L < beta / alpha.  The extended prediction adds the fixed cost of a
    round (c, the time of a round of the single-workgroup tail, which is all
    latency): T = rounds * c + (T_base - rounds_base * c) * candidates / candidates_base
    + l.  The measured gain is the Steiner/s ratio.  The waste ratio is the measured
    HBM traffic of a refine (rocprofv3, per setting) over its algorithmic bytes."""
    from paper_2007_00324_amd import gdp2d
    traffic = recorded_setting_traffic()
    rows = []
    for name, kw in ABLATION_SETTINGS:
        rows.append(_ablation_row(ctx, init, work, p, name, kw, traffic))
    base = rows[0]
    # fixed cost of a round: the single-workgroup tail's time per round (pure latency)
    c = base.get("tail_ms_per_round") or 0.0
    for row in rows[1:]:
        row["rule2_beta_over_alpha"] = row["concurrency_fraction"] / base["concurrency_fraction"]
        row["rule2_latency_ratio"] = 1.0 + row["filter_share"]
        row["rule2_predicts_gain"] = row["rule2_latency_ratio"] < row["rule2_beta_over_alpha"]
        work_ms = max(base["refine_ms"] - base["rounds"] * c, 1e-9)
        pred_ms = row["rounds"] * c + work_ms * row["candidates"] / max(base["candidates"], 1) + row["filter_ms"]
        row["rule2_extended_predicted_gain"] = base["refine_ms"] / pred_ms
        row["measured_gain"] = row["steiner_per_s"] / base["steiner_per_s"]
        log(f"ablation {row['setting']}: gain {row['measured_gain']:.3f} (Rule 2 predicts {row['rule2_predicts_gain']}, "
            f"extended {row['rule2_extended_predicted_gain']:.3f})")
    out = {"workload": "the 1M-point PSLG above, same initial CDT", "timing": "device refine time, median of 3",
           "round_fixed_cost_ms": c, "settings": rows}
    if init2 is not None:
        w2 = init2.clone()
        coop = [_ablation_row(ctx, init2, w2, p2, name, kw, traffic) for name, kw in COOP_SETTINGS]
        for row in coop[1:]:
            row["measured_gain"] = row["steiner_per_s"] / coop[0]["steiner_per_s"]
        out["cooperative_path"] = {"workload": f"{p2.name}: {p2.n_vertices:,} vertices / {p2.n_segments:,} segments "
                                               "(512 closed 1000-gons + 100,000 free points)",
                                   "settings": coop}
    return out


def _ablation_row(ctx, init, work, p, name, kw, traffic) -> dict:
    from paper_2007_00324_amd import gdp2d
    filt_kernels = {"k_cap", "k_prefilter"}
    n_in = init.info()["n_vertices"]
    work.assign_from(init)
    gdp2d.gdp_mesh_refine(ctx, work, p.ratio_bound_sq, gdp2d.make_params(profile_kernels=1, **kw))
    profs = [k for k in work.kernel_profile() if k["launches"]]
    prof = {k["name"]: k["total_ms"] for k in profs}
    eng = next((k for k in profs if k["name"] == "k_engine"), None)
    rs = work.round_stats()
    tot = {k: sum(r[k] for r in rs) for k in rs[0]} if rs else {}
    attempts = sum(r["n_kept_cc"] + r["n_kept_mid"] for r in rs)
    useful = sum(r["n_ins_cc"] + r["n_ins_mid"] for r in rs)
    big = sum(r["n_big_cavities"] for r in rs)
    filt_ms = sum(v for k, v in prof.items() if k in filt_kernels)
    tot_ms = sum(prof.values())
    ms = []
    prm = gdp2d.make_params(**kw)
    for rep in range(4):
        work.assign_from(init)
        gdp2d.gdp_mesh_refine(ctx, work, p.ratio_bound_sq, prm)
        if rep:
            ms.append(work.last_refine_ms())
    ms.sort()
    steiner = work.info()["n_vertices"] - n_in
    alg = loop_alg_bytes(tot)
    row = {"setting": name, **kw, "refine_ms": ms[1], "steiner_points": steiner, "rounds": work.info()["rounds"],
           "steiner_per_s": steiner / (ms[1] / 1000.0), "candidates": attempts, "insertions": useful,
           "concurrency_fraction": useful / max(attempts, 1), "filter_ms": filt_ms,
           "filter_share": filt_ms / max(tot_ms - filt_ms, 1e-9), "big_cavities": big,
           "alg_bytes": alg, "traffic_bytes": traffic.get(name),
           "waste_ratio": (traffic[name] / alg) if name in traffic and alg else None}
    if eng is not None:
        tail_rounds = max(1, len([r for r in rs]) - (prof_rounds_grid(profs)))
        row["tail_ms_per_round"] = eng["total_ms"] / tail_rounds
    log(f"ablation {name}: {ms[1]:.2f} ms, {steiner:,} Steiner, {row['rounds']} rounds, "
        f"alpha {row['concurrency_fraction']:.3f}, filter {filt_ms:.2f} ms, {big} cooperative cavities")
    return row


def prof_rounds_grid(profs) -> int:
    """Rounds that ran on the grid kernels (one k_locate launch each)."""
    loc = next((k for k in profs if k["name"] == "k_locate"), None)
    return loc["launches"] if loc else 0


def make_batch(count: int, workers: int):
    """The batched workload, generated by worker processes before this
    process touches the GPU."""
    import workloads
    t = time.perf_counter()
    ps = workloads.batch_config3(count, workers=workers)
    log(f"batched: generated {count:,} PSLGs ({sum(p.n_vertices for p in ps):,} vertices) in "
        f"{time.perf_counter() - t:.1f} s")
    return ps


def batched_leg(ctx, ps, plain_every: int, line1_dev_min: int = 0) -> dict:
    """Batched form: independent PSLGs refined in one persistent launch,
    against the plain per-instance loop on a sample of the same instances."""
    from paper_2007_00324_amd import gdp2d
    count = len(ps)
    nv = sum(p.n_vertices for p in ps)
    inputs = [(p.xy, p.seg) for p in ps]
    bsq = [p.ratio_bound_sq for p in ps]
    from paper_2007_00324_amd import tune_batch
    table = tune_batch.load_table()
    prm = tune_batch.tuned_params(table)
    default_prm = gdp2d.make_params()
    gdp2d.gdp_refine_batch(ctx, inputs[:8], bsq[:8], prm)  # warm-up (code objects, scratch)
    t = time.perf_counter()
    meshes, st, dev_ms = gdp2d.gdp_refine_batch(ctx, inputs, bsq, prm)
    wall = time.perf_counter() - t
    bad = sum(1 for s_ in st if s_ != 0)
    steiner = sum(m.info()["n_vertices"] - p.n_vertices for m, p in zip(meshes, ps) if m is not None)
    del meshes
    log(f"batched (tuned: engine up to {prm.batch_engine_max_v or 'all'} input vertices, shared rounds above): "
        f"{count:,} jobs, device {dev_ms:.1f} ms, call {wall:.2f} s (host CDT, upload, download), {bad} not OK")
    m2, st2, default_ms = gdp2d.gdp_refine_batch(ctx, inputs, bsq, default_prm)
    del m2
    log(f"batched (default: every mesh in the engine): device {default_ms:.1f} ms")
    line1_dev = None
    if line1_dev_min > 0:
        prm_dev = tune_batch.tuned_params(table)
        prm_dev.batch_line1_device_min_v = line1_dev_min
        t = time.perf_counter()
        m3, st3, dev3_ms = gdp2d.gdp_refine_batch(ctx, inputs, bsq, prm_dev)
        wall3 = time.perf_counter() - t
        bad3 = sum(1 for s_ in st3 if s_ != 0)
        del m3
        n_dev = sum(1 for p in ps if p.n_vertices >= line1_dev_min)
        line1_dev = {"device_min_vertices": line1_dev_min, "device_built": n_dev, "call_s": wall3,
                     "jobs_per_s_with_line1": count / wall3, "device_ms": dev3_ms, "failed": bad3}
        log(f"batched, Line 1 of the {n_dev} inputs with >= {line1_dev_min:,} vertices on the device: call "
            f"{wall3:.2f} s ({count / wall3:,.0f} jobs/s with Line 1), {bad3} not OK")
    sample = ps[::plain_every]
    plain_ms = 0.0
    for p in sample:
        m = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)
        gdp2d.gdp_mesh_refine(ctx, m, p.ratio_bound_sq, prm)
        plain_ms += m.last_refine_ms()
        m.free()
    plain_jobs_s = len(sample) / (plain_ms / 1000.0)
    jobs_s = count / (dev_ms / 1000.0)
    log(f"plain loop: {len(sample)} of the jobs in {plain_ms:.1f} ms of refinement -> {plain_jobs_s:,.0f} jobs/s")
    return {
        "workload": (f"{count:,} PSLGs: log-uniform 100..50,000 uniform points, k-nearest-neighbour segments on 5% "
                     "of the vertices, unit square, B^2 drawn from {2.0, 2.56, 4.0}; refinement from the initial "
                     "CDTs (Line 1 on the host, as for the single instance)"),
        "jobs": count,
        "input_vertices": nv,
        "steiner_points": steiner,
        "jobs_per_s": jobs_s,
        "device_ms": dev_ms,
        "tuned": {"batch_engine_max_v": prm.batch_engine_max_v, "rounds_per_group": prm.rounds_per_sync,
                  "table": "paper_2007_00324_amd/tuning/batch.json" if table else None},
        "default_jobs_per_s": count / (default_ms / 1000.0),
        "tuned_vs_default": default_ms / dev_ms,
        "jobs_per_s_with_host_cdt": count / wall,
        "line1_device": line1_dev,
        "plain_jobs_per_s": plain_jobs_s,
        "plain_sample": f"every {plain_every}th job ({len(sample)} jobs), each gdp_mesh_refine timed alone",
        "speedup_vs_plain": jobs_s / plain_jobs_s,
        "failed": bad,
    }


def serve_stream(ctx, jobs, lam, budget_gb, slots, engine_max_v, mode, rounds=0, line1=None, l1_out=None):
    """One replay of the job set as a Poisson stream of rate lam (None: every
    job arrives at once); returns latencies (ms), the achieved rate and the
    count of failed jobs.  line1 = (host threads, device threshold): Line 1
    runs in the server after arrival (l1_out receives each job's Line-1 ms)."""
    import threading
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    from paper_2007_00324_amd import gdp2d
    n = len(jobs)
    srv = gdp2d.Server(ctx, int(budget_gb * (1 << 30)), slots, engine_max_vertices=engine_max_v, mode=mode,
                       rounds_per_group=rounds, line1=line1)
    with ThreadPoolExecutor(16) as ex:  # Line 1 of every job (unless in the server) before the stream starts
        ids = list(ex.map(lambda p: srv.prepare(p.xy, p.seg, p.ratio_bound_sq), jobs))
    gaps = np.random.default_rng(7).exponential(1.0 / lam, size=n) if lam else np.zeros(n)
    results = [None] * n

    def collect():
        for k, j in enumerate(ids):
            m, rc, t = srv.wait(j)
            results[k] = (rc, t)
            if m is not None:
                m.free()
    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    due = 0.0
    for k, j in enumerate(ids):
        due += gaps[k]
        while time.perf_counter() - t0 < due:
            time.sleep(min(0.0005, max(0.0, due - (time.perf_counter() - t0))))
        srv.arrive(j)
    th.join()
    srv.close()
    lat = np.array([t["done_ms"] - t["submit_ms"] for _, t in results])
    if l1_out is not None:
        l1_out.extend(t["line1_ms"] - t["submit_ms"] for _, t in results)
    span = max(1e-9, (max(t["done_ms"] for _, t in results) - min(t["submit_ms"] for _, t in results)) / 1000.0)
    return lat, n / span, sum(1 for rc, _ in results if rc != 0)


def serving_line1_leg(ctx, jobs, budget_gb: float, slots: int, dev_min_v: int, rate_frac: float = 0.5) -> dict:
    """Serving with Line 1 inside the server (latency from the PSLG's arrival,
    initial CDT included): host threads only, against the device builder for
    jobs of at least dev_min_v input vertices.  Each setting: capacity (every
    job at once), then a Poisson stream at rate_frac of the host setting's
    capacity."""
    import numpy as np
    rows = []
    lam = None
    for name, l1 in (("host", (16, 0)), (f"device for jobs >= {dev_min_v:,} vertices", (16, dev_min_v))):
        row = {"line1": name, "host_threads": l1[0], "device_min_vertices": l1[1]}
        l1ms = []
        lat, cap, bad = serve_stream(ctx, jobs, None, budget_gb, slots, 0, 0, line1=l1, l1_out=l1ms)
        row["capacity_jobs_per_s"] = cap
        row["capacity_run"] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                               "line1_mean_ms": float(np.mean(l1ms)), "failed": bad}
        if lam is None:
            lam = cap * rate_frac
        l1ms = []
        lat, ach, bad = serve_stream(ctx, jobs, lam, budget_gb, slots, 0, 0, line1=l1, l1_out=l1ms)
        row["stream"] = {"rate_jobs_per_s": lam, "p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)), "achieved_jobs_per_s": ach,
                         "line1_mean_ms": float(np.mean(l1ms)), "line1_p99_ms": float(np.percentile(l1ms, 99)),
                         "failed": bad}
        log(f"serving, Line 1 in the server ({name}): capacity {cap:.0f} jobs/s; at {lam:.0f}/s p50 "
            f"{row['stream']['p50_ms']:.1f} ms, p99 {row['stream']['p99_ms']:.1f} ms (Line 1 mean "
            f"{row['stream']['line1_mean_ms']:.1f} ms), {bad} not OK")
        rows.append(row)
    return {"workload": "the serving job set; latency from the arrival of the PSLG (Line 1 included)",
            "settings": rows}


def serving_full_leg(count: int, rates: list, budget_gb: float, slots: int, dev_min_v: int) -> dict:
    """The serving workload at its full size: count jobs (the 20,000-job set by
    default) replayed as one Poisson stream per rate, Line 1 in the server
    (host threads, the device builder from dev_min_v input vertices), latency
    from the PSLG's arrival.  Progress lines every 1,000 jobs."""
    import multiprocessing as mp
    import threading
    import numpy as np
    from workloads import generators as G
    from paper_2007_00324_amd import gdp2d
    t0 = time.perf_counter()
    n, bsq, seeds = G.serving_plan(count, 4, 1_000, 200_000)
    args = list(zip(n.tolist(), bsq.tolist(), seeds.tolist()))
    jobs = []
    with mp.get_context("fork").Pool(16) as pool:
        for k, p in enumerate(pool.imap(G._serving_job_args, args, chunksize=4)):
            jobs.append(p)
            if (k + 1) % 1000 == 0:
                log(f"serving (full): generated {k + 1:,} jobs in {time.perf_counter() - t0:.0f} s")
    ctx = gdp2d.Context(0)
    out = {"workload": (f"{count:,} jobs: the 1M-point generator scaled to log-uniform 1,000..200,000 points, "
                        "segments 5% of the points, B^2 drawn from {2.0, 2.56, 4.0}; one Poisson stream per rate; "
                        f"Line 1 in the server (16 host threads, the device builder from {dev_min_v:,} vertices); "
                        "latency from the arrival of the PSLG"),
           "jobs": count, "input_vertices": sum(p.n_vertices for p in jobs), "rates": []}
    for rate in rates:
        srv = gdp2d.Server(ctx, int(budget_gb * (1 << 30)), slots, engine_max_vertices=0, line1=(16, dev_min_v))
        ids = [srv.prepare(p.xy, p.seg, p.ratio_bound_sq) for p in jobs]
        gaps = np.random.default_rng(7).exponential(1.0 / rate, size=count)
        res = [None] * count

        def collect():
            for k, j in enumerate(ids):
                m, rc, t = srv.wait(j)
                res[k] = (rc, t)
                if m is not None:
                    m.free()
                if (k + 1) % 1000 == 0:
                    log(f"serving (full) at {rate:g}/s: {k + 1:,} jobs done")
        th = threading.Thread(target=collect)
        th.start()
        ts = time.perf_counter()
        due = 0.0
        for k, j in enumerate(ids):
            due += gaps[k]
            while time.perf_counter() - ts < due:
                time.sleep(min(0.0005, max(0.0, due - (time.perf_counter() - ts))))
            srv.arrive(j)
        th.join()
        srv.close()
        lat = np.array([t["done_ms"] - t["submit_ms"] for _, t in res])
        l1 = np.array([t["line1_ms"] - t["submit_ms"] for _, t in res])
        span = (max(t["done_ms"] for _, t in res) - min(t["submit_ms"] for _, t in res)) / 1000.0
        row = {"rate_jobs_per_s": rate, "achieved_jobs_per_s": count / span, "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99)), "line1_mean_ms": float(l1.mean()),
               "failed": int(sum(1 for rc, _ in res if rc != 0))}
        log(f"serving (full) at {rate:g}/s: p50 {row['p50_ms']:.0f} ms, p99 {row['p99_ms']:.0f} ms, "
            f"{row['achieved_jobs_per_s']:.1f} jobs/s, {row['failed']} not OK")
        out["rates"].append(row)
    return out


def serving_leg(ctx, jobs, rates, budget_gb: float, slots: int, plain_every: int, engine_max_v=None,
                mode: int = 0) -> dict:
    """Serving form: the same job set replayed as a Poisson stream at each
    rate; latency = completion - arrival (Line 1 runs before arrival).  The
    capacity is measured first (every job arriving at once); rates given as
    fractions ("0.5x") are taken of it."""
    import numpy as np
    from paper_2007_00324_amd import gdp2d
    n = len(jobs)
    out = {"workload": (f"{n} jobs (a reduced stream, not the 20,000-job set): the 1M-point generator scaled to "
                        "log-uniform 1,000..200,000 points, segments 5% of the points, B^2 drawn from "
                        "{2.0, 2.56, 4.0}; Poisson arrivals, the same jobs at every rate; Line 1 on the host before "
                        "arrival"),
           "jobs": n, "input_vertices": sum(p.n_vertices for p in jobs), "budget_gb": budget_gb, "slots": slots,
           "mode": ["shared rounds", "stream per slot"][mode],
           "engine_max_vertices": engine_max_v if engine_max_v is not None else 0,
           "rates": []}
    lat, cap, bad = serve_stream(ctx, jobs, None, budget_gb, slots, engine_max_v, mode)
    out["capacity_jobs_per_s"] = cap
    out["capacity_run"] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                           "failed": bad}
    log(f"serving capacity ({out['mode']}): {cap:.0f} jobs/s with every job arriving at once, {bad} not OK")
    for r in rates:
        lam = cap * float(r[:-1]) if r.endswith("x") else float(r)
        lat, ach, bad = serve_stream(ctx, jobs, lam, budget_gb, slots, engine_max_v, mode)
        row = {"rate_jobs_per_s": lam, "rate_vs_capacity": lam / cap, "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99)), "achieved_jobs_per_s": ach, "failed": bad}
        log(f"serving at {lam:.0f}/s ({lam / cap:.2f} of capacity): p50 {row['p50_ms']:.1f} ms, "
            f"p99 {row['p99_ms']:.1f} ms, {ach:.0f} jobs/s, {bad} not OK")
        out["rates"].append(row)
    # the plain loop on a sample: Line 1 untimed (the server runs it before arrival),
    # then upload + refine one job after another (end to end), and the device
    # refine time alone
    sample = jobs[::plain_every]
    plain_ms, plain_wall = 0.0, 0.0
    for p in sample:
        m0 = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)
        arr, info = m0.arrays(), m0.info()
        m0.free()
        t = time.perf_counter()
        m = gdp2d.gdp_mesh_upload(ctx, arr, info["n_input_vertices"], info["n_input_segments"])
        gdp2d.gdp_mesh_refine(ctx, m, p.ratio_bound_sq, gdp2d.make_params())
        plain_wall += time.perf_counter() - t
        plain_ms += m.last_refine_ms()
        m.free()
    out["plain_jobs_per_s"] = len(sample) / plain_wall
    out["plain_device_jobs_per_s"] = len(sample) / (plain_ms / 1000.0)
    out["plain_sample"] = (f"every {plain_every}th job ({len(sample)} jobs), one after another: upload + refine "
                           "wall time (plain_jobs_per_s) and device refine time alone (plain_device_jobs_per_s)")
    out["capacity_vs_plain"] = out["capacity_jobs_per_s"] / out["plain_jobs_per_s"]
    log(f"serving: plain loop {out['plain_jobs_per_s']:.0f} jobs/s end to end, "
        f"{out['plain_device_jobs_per_s']:.0f} jobs/s of device refine time")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="points of the oracle's CPU baseline (1,000,000: the benchmark's own workload)")
    ap.add_argument("--f1", type=int, default=0, help="Line 6 filter: one circumcenter per located triangle")
    ap.add_argument("--approx-n", type=int, default=0, help="Line 7 filter: n-triangle cavity approximation")
    ap.add_argument("--tail-engine-max", type=int, default=0,
                    help="candidates per round below which rounds run inside one workgroup (0 default, -1 never)")
    ap.add_argument("--no-criteria", action="store_true", help="skip the lens / length-bound / theta legs")
    ap.add_argument("--no-ablation", action="store_true", help="skip the rule ablation leg")
    ap.add_argument("--no-cdt", action="store_true", help="skip the device initial-CDT leg")
    ap.add_argument("--no-flipflop", action="store_true", help="skip the Flip-Flop insertion leg")
    ap.add_argument("--batch", type=int, default=4096, help="jobs of the batched form (0: skip)")
    ap.add_argument("--batch-plain-every", type=int, default=16, help="plain-loop sample: every k-th job")
    ap.add_argument("--batch-line1-device-min", type=int, default=30000,
                    help="batched form also run with Line 1 on the device from this many input vertices (0: skip)")
    ap.add_argument("--workers", type=int, default=16, help="processes generating the batched inputs")
    ap.add_argument("--serve", type=int, default=400, help="jobs of the serving stream (0: skip)")
    ap.add_argument("--serve-rates", type=str, default="0.25x,0.5x,0.9x,1.5x",
                    help="arrival rates, jobs/s, or fractions of the measured capacity (0.5x)")
    ap.add_argument("--serve-mode", type=int, default=0, help="0: shared rounds, 1: a stream per slot")
    ap.add_argument("--only-setting", type=str, default="",
                    help="run one refine of the named ablation setting (on its workload) and exit, for counters")
    ap.add_argument("--serve-sweep", type=str, default="",
                    help="only measure the serving capacity for slots:rounds pairs (e.g. 16:2,32:4) and exit")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-full-jobs", type=int, default=0,
                    help="only run the serving workload at full size (e.g. 20000 jobs) at --serve-full-rates, and exit")
    ap.add_argument("--serve-full-rates", type=str, default="50", help="arrival rates (jobs/s) of the full stream")
    ap.add_argument("--serve-line1-device-min", type=int, default=100000,
                    help="serving with Line 1 in the server: device builder from this many input vertices (0: skip)")
    ap.add_argument("--serve-engine-max", type=int, default=None,
                    help="jobs up to this many input vertices run in batched launches (default: the library's)")
    ap.add_argument("--pmc-sum", nargs=2, default=None, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the HBM bytes of the refinement kernels in two rocprofv3 --pmc output folders")
    ap.add_argument("--pmc-scale", nargs=2, type=float, default=(1.0, 1.0), metavar=("FETCH", "WRITE"),
                    help="copy-calibrated scale factors for --pmc-sum")
    ap.add_argument("--pmc-match", type=str, default=r"gdp::(k|kf|kg)_",
                    help="kernel-name regex for --pmc-sum (copyBuffer for the copy calibration)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration) and exit")
    ap.add_argument("--points", type=int, default=1_000_000, help=argparse.SUPPRESS)
    ap.add_argument("--segments", type=int, default=50_000, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.serve_full_jobs > 0:
        import torch  # noqa: F401
        rates = [float(r) for r in args.serve_full_rates.split(",") if r]
        r = serving_full_leg(args.serve_full_jobs, rates, args.serve_budget_gb, args.serve_slots,
                             args.serve_line1_device_min)
        print(json.dumps({"serving_full": r}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the refinement loop of one PSLG runs on a "
              "single device, it would shard by instance or by spatial blocks.", file=sys.stderr)
        return 2
    if args.pmc_sum:
        r = pmc_sum(args.pmc_sum[0], args.pmc_sum[1], args.pmc_scale[0], args.pmc_scale[1], args.pmc_match)
        print(json.dumps(r), flush=True)
        return 0

    batch = make_batch(args.batch, args.workers) if args.batch > 0 and not args.calibrate_copy else None
    serve_jobs = None
    if args.serve > 0 and not args.calibrate_copy:
        import workloads
        t = time.perf_counter()
        serve_jobs = workloads.serving_jobs(args.serve, workers=args.workers)
        log(f"serving: generated {len(serve_jobs)} jobs in {time.perf_counter() - t:.1f} s")
    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {n * 4} bytes three times")
        return 0
    import workloads
    from paper_2007_00324_amd import gdp2d

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.serve_sweep:
        ctx = gdp2d.Context(0)
        rows = []
        for pair in args.serve_sweep.split(","):
            slots, rounds = (int(x) for x in pair.split(":"))
            lat, cap, bad = serve_stream(ctx, serve_jobs, None, args.serve_budget_gb, slots, 0, 0, rounds)
            log(f"serving sweep: {slots} slots, {rounds} rounds per group: {cap:.1f} jobs/s, {bad} not OK")
            rows.append({"slots": slots, "rounds_per_group": rounds, "capacity_jobs_per_s": cap, "failed": bad})
        print(json.dumps({"serving_sweep": rows}), flush=True)
        return 0
    t = time.perf_counter()
    if args.points == 1_000_000 and args.segments == 50_000:
        p = workloads.config1()
    else:
        p = workloads.scaled_config1(args.points, args.segments)
    log(f"generated {p.name}: {p.n_vertices:,} vertices, {p.n_segments:,} segments in {time.perf_counter() - t:.1f} s")
    ctx = gdp2d.Context(0)
    if args.only_setting:
        table = dict(ABLATION_SETTINGS + COOP_SETTINGS)
        kw = table[args.only_setting]
        q = workloads.config2() if args.only_setting.startswith("coop") else p
        m0 = gdp2d.gdp_mesh_create(ctx, q.xy, q.seg)
        m1 = m0.clone()
        gdp2d.gdp_mesh_refine(ctx, m1, q.ratio_bound_sq, gdp2d.make_params(**kw))  # warm-up
        m1.assign_from(m0)
        torch.cuda.synchronize()
        log(f"setting {args.only_setting}: timed refine begins")
        gdp2d.gdp_mesh_refine(ctx, m1, q.ratio_bound_sq, gdp2d.make_params(**kw))
        rs = m1.round_stats()
        tot = {k: sum(r[k] for r in rs) for k in rs[0]}
        print(json.dumps({"setting": args.only_setting, "workload": q.name, "refine_ms": m1.last_refine_ms(),
                          "alg_bytes": loop_alg_bytes(tot), "rounds": m1.info()["rounds"]}), flush=True)
        return 0
    t = time.perf_counter()
    init = gdp2d.gdp_mesh_create(ctx, p.xy, p.seg)
    log(f"initial CDT (host) + upload: {init.info()['n_triangles']:,} triangles in {time.perf_counter() - t:.1f} s")
    work = init.clone()
    prm = gdp2d.make_params(prefilter_f1=args.f1, cavity_approx_n=args.approx_n, tail_engine_max=args.tail_engine_max)
    for i in range(args.warmup):
        work.assign_from(init)
        gdp2d.gdp_mesh_refine(ctx, work, p.ratio_bound_sq, prm)
        log(f"warmup {i + 1}: {work.last_refine_ms():.1f} ms, {work.info()['rounds']} rounds")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        work.assign_from(init)
        gdp2d.gdp_mesh_refine(ctx, work, p.ratio_bound_sq, prm)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1000.0 / max(args.steps, 1)
    info = work.info()
    steiner = info["n_vertices"] - info["n_input_vertices"]
    tris = info["n_triangles"]
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {steiner:,} Steiner points, {tris:,} triangles, "
        f"{info['rounds']} rounds")
    out = {
        "metric": METRIC,
        "value": steiner / (ms_per_step / 1000.0),
        "unit": "Steiner points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("c1_1M_mixed: 1,000,000 FP64 points (uniform / 64 Gaussian clusters sigma 0.01 / ellipse "
                         "a=0.45 b=0.3 jitter 1e-4) + 50,000 kNN segments + unit square, B=sqrt(2), "
                         "refinement from the resident initial CDT"),
            "n_input_vertices": info["n_input_vertices"],
            "n_input_segments": info["n_input_segments"],
            "ratio_bound_sq": p.ratio_bound_sq,
            "prefilter_f1": args.f1,
            "cavity_approx_n": args.approx_n,
            "steiner_points": steiner,
            "output_triangles": tris,
            "rounds": info["rounds"],
        },
        "output_triangles_per_s": tris / (ms_per_step / 1000.0),
        "roofline": None,
        "cpu_baseline": None,
    }
    if not args.no_profile:
        work.assign_from(init)
        gdp2d.gdp_mesh_refine(ctx, work, p.ratio_bound_sq,
                              gdp2d.make_params(profile_kernels=1, prefilter_f1=args.f1, cavity_approx_n=args.approx_n))
        prof = work.kernel_profile()
        for k in sorted(prof, key=lambda r: -r["total_ms"]):
            if k["launches"]:
                log(f"  {k['name']:<14} {k['launches']:>5} launches {k['total_ms']:9.3f} ms "
                    f"avg {k['total_ms'] / k['launches'] * 1000:8.1f} us items {k['items']:,}")
        by = {k["name"]: k for k in prof}
        dom = max(prof, key=lambda r: r["total_ms"])
        rk = by[ROOFLINE_KERNEL]
        avg_s = rk["total_ms"] / rk["launches"] / 1000.0
        bytes_per_launch = rk["alg_bytes"] / rk["launches"]
        achieved = bytes_per_launch / avg_s / 1e9
        traffic = recorded_traffic()
        scan = by["k_scan"]
        scan_avg_s = scan["total_ms"] / scan["launches"] / 1000.0
        rs = work.round_stats()
        tot = {k: sum(r[k] for r in rs) for k in rs[0]} if rs else {}
        loop_bytes = loop_alg_bytes(tot)
        marks_cc = tot.get("n_marks_cc", 0)
        atomic = atomic_peak(ctx)
        out["roofline"] = {
            "bound": "hbm",
            "kernel": ROOFLINE_KERNEL,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_us": avg_s * 1e6,
            "launches": rk["launches"],
            "alg_bytes_per_launch": bytes_per_launch,
            "alg_bytes_rule": ("winners only: 52 B per cavity triangle (36 B record + 16 B mark read-modify-write "
                               "and read) + 28 B per fan edge (incircle test of the outside triangle)"),
            "waste_ratio": (traffic / bytes_per_launch) if traffic else None,
            "dominant_kernel_by_time": dom["name"],
            "loop": {"alg_bytes_per_step": loop_bytes,
                     "alg_bytes_rule": ("per inserted point: 52 B per cavity triangle + 140 B per fan edge (incircle "
                                        "test, new triangle, outside repair, next-round quality test) + 52 B per walk "
                                        "step + 20 B vertex"),
                     "achieved_gbs": loop_bytes / (ms_per_step / 1000.0) / 1e9,
                     "frac": loop_bytes / (ms_per_step / 1000.0) / 1e9 / HBM_PEAK_GBS},
            "fallbacks": {"incircle_tests": tot.get("n_incircle_tests", 0),
                          "orient_tests": tot.get("n_orient_tests", 0),
                          "exact_orient": tot.get("n_exact_orient", 0), "exact_dot": tot.get("n_exact_dot", 0),
                          "exact_incircle_b": tot.get("n_exact_incircle_b", 0),
                          "exact_incircle_c": tot.get("n_exact_incircle_c", 0),
                          "incircle_rate": ((tot.get("n_exact_incircle_b", 0) + tot.get("n_exact_incircle_c", 0))
                                            / max(1, tot.get("n_incircle_tests", 0))),
                          "orient_rate": tot.get("n_exact_orient", 0) / max(1, tot.get("n_orient_tests", 0))},
            "atomics": {**atomic,
                        "k_cavity_cc_marks_per_launch": marks_cc / rk["launches"],
                        "k_cavity_cc_gatomic_per_s": marks_cc / rk["launches"] / avg_s / 1e9,
                        "k_cavity_cc_frac_of_peak": (marks_cc / rk["launches"] / avg_s / 1e9) / atomic["gatomic_per_s"]},
            "k_scan": {"achieved": scan["alg_bytes"] / scan["launches"] / scan_avg_s / 1e9,
                       "avg_launch_us": scan_avg_s * 1e6, "alg_bytes_per_launch": scan["alg_bytes"] / scan["launches"]},
            "kernel_ms": {k["name"]: round(k["total_ms"], 3) for k in prof if k["launches"]},
            "profiled_refine_ms": work.last_refine_ms(),
        }
    if not args.no_cdt:
        out["initial_cdt"] = cdt_leg(ctx, init, p)
    if not args.no_criteria:
        out["criteria"] = criteria_leg(ctx, init, work, p)
    if not args.no_flipflop:
        out["flipflop"] = flipflop_leg(ctx, init, work, p)
    if not args.no_ablation:
        p2 = workloads.config2()
        init2 = gdp2d.gdp_mesh_create(ctx, p2.xy, p2.seg)
        out["ablation"] = ablation_leg(ctx, init, work, p, init2, p2)
        del init2
    if args.batch > 0:
        out["batched"] = batched_leg(ctx, batch, args.batch_plain_every, args.batch_line1_device_min)
    if serve_jobs:
        rates = [r for r in args.serve_rates.split(",") if r]
        out["serving"] = serving_leg(ctx, serve_jobs, rates, args.serve_budget_gb, args.serve_slots, 8,
                                     args.serve_engine_max, args.serve_mode)
        if args.serve_line1_device_min > 0:
            out["serving"]["line1_in_server"] = serving_line1_leg(ctx, serve_jobs, args.serve_budget_gb,
                                                                  args.serve_slots, args.serve_line1_device_min)
    if not args.no_cpu_baseline:
        n = args.cpu_sample
        log(f"cpu baseline: oracle on {n:,} points")
        out["cpu_baseline"] = cpu_baseline(p, n, max(4, n // 20))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
