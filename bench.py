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


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(n_points: int, n_segments: int) -> dict:
    """Times the oracle (single thread) on a scaled sample of the workload."""
    import oracle
    import workloads
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
        "sample": (f"oracle refinement (initial CDT excluded) of the same generator at {n_points:,} points / "
                   f"{n_segments:,} segments: {steiner:,} Steiner points, {m.nT:,} output triangles in {dt:.2f} s"),
        "output_triangles_per_s": m.nT / dt,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=300_000)
    ap.add_argument("--f1", type=int, default=0, help="Line 6 filter: one circumcenter per located triangle")
    ap.add_argument("--approx-n", type=int, default=0, help="Line 7 filter: n-triangle cavity approximation")
    ap.add_argument("--tail-engine-max", type=int, default=0,
                    help="candidates per round below which rounds run inside one workgroup (0 default, -1 never)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration) and exit")
    ap.add_argument("--points", type=int, default=1_000_000, help=argparse.SUPPRESS)
    ap.add_argument("--segments", type=int, default=50_000, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the refinement loop of one PSLG runs on a "
              "single device, it would shard by instance or by spatial blocks.", file=sys.stderr)
        return 2

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
    t = time.perf_counter()
    if args.points == 1_000_000 and args.segments == 50_000:
        p = workloads.config1()
    else:
        p = workloads.scaled_config1(args.points, args.segments)
    log(f"generated {p.name}: {p.n_vertices:,} vertices, {p.n_segments:,} segments in {time.perf_counter() - t:.1f} s")
    ctx = gdp2d.Context(0)
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
        scan = next(k for k in prof if k["name"] == "k_scan")
        dom = max(prof, key=lambda r: r["total_ms"])
        avg_s = scan["total_ms"] / scan["launches"] / 1000.0
        bytes_per_launch = scan["alg_bytes"] / scan["launches"]
        achieved = bytes_per_launch / avg_s / 1e9
        out["roofline"] = {
            "bound": "hbm",
            "kernel": "k_scan",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": avg_s * 1e6,
            "launches": scan["launches"],
            "alg_bytes_per_launch": bytes_per_launch,
            "dominant_kernel_by_time": dom["name"],
            "kernel_ms": {k["name"]: round(k["total_ms"], 3) for k in prof if k["launches"]},
            "profiled_refine_ms": work.last_refine_ms(),
        }
    if not args.no_cpu_baseline:
        n = args.cpu_sample
        log(f"cpu baseline: oracle on {n:,} points")
        out["cpu_baseline"] = cpu_baseline(n, max(4, n // 20))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
