"""Autotuner of the batched form's launch shapes (perf only: meshes are the
same for every setting).

The batched form refines each mesh either in one workgroup of the
single-workgroup engine (small meshes: the whole refinement without a
launch per phase) or in shared rounds over the whole chip (large meshes:
each phase one launch for all of them).  Which size classes go where, and
how many shared rounds run between host reads, is picked here by measured
search on a sample drawn from the batched workload's distribution (its own
seed, so the sample is not the benchmark), and stored as a table:

    python -m paper_2007_00324_amd.tune_batch --out TABLE.json [--sample 1024]

The table maps size classes (input vertices) to a path; the library takes
it as one threshold (`batch_engine_max_v`: classes above it run in shared
rounds) and `rounds_per_sync`.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning", "batch.json")
# size classes of the batched workload (input vertices, log-uniform 100..50,000)
CLASS_EDGES = [100, 1_000, 3_000, 10_000, 25_000, 50_001]
SPLITS = [0, 25_000, 10_000, 3_000, 1_000]      # 0: every mesh in the engine
ROUNDS = [2, 4]


def classes_for(split: int) -> list[dict]:
    out = []
    for lo, hi in zip(CLASS_EDGES[:-1], CLASS_EDGES[1:]):
        path = "engine" if split == 0 or hi - 1 <= split else "shared rounds"
        out.append({"input_vertices": [lo, hi - 1], "path": path})
    return out


def load_table(path: str = TABLE) -> dict | None:
    try:
        with open(path) as fh:
            return json.load(fh)
    except OSError:
        return None


def tuned_params(table: dict | None = None):
    """gdp_params of the tuned setting (defaults if there is no table)."""
    from paper_2007_00324_amd import gdp2d
    t = table if table is not None else load_table()
    if not t:
        return gdp2d.make_params()
    return gdp2d.make_params(batch_engine_max_v=int(t["batch_engine_max_v"]),
                             rounds_per_sync=int(t["rounds_per_group"]))


def measure(ctx, inputs, bsq, split: int, rounds: int, reps: int = 2) -> float:
    from paper_2007_00324_amd import gdp2d
    prm = gdp2d.make_params(batch_engine_max_v=split, rounds_per_sync=rounds)
    best = math.inf
    for _ in range(reps):
        meshes, st, ms = gdp2d.gdp_refine_batch(ctx, inputs, bsq, prm)
        assert all(s == 0 for s in st), "a sample instance failed"
        del meshes
        best = min(best, ms)
    return best


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--sample", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=31)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    import workloads
    t = time.perf_counter()
    ps = workloads.batch_config3(args.sample, seed=args.seed, workers=args.workers)
    print(f"[tune] sample of {len(ps)} PSLGs in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    import torch
    from paper_2007_00324_amd import gdp2d
    assert torch.cuda.is_available(), "the tuner measures on a HIP device"
    ctx = gdp2d.Context(0)
    inputs = [(p.xy, p.seg) for p in ps]
    bsq = [p.ratio_bound_sq for p in ps]
    gdp2d.gdp_refine_batch(ctx, inputs[:16], bsq[:16], gdp2d.make_params())  # warm-up
    rows = []
    for split in SPLITS:
        for rounds in (ROUNDS if split else [0]):
            ms = measure(ctx, inputs, bsq, split, rounds)
            rows.append({"batch_engine_max_v": split, "rounds_per_group": rounds, "device_ms": ms,
                         "jobs_per_s": len(ps) / (ms / 1000.0)})
            print(f"[tune] split {split:>6} rounds {rounds}: {ms:8.1f} ms, {rows[-1]['jobs_per_s']:8.0f} jobs/s",
                  file=sys.stderr, flush=True)
    best = min(rows, key=lambda r: r["device_ms"])
    table = {"sample": f"{len(ps)} PSLGs of the batched workload's distribution, seed {args.seed}",
             "batch_engine_max_v": best["batch_engine_max_v"], "rounds_per_group": best["rounds_per_group"] or 2,
             "classes": classes_for(best["batch_engine_max_v"]), "measured": rows}
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(json.dumps({"best": best}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
