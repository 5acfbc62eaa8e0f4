"""The whole batched workload: 4,096 PSLGs (log-uniform 100..50,000 points,
kNN segments on 5% of them, B^2 from {2.0, 2.56, 4.0}) refined in one
persistent launch; every instance must equal the oracle's mesh bit for bit.
The instances and the oracle meshes come from a pool of spawned processes
that never touch the GPU; meshes are compared by a digest of all arrays."""
import multiprocessing as mp
import os
import time

import pytest

import workloads
from tests.parity_util import batch_instance_with_oracle, mesh_digest

pytestmark = pytest.mark.gpu


def test_batch_config3_every_instance_matches_oracle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_00324_amd import gdp2d
    n, bsq, seeds = workloads.batch_plan(4096, seed=3)
    args = list(zip(n.tolist(), bsq.tolist(), seeds.tolist()))
    t = time.time()
    workers = min(16, os.cpu_count() or 1)
    print(f"[batch_all] oracle on {len(args)} instances with {workers} processes", flush=True)
    res = []
    with mp.get_context("spawn").Pool(workers) as pool:
        for i, r in enumerate(pool.imap(batch_instance_with_oracle, args, chunksize=4)):
            res.append(r)
            if (i + 1) % 512 == 0:
                print(f"[batch_all] oracle {i + 1}/{len(args)} ({time.time() - t:.0f} s)", flush=True)
    assert all(r[3] == 0 for r in res), [i for i, r in enumerate(res) if r[3] != 0][:10]
    ctx = gdp2d.Context(0)
    from paper_2007_00324_amd import tune_batch
    # the tuned launch shapes (perf only), or a split that uses both paths
    prm = tune_batch.tuned_params() if tune_batch.load_table() else gdp2d.make_params(batch_engine_max_v=10_000)
    print(f"[batch_all] GPU batch of {len(res)} instances (engine up to {prm.batch_engine_max_v or 'all'} input "
          f"vertices, shared rounds above)", flush=True)
    meshes, st, ms = gdp2d.gdp_refine_batch(ctx, [(r[0], r[1]) for r in res], [r[2] for r in res], prm)
    assert all(s == 0 for s in st), [i for i, s in enumerate(st) if s != 0][:10]
    bad = []
    for i, (m, r) in enumerate(zip(meshes, res)):
        if mesh_digest(m.arrays()) != r[4] or m.info()["rounds"] != r[5]:
            bad.append(i)
        m.free()
    print(f"[batch_all] {len(res) - len(bad)} of {len(res)} identical ({ms:.0f} ms on the device)", flush=True)
    assert not bad, (len(bad), bad[:10])
