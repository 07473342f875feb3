"""Launch-shape autotuner for the forward kernels.

For one batch it times every valid launch shape (threads per workgroup,
vertices per work item, plain / persistent-static / persistent-dynamic /
env-chunked scheduling, workgroups per compute unit, XCD ranges) with HIP
events on the current
stream, checks that each shape's contacts are bit-identical to the default
shape's (the reduction is an integer max, so any difference is a bug), and
records the fastest in a JSON cache keyed by the batch signature:

    {"entries": [{"key": "<signature>", "block": 256, "tile": 1024,
                  "persistent": 2, "grid_mult": 8, "ms": 0.41}, ...]}

``fc_autotune_load(path)`` makes later ``fc_batch_create`` calls with a
matching signature start from that shape.

    python -m paper_2205_03532_amd.autotune --workload nutbolt --out tune.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

from . import fc

DEFAULT = dict(block=256, tile=1024, persistent=0, grid_mult=8, xcd_remap=0)


def candidate_shapes():
    out = []
    for block in (128, 256, 512):
        for vpt in (1, 2, 4):
            for persistent in (0, 1, 2):
                for gm in ((8,) if persistent == 0 else (2, 4, 8, 16)):
                    for xr in (0, 1):
                        out.append(dict(block=block, tile=block * vpt, persistent=persistent, grid_mult=gm,
                                        xcd_remap=xr))
    # env-chunked items (block, tile and grid_mult do not apply)
    for xr in (0, 1):
        out.append(dict(DEFAULT, persistent=3, xcd_remap=xr))
    return out


def _snapshot(out):
    return {k: v.detach().cpu().numpy().copy() for k, v in out.items()}


def _same(a, b):
    return all(np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)) for k in a)


def time_shape(batch, pose, out, reps, warmup):
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fc.fc_sdf_query(batch, pose, fused_out=out)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fc.fc_sdf_query(batch, pose, fused_out=out)
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def tune(batch, pose, shapes=None, reps=10, warmup=3, log=print):
    """Time every shape; returns (best entry, all results)."""
    import torch

    shapes = shapes or candidate_shapes()
    out = batch.new_contacts()
    batch.set_launch(**DEFAULT)
    fc.fc_sdf_query(batch, pose, fused_out=out)
    torch.cuda.synchronize()
    ref = _snapshot(out)
    results = []
    for sh in shapes:
        batch.set_launch(**sh)
        ms = time_shape(batch, pose, out, reps, warmup)
        if not _same(_snapshot(out), ref):
            raise RuntimeError(f"launch shape {sh} changed the contacts")
        results.append(dict(sh, ms=ms))
        log(f"  {sh} -> {ms:.4f} ms")
    best = min(results, key=lambda r: r["ms"])
    batch.set_launch(**{k: best[k] for k in DEFAULT})
    return dict(best, key=batch.signature()), results


def save(entries, path):
    old = []
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f).get("entries", [])
    keys = {e["key"] for e in entries}
    merged = [e for e in old if e["key"] not in keys] + entries
    with open(path, "w") as f:
        json.dump({"entries": merged}, f, indent=1)


def _workload(name, dtype):
    from . import workloads as W

    if name == "nutbolt":
        w = W.nut_bolt_workload()
    elif name == "mixed":
        w = W.mixed_workload()
    elif name == "torus":
        w = W.torus_workload()
    else:
        raise ValueError(name)
    return W.half_storage(w, dtype) if dtype != "f32" else w


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="nutbolt", choices=["nutbolt", "mixed", "torus"])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--layout", default="brick", choices=["linear", "brick", "slab", "sparse"])
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    w = _workload(a.workload, a.dtype)
    batch = fc.Batch.from_workload(w, layout=a.layout, env_order=fc.locality_order(w))
    pose = fc.pose_tensor(w.pose)
    print(f"tuning {w.name} ({a.dtype}, {a.layout}): {batch.Q} queries", flush=True)
    best, _ = tune(batch, pose, reps=a.reps, log=lambda s: print(s, flush=True))
    save([best], a.out)
    print(json.dumps(best), flush=True)


if __name__ == "__main__":
    sys.exit(main())
