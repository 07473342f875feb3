"""Throughput of the vertex-vs-SDF contact path on one MI355X.

One step = the whole hot path over one batch, as one
``fc_sdf_query_and_backward`` call: per query the transform, trilinear SDF
value and gradient, candidate, normal bin and deepest-per-bin reduction with
the winner records (the forward), and the adjoint of the penetration penalty
(loss, per-env twist gradient, shared vertex gradient), from one gather.
Workload: 1000 hex nuts (16,396 vertices each) on one M16-like threaded bolt
SDF of 256x256x512 FP32 samples (h = 0.1 mm), K = 32 normal bins, k = 1e4;
inputs resident in HBM before timing.  The separate forms (``fc_sdf_query``
alone; then ``fc_sdf_query_backward``) are timed after the step, outside it.

Prints ONE JSON line (rank 0).  ``value`` is queries per second of the whole
step (one query = one (env, vertex) pair, counted once per step).  The
``roofline`` object is for the dominant kernel, timed with HIP events on the
stream it runs on; ``cpu_baseline`` times the CPU oracle on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vertex-SDF contact queries/sec (fwd, fwd+bwd) and % HBM roofline at stated depth error"
HBM_PEAK_GBS = 8000.0
K_PENALTY = 1e4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the configuration the bench times (and the full-size parity tests check)
BENCH_LAYOUT = "brick"
BENCH_LAUNCH = dict(block=256, tile=1024, persistent=0, grid_mult=8, xcd_remap=1)
TUNE_CACHE = os.path.join(ROOT, "paper_2205_03532_amd", "autotune.json")


TRAFFIC_FILE = os.path.join(ROOT, "paper_2205_03532_amd", "traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2205_03532_amd", "csrc", f)
                  for f in ("fc_kernels.hip", "fc_device.h", "fc_internal.h")]
COPY_PROBE_BYTES = 256 << 20


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


PROFILED_KERNELS = ("k_query_backward", "k_forward", "k_backward")


def _median_counter(csv_dir, kernel, counter, required=True):
    """Median per-dispatch value of `counter` for kernel `kernel`: a name of
    this library's templates is matched as '::kernel<' in the demangled name
    (so k_backward does not match k_query_backward), any other as a substring."""
    import csv
    import glob

    pat = f"::{kernel}<" if kernel in PROFILED_KERNELS else kernel
    vals = []
    for path in glob.glob(os.path.join(csv_dir, "*counter_collection.csv")):
        for r in csv.DictReader(open(path)):
            if pat in r["Kernel_Name"] and r["Counter_Name"] == counter:
                vals.append(float(r["Counter_Value"]))
    if not vals:
        if required:
            raise SystemExit(f"no {counter} samples for {kernel} under {csv_dir}")
        return None
    return sorted(vals)[len(vals) // 2]


def record_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """Turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this bench (and of
    --copy-probe, for calibration) into bytes per launch of each kernel."""
    f_scale = COPY_PROBE_BYTES / 1024 / _median_counter(copy_fetch_dir, "copyBuffer", "FETCH_SIZE")
    w_scale = COPY_PROBE_BYTES / 1024 / _median_counter(copy_write_dir, "copyBuffer", "WRITE_SIZE")
    rec = {"kernel_source_sha256": kernel_source_hash(), "fetch_scale": f_scale, "write_scale": w_scale}
    for k in PROFILED_KERNELS:
        fetch = _median_counter(fetch_dir, k, "FETCH_SIZE", required=False)
        write = _median_counter(write_dir, k, "WRITE_SIZE", required=False)
        if fetch is None or write is None:
            continue
        rec[k] = {"fetch_bytes": fetch * 1024 * f_scale, "write_bytes": write * 1024 * w_scale}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def measured_traffic(kernel):
    """HBM-side bytes per launch of `kernel` from the recorded counters, or None
    when the kernels changed since they were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    if rec.get("kernel_source_sha256") != kernel_source_hash() or kernel not in rec:
        return None
    return rec[kernel]["fetch_bytes"] + rec[kernel]["write_bytes"]


def make_batch(w, device, layout=None, launch=None):
    """The bench's batch: envs scheduled in spatial order, the tuned layout
    (when no layout is asked for and the autotune cache records one for this
    batch, else BENCH_LAYOUT) and the tuned launch shape (cache entry for the
    signature if present, else BENCH_LAUNCH)."""
    from paper_2205_03532_amd import autotune, fc

    if os.path.exists(TUNE_CACHE):
        fc.fc_autotune_load(TUNE_CACHE)
    b = fc.Batch.from_workload(w, device=device, layout=layout or BENCH_LAYOUT, env_order=fc.locality_order(w))
    tuned = autotune.best_layout(b.signature(), TUNE_CACHE) if layout is None else None
    if tuned is not None and tuned != b.layout:
        del b
        b = fc.Batch.from_workload(w, device=device, layout=tuned, env_order=fc.locality_order(w))
    cached = os.path.exists(TUNE_CACHE) and any(e["key"] == b.signature()
                                                 for e in json.load(open(TUNE_CACHE))["entries"])
    if launch is not None or not cached:
        b.set_launch(**(launch or BENCH_LAUNCH))
    return b


def alg_bytes_per_query(dtype):
    s = 4 if dtype == "f32" else 2
    return 12 + 8 * s  # vertex (SoA FP32) + 8 corner samples; pose/output amortise to < 0.1 B


def cpu_baseline(w, n_sample):
    """The oracle as it stands, one thread, on the first n_sample envs."""
    from threadpoolctl import threadpool_limits

    from oracle import adjoint as OA
    from oracle import query as OQ
    from oracle import reduce as ORD

    envs = list(range(n_sample))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        o = OQ.query_workload(w, envs)
        ORD.reduce_contacts(o["env"], o["vidx"], o["depth"].astype(np.float32), o["bin"], o["cand"], w.n_env, w.K)
        g = w.grids[0]
        vals = OQ.grid_values_f64(g.values, g.dtype)
        for e in envs:
            OA.penalty_env(g, w.meshes[0].verts, w.pose[:, e], K_PENALTY, vals)
        dt = time.perf_counter() - t0
    q = sum(w.meshes[int(w.env_mesh[e])].n for e in envs)
    return dict(value=q / dt, unit="queries/s", cores=1, kind="oracle",
                sample=f"first {n_sample} of {w.n_env} envs ({q} queries): FP64 query + exact reduction + "
                       f"penalty adjoint, one thread, {dt:.1f} s")


_PAR = {}


def _par_init(grid_path, verts, pose, bins, margin, origin, h):
    """Worker set-up for the parallel oracle run: the grid memory-mapped."""
    from paper_2205_03532_amd import workloads as W

    g = W.Grid(values=np.load(grid_path, mmap_mode="r"), dtype="f32", origin=origin, h=h)
    _PAR.update(grid=g, verts=verts, pose=pose, bins=bins, margin=margin)


def _par_envs(envs):
    """Oracle query + per-env penalty adjoint for a list of envs (one thread);
    returns the query count and the candidates' (env, vidx, depth, bin)."""
    from threadpoolctl import threadpool_limits

    from oracle import adjoint as OA
    from oracle import query as OQ

    g = _PAR["grid"]
    with threadpool_limits(limits=1):
        vals = OQ.grid_values_f64(np.asarray(g.values), g.dtype)
        out = []
        for e in envs:
            r = OQ.query_env(g, _PAR["verts"], _PAR["pose"][:, e], _PAR["margin"], _PAR["bins"], vals)
            OA.penalty_env(g, _PAR["verts"], _PAR["pose"][:, e], K_PENALTY, vals)
            c = np.nonzero(r["cand"])[0]
            out.append((e, c, r["depth"][c].astype(np.float32), r["bin"][c]))
    return len(envs) * len(_PAR["verts"]), out


def cpu_baseline_parallel(w, procs):
    """The same oracle over all envs in a pool of worker processes (spawned,
    grid memory-mapped from a temporary file), the exact reduction in the
    parent.  Wall time includes the pool's start-up."""
    import multiprocessing as mp
    import tempfile

    from oracle import reduce as ORD

    g = w.grids[0]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "grid.npy")
        np.save(path, np.ascontiguousarray(g.values))
        chunks = [list(range(i, w.n_env, procs)) for i in range(procs)]
        t0 = time.perf_counter()
        ctx = mp.get_context("spawn")
        with ctx.Pool(procs, initializer=_par_init,
                      initargs=(path, w.meshes[0].verts, w.pose, w.bins, w.margin, g.origin, g.h)) as pool:
            parts = pool.map_async(_par_envs, chunks).get(timeout=300)  # a worker that dies cannot hang the bench
        env = np.concatenate([np.full(len(c), e) for _, lst in parts for e, c, _, _ in lst])
        vidx = np.concatenate([c for _, lst in parts for _, c, _, _ in lst])
        depth = np.concatenate([dd for _, lst in parts for _, _, dd, _ in lst])
        bins = np.concatenate([b for _, lst in parts for _, _, _, b in lst])
        ORD.reduce_contacts(env, vidx, depth, bins, np.ones(len(env), bool), w.n_env, w.K)
        dt = time.perf_counter() - t0
    q = sum(n for n, _ in parts)
    return dict(value=q / dt, unit="queries/s", cores=procs, kind="oracle",
                sample=f"all {w.n_env} envs ({q} queries): FP64 query + penalty adjoint in {procs} spawned "
                       f"processes, exact reduction in the parent, {dt:.1f} s including the pool's start-up")


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "cpus_visible": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0))}


def depth_check(w, cand_phi, n_env=4):
    from oracle import query as OQ

    o = OQ.query_workload(w, range(n_env))
    phi = cand_phi[: len(o["phi"])].astype(np.float64)
    ins = o["inside"] & np.isfinite(phi)
    return float(np.max(np.abs(phi[ins] - o["phi"][ins])))


def time_calls(fn, n, warmup):
    """Mean wall time per call (ms) of n calls between two synchronisations."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / n


def measure_faces(batch, pose, n, warmup):
    """Per-face contact generation on the bench batch (fc_sdf_query_faces, fused
    reduction): faces per second, and the main kernel's time."""
    import torch

    from paper_2205_03532_amd import fc

    o = batch.new_contacts()
    call = lambda: fc.fc_sdf_query_faces(batch, pose, fused_out=o)
    ms = time_calls(call, n, warmup)
    batch.set_timing(n)
    for _ in range(n):
        call()
    k, _ = batch.read_timing()
    batch.set_timing(0)
    torch.cuda.synchronize()
    return {"faces_per_s": batch.Qf / (ms * 1e-3), "faces_per_call": batch.Qf, "call_ms": ms,
            "k_faces_ms": float(k.mean()), "iters": fc.PGD_ITERS, "step0": fc.PGD_STEP0,
            "samples_per_face": fc.PGD_ITERS + 1}


def measure_bake(n, warmup, cpu_nodes):
    """Mesh-to-SDF bake of an M4-class bolt (47,104 triangles) on a
    144 x 144 x 256 grid: the host table (once), then fc_bake_sdf timed with
    HIP events on the launch stream; the oracle on a few nodes, one thread."""
    import torch

    from paper_2205_03532_amd import fc
    from paper_2205_03532_amd import workloads as W

    v, t, dims, origin, h = W.bake_workload()
    t0 = time.perf_counter()
    table = fc.BakeTable(v, t)
    torch.cuda.synchronize()
    table_ms = (time.perf_counter() - t0) * 1e3
    out = fc.fc_bake_sdf(table, dims, origin, h)
    for _ in range(warmup):
        fc.fc_bake_sdf(table, dims, origin, h, out=out)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record(stream)
        fc.fc_bake_sdf(table, dims, origin, h, out=out)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    nodes = int(np.prod(dims))
    res = {"workload": f"M4-class threaded bolt mesh ({len(t)} triangles) baked on a {'x'.join(map(str, dims))} "
                       f"grid, h = 0.06 mm", "nodes": nodes, "triangles": int(len(t)), "kernel_ms": ms,
           "nodes_per_s": nodes / (ms * 1e-3),
           "brute_force_equivalent_pairs_per_s": nodes * len(t) / (ms * 1e-3),
           "host_table_ms": table_ms}
    if cpu_nodes > 0:
        from threadpoolctl import threadpool_limits

        from oracle import bake as OB

        rng = np.random.default_rng(11)
        idx = rng.integers(0, nodes, cpu_nodes)
        k, rem = np.divmod(idx, dims[0] * dims[1])
        j, i = np.divmod(rem, dims[0])
        P = np.stack([origin[0] + h * i, origin[1] + h * j, origin[2] + h * k], -1)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            OB.bake_points(v.astype(np.float64), t, P)
            dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": cpu_nodes / dt, "unit": "nodes/s", "cores": 1, "kind": "oracle",
                               "sample": f"{cpu_nodes} random nodes against all {len(t)} triangles, FP64, "
                                         f"one thread, {dt:.1f} s"}
    return res


def measure_patches(batch, pose, n, warmup):
    """Patch reduction (Algorithm 1, fc_contact_patches) on the bench batch:
    environments per second, patches per environment, the kernel's time."""
    import torch

    from paper_2205_03532_amd import fc

    out = batch.new_patches(fc.PATCH_MAX)
    call = lambda: fc.fc_contact_patches(batch, pose, out)  # noqa: E731
    ms = time_calls(call, n, warmup)
    batch.set_timing(n)
    for _ in range(n):
        call()
    k, _ = batch.read_timing()
    batch.set_timing(0)
    torch.cuda.synchronize()
    cnt = out["count"].cpu().numpy()
    return {"envs_per_s": batch.n_env / (ms * 1e-3), "queries_per_s": batch.Q / (ms * 1e-3), "call_ms": ms,
            "k_patches_ms": float(k.mean()), "max_patches": fc.PATCH_MAX, "cos_sim": fc.PATCH_COS,
            "batch_vertices": 1024, "patches_per_env_mean": float(cnt.mean()), "patches_per_env_max": int(cnt.max())}


def step_roofline(b, pose, n, warmup, bpq):
    """Mean duration of the one-pass kernel (library events on the launch
    stream) and of the gather probe on batch b; the algorithmic rate."""
    import torch

    from paper_2205_03532_amd import fc

    o, g = b.new_contacts(), b.new_grads(per_env=False)
    sink = torch.zeros(1, device=b.device)
    for _ in range(warmup):
        fc.fc_sdf_query_and_backward(b, pose, o, K_PENALTY, g)
        fc.fc_gather_probe(b, pose, sink)
    b.set_timing(n)
    for _ in range(n):
        fc.fc_sdf_query_and_backward(b, pose, o, K_PENALTY, g)
    k_one, kid = b.read_timing()
    assert np.all(kid == fc.FC_KERNEL_QUERY_BACKWARD)
    b.set_timing(n)
    for _ in range(n):
        fc.fc_gather_probe(b, pose, sink)
    k_probe, kid = b.read_timing()
    b.set_timing(0)
    assert np.all(kid == fc.FC_KERNEL_GATHER_PROBE)
    torch.cuda.synchronize()
    kms, pms = float(k_one.mean()), float(k_probe.mean())
    ach = bpq * b.Q / (kms * 1e-3) / 1e9
    return {"kernel": "k_query_backward", "kernel_ms": kms, "alg_bytes_per_query": bpq, "achieved": ach,
            "unit": "GB/s", "hbm_peak": HBM_PEAK_GBS, "frac_of_hbm_peak": ach / HBM_PEAK_GBS,
            "gather_probe_ms": pms, "frac_of_achievable_gather": pms / kms}


def contact_errors(w32, cand, envs):
    """Depth and normal error of a batch's candidates against the FP64 oracle
    on the FP32 grids of w32, over every contact of the listed envs (queries
    the oracle makes candidates and both sides place inside the grid)."""
    from oracle import query as OQ

    o = OQ.query_workload(w32, envs)
    off = w32.env_query_offsets()
    rows = np.concatenate([np.arange(off[e], off[e + 1]) for e in envs])
    phi = cand["phi"].cpu().numpy()[rows].astype(np.float64)
    nrm = cand["normal"].cpu().numpy()[:, rows].T.astype(np.float64)
    c = o["cand"] & np.isfinite(phi)
    derr = np.abs(phi[c] - o["phi"][c])
    nerr = np.linalg.norm(nrm[c] - o["normal"][c], axis=1)
    near = np.abs(o["phi"][c]) < 1e-3

    def q(a, p):
        return float(np.percentile(a, p)) if a.size else 0.0
    return {"contacts": int(c.sum()), "envs": len(envs),
            "max_depth_err_m": float(derr.max()) if derr.size else 0.0,
            "max_depth_err_m_within_1mm": float(derr[near].max()) if near.any() else 0.0,
            "p99_depth_err_m": q(derr, 99),
            "max_normal_err": float(nerr.max()) if nerr.size else 0.0,
            "p99_normal_err": q(nerr, 99), "p50_normal_err": q(nerr, 50),
            "normal_err_unit": "chord |n - n_fp64| (radians for small angles)"}


def sample_envs_per_type(w, per_type, seed=0):
    rng = np.random.default_rng(seed)
    envs = []
    for t in range(len(w.meshes)):
        ids = np.nonzero(w.env_mesh == t)[0]
        envs += list(rng.choice(ids, min(per_type, len(ids)), replace=False))
    return sorted(int(e) for e in envs)


def measure_torus(device, n, warmup):
    """The L2-resident case: analytic torus (R = 2 cm, r = 0.5 cm) on a 64^3
    FP32 grid (1 mm), 2,562-vertex icosphere, 256 random poses, K = 16.  The
    1 MiB grid sits in every XCD's 4 MB L2, so the ceiling is the gather
    probe (L2 and texture units), not HBM.  Depth error over all 256 envs."""
    import torch

    from paper_2205_03532_amd import fc
    from paper_2205_03532_amd import workloads as W

    w = W.torus_workload()
    b = make_batch(w, device)
    pose = fc.pose_tensor(w.pose, device)
    o, g = b.new_contacts(), b.new_grads(per_env=False)
    ms_one = time_calls(lambda: fc.fc_sdf_query_and_backward(b, pose, o, K_PENALTY, g), n, warmup)
    ms_fwd = time_calls(lambda: fc.fc_sdf_query(b, pose, fused_out=o), n, warmup)
    rl = step_roofline(b, pose, n, warmup, alg_bytes_per_query("f32"))
    rl["bound"] = "l2 gather (grid resident in each XCD's L2)"
    cand = b.new_candidates()
    fc.fc_sdf_query(b, pose, cand=cand)
    torch.cuda.synchronize()
    err = contact_errors(w, cand, list(range(w.n_env)))
    return {"workload": "torus R = 2 cm, r = 0.5 cm, 64^3 FP32 grid (h = 1 mm); icosphere r = 1 cm, "
                        f"{w.meshes[0].n} vertices; {w.n_env} poses; K = {w.K}",
            "queries_per_step": b.Q, "fwd_bwd_queries_per_s": b.Q / (ms_one * 1e-3),
            "fwd_queries_per_s": b.Q / (ms_fwd * 1e-3), "call_ms": {"query_and_backward": ms_one, "query": ms_fwd},
            "roofline": rl, "errors_vs_fp64_oracle_all_envs": err, "launch": b.get_launch()}


def measure_nutbolt_1024(device, n, warmup):
    """Forward plus backward on 1,024 nut-bolt envs (the differentiation
    configuration; its gradients are checked against FP64 finite differences
    on 64 envs by the parity tests)."""
    import torch

    from paper_2205_03532_amd import fc
    from paper_2205_03532_amd import workloads as W

    w = W.nut_bolt_workload(n_env=1024)
    b = make_batch(w, device)
    pose = fc.pose_tensor(w.pose, device)
    o, g = b.new_contacts(), b.new_grads(per_env=False)
    ms_one = time_calls(lambda: fc.fc_sdf_query_and_backward(b, pose, o, K_PENALTY, g), n, warmup)
    ms_sep = time_calls(lambda: (fc.fc_sdf_query(b, pose, fused_out=o),
                                 fc.fc_sdf_query_backward(b, pose, K_PENALTY, g)), n, warmup)
    rl = step_roofline(b, pose, n, warmup, alg_bytes_per_query("f32"))
    cand = b.new_candidates()
    fc.fc_sdf_query(b, pose, cand=cand)
    torch.cuda.synchronize()
    err = contact_errors(w, cand, [0, 1, 2, 3])
    return {"workload": f"nut-on-bolt, {w.n_env} envs x {w.meshes[0].n} vertices, 256x256x512 FP32 bolt SDF, "
                        "penalty 0.5 k depth^2 (k = 1e4), gradients for pose twists and shared vertices",
            "queries_per_step": b.Q, "fwd_bwd_queries_per_s": b.Q / (ms_one * 1e-3),
            "separate_fwd_then_bwd_queries_per_s": b.Q / (ms_sep * 1e-3), "call_ms": ms_one,
            "errors_vs_fp64_oracle": err, "roofline": rl, "launch": b.get_launch()}


def measure_forms(w32, device, n, warmup):
    """The other forms of the path beside the FP32 nut-bolt step: the same
    batch with FP16 and BF16 grid storage, with narrow-band sparse storage,
    and the uneven mixed batch
    (4,096 envs, five part types) replayed as hipGraphs.  Queries/s of the
    one-pass step and of the fused forward; depth error of the half forms
    against the FP64 oracle on the FP32 grid (4 envs)."""
    import torch

    from paper_2205_03532_amd import fc
    from paper_2205_03532_amd import workloads as W

    out = {}
    for dt in ("f16", "bf16"):
        wh = W.half_storage(w32, dt)
        b = make_batch(wh, device)
        pose = fc.pose_tensor(wh.pose, device)
        o, g = b.new_contacts(), b.new_grads(per_env=False)
        ms_one = time_calls(lambda: fc.fc_sdf_query_and_backward(b, pose, o, K_PENALTY, g), n, warmup)
        ms_fwd = time_calls(lambda: fc.fc_sdf_query(b, pose, fused_out=o), n, warmup)
        cand = b.new_candidates()
        fc.fc_sdf_query(b, pose, cand=cand)
        torch.cuda.synchronize()
        out[f"nutbolt_{dt}_grid"] = {
            "fwd_bwd_queries_per_s": b.Q / (ms_one * 1e-3), "fwd_queries_per_s": b.Q / (ms_fwd * 1e-3),
            "alg_bytes_per_query": alg_bytes_per_query(dt),
            "max_depth_err_m_vs_fp32_grid_oracle": depth_check(w32, cand["phi"].cpu().numpy()),
            "errors_vs_fp32_grid_fp64_oracle": contact_errors(w32, cand, [0, 1, 2, 3]),
            "roofline": step_roofline(b, pose, n, warmup, alg_bytes_per_query(dt)),
            "launch": b.get_launch()}
        del b, o, g, cand
    # narrow-band sparse storage of the same FP32 grid (4-voxel band): every nut
    # query lies in a stored brick, so the outputs must equal the brick layout's
    bs = make_batch(w32, device, layout="sparse")
    bb = make_batch(w32, device, layout="brick")
    pose = fc.pose_tensor(w32.pose, device)
    outs = []
    for b in (bs, bb):
        o, g = b.new_contacts(), b.new_grads(per_env=False)
        fc.fc_sdf_query_and_backward(b, pose, o, K_PENALTY, g)
        outs.append((o, g))
    torch.cuda.synchronize()
    same = all(torch.equal(outs[0][0][k], outs[1][0][k]) for k in outs[0][0]) and all(
        torch.equal(outs[0][1][k], outs[1][1][k]) for k in ("loss", "d_pose", "d_verts"))
    o, g = outs[0]
    ms_one = time_calls(lambda: fc.fc_sdf_query_and_backward(bs, pose, o, K_PENALTY, g), n, warmup)
    ms_fwd = time_calls(lambda: fc.fc_sdf_query(bs, pose, fused_out=o), n, warmup)
    out["nutbolt_f32_sparse_grid"] = {
        "fwd_bwd_queries_per_s": bs.Q / (ms_one * 1e-3), "fwd_queries_per_s": bs.Q / (ms_fwd * 1e-3),
        "grid_bytes": bs.sparse_bytes, "brick_grid_bytes": int(bb.grid_tensors[0].numel()),
        "linear_grid_bytes": int(w32.grids[0].values.nbytes), "band_m": fc.SPARSE_BAND_VOXELS * w32.grids[0].h,
        "equals_brick_layout": bool(same), "launch": bs.get_launch()}
    del bs, bb, outs, o, g
    wm = W.mixed_workload()
    b = make_batch(wm, device)
    pose = fc.pose_tensor(wm.pose, device)
    o, g = b.new_contacts(), b.new_grads(per_env=False)
    g_one = fc.fc_graph_create(b, pose, fused_out=o, k=K_PENALTY, grads=g)
    g_fwd = fc.fc_graph_create(b, pose, fused_out=o)
    ms_one = time_calls(g_one.launch, n, warmup)
    ms_fwd = time_calls(g_fwd.launch, n, warmup)
    envs = sample_envs_per_type(wm, 2, seed=3)
    cand = b.new_candidates()
    fc.fc_sdf_query(b, pose, cand=cand)
    torch.cuda.synchronize()
    out["mixed_4096_envs_5_types_graph"] = {
        "fwd_bwd_queries_per_s": b.Q / (ms_one * 1e-3), "fwd_queries_per_s": b.Q / (ms_fwd * 1e-3),
        "queries_per_step": b.Q, "launch": b.get_launch(),
        "errors_vs_fp64_oracle": contact_errors(wm, cand, envs),
        "roofline": step_roofline(b, pose, n, warmup, alg_bytes_per_query("f32"))}
    del b, o, g, g_one, g_fwd, cand
    # the same uneven batch with every grid in FP16, then BF16: depth and normal
    # error against the FP64 oracle on the FP32 grids over all contacts of two
    # sampled envs per part type
    for dt in ("f16", "bf16"):
        wh = W.half_storage(wm, dt)
        b = make_batch(wh, device)
        pose = fc.pose_tensor(wh.pose, device)
        o, g = b.new_contacts(), b.new_grads(per_env=False)
        g_one = fc.fc_graph_create(b, pose, fused_out=o, k=K_PENALTY, grads=g)
        g_fwd = fc.fc_graph_create(b, pose, fused_out=o)
        ms_one = time_calls(g_one.launch, n, warmup)
        ms_fwd = time_calls(g_fwd.launch, n, warmup)
        cand = b.new_candidates()
        fc.fc_sdf_query(b, pose, cand=cand)
        torch.cuda.synchronize()
        out[f"mixed_4096_envs_5_types_{dt}_graph"] = {
            "fwd_bwd_queries_per_s": b.Q / (ms_one * 1e-3), "fwd_queries_per_s": b.Q / (ms_fwd * 1e-3),
            "queries_per_step": b.Q, "alg_bytes_per_query": alg_bytes_per_query(dt),
            "errors_vs_fp32_grid_fp64_oracle": contact_errors(wm, cand, envs),
            "roofline": step_roofline(b, pose, n, warmup, alg_bytes_per_query(dt)),
            "launch": b.get_launch()}
        del b, o, g, g_one, g_fwd, cand
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n-env", type=int, default=1000)
    ap.add_argument("--layout", default=None, choices=[None, "linear", "brick", "slab"])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--cpu-sample", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP16/BF16 and mixed-batch measurements")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (calibrates rocprof byte counters) and exit")
    ap.add_argument("--only-bake", action="store_true",
                    help="only time the mesh-to-SDF bake form (fc_bake_sdf) and print its JSON object")
    ap.add_argument("--record-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write the measured bytes per launch from rocprofv3 --pmc output directories and exit")
    args = ap.parse_args()

    if args.record_traffic:
        record_traffic(*args.record_traffic)
        return

    if args.copy_probe:
        import torch

        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")  # 256 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "launches": 3}), flush=True)
        return

    if args.only_bake:
        print(json.dumps(measure_bake(args.steps, args.warmup, 0 if args.no_cpu_baseline else 100)), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (--gpus 1): the path shards by environment with no "
              "communication in the forward pass, and the library has no multi-GPU launch.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2205_03532_amd import fc
    from paper_2205_03532_amd import workloads as W

    t0 = time.perf_counter()
    w = W.nut_bolt_workload(n_env=args.n_env)
    if args.dtype != "f32":
        w = W.half_storage(w, args.dtype)
    log(f"workload {w.name}: {w.n_env} envs x {w.meshes[0].n} verts, grid {w.grids[0].dims} "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    dev = torch.device("cuda:0")
    batch = make_batch(w, dev, layout=args.layout)
    launch = batch.get_launch()
    pose = fc.pose_tensor(w.pose, dev)
    out = batch.new_contacts()
    grads = batch.new_grads(per_env=False)
    Q = batch.Q
    stream = torch.cuda.current_stream()

    def step():
        fc.fc_sdf_query_and_backward(batch, pose, out, K_PENALTY, grads)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K steps between two synchronisations, nothing else on the stream
    n = args.steps
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(n):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_step = wall * 1e3 / n
    value = Q * n / wall

    # the same K steps again, timed per call (torch events on the stream the kernels run on)
    # and per main kernel (the library's events around k_query_backward alone)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(n)]
    batch.set_timing(n)
    torch.cuda.synchronize()
    for i in range(n):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    one_ms = np.array([ev[i][0].elapsed_time(ev[i][1]) for i in range(n)])
    k_one, kid = batch.read_timing()
    assert len(k_one) == n and np.all(kid == fc.FC_KERNEL_QUERY_BACKWARD)

    def quantiles(a):
        return {f"p{q}": float(np.percentile(a, q)) for q in (10, 50, 90)}

    # the achievable gather rate of this path: the same kernel loop and loads with no
    # arithmetic (fc_gather_probe), timed the same way
    sink = torch.zeros(1, device=dev)
    for _ in range(args.warmup):
        fc.fc_gather_probe(batch, pose, sink)
    batch.set_timing(n)
    for _ in range(n):
        fc.fc_gather_probe(batch, pose, sink)
    k_probe, kid = batch.read_timing()
    assert len(k_probe) == n and np.all(kid == fc.FC_KERNEL_GATHER_PROBE)

    # the separate forms, for comparison (not part of the step)
    out2 = batch.new_contacts()
    grads2 = batch.new_grads(per_env=False)
    for _ in range(args.warmup):
        fc.fc_sdf_query(batch, pose, fused_out=out2)
        fc.fc_sdf_query_backward(batch, pose, K_PENALTY, grads2)
    ev2 = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(n)]
    batch.set_timing(2 * n)
    torch.cuda.synchronize()
    for i in range(n):
        ev2[i][0].record(stream)
        fc.fc_sdf_query(batch, pose, fused_out=out2)
        ev2[i][1].record(stream)
        fc.fc_sdf_query_backward(batch, pose, K_PENALTY, grads2)
        ev2[i][2].record(stream)
    torch.cuda.synchronize()
    fwd_ms = np.array([ev2[i][0].elapsed_time(ev2[i][1]) for i in range(n)])
    bwd_ms = np.array([ev2[i][1].elapsed_time(ev2[i][2]) for i in range(n)])
    k_sep, kid = batch.read_timing()
    batch.set_timing(0)
    k_fwd, k_bwd = k_sep[kid == fc.FC_KERNEL_FORWARD], k_sep[kid == fc.FC_KERNEL_BACKWARD]
    same = all(torch.equal(out[k], out2[k]) for k in out) and all(
        torch.equal(grads[k], grads2[k]) for k in ("loss", "d_pose", "d_verts"))

    # the unfused forward: candidates written, then the reduction reads them
    cand_u = batch.new_candidates()
    unf_ms = time_calls(lambda: (fc.fc_sdf_query(batch, pose, cand=cand_u),
                                 fc.fc_contact_reduce(batch, pose, cand_u, out2)), n, args.warmup)
    del cand_u

    bpq = alg_bytes_per_query(args.dtype)
    o_avg, f_avg, b_avg = float(one_ms.mean()), float(fwd_ms.mean()), float(bwd_ms.mean())
    kname, kkey = "k_query_backward (one-pass query, reduction and penalty adjoint)", "k_query_backward"
    kms = float(k_one.mean())  # the main kernel alone, mean over the timed launches
    achieved = bpq * Q / (kms * 1e-3) / 1e9
    # the counters were taken on the FP32 brick layout
    traffic = measured_traffic(kkey) if batch.layout == "brick" and args.dtype == "f32" else None

    # accuracy of the timed configuration on a sample (outside the timed region)
    cand = batch.new_candidates()
    fc.fc_sdf_query(batch, pose, cand=cand)
    torch.cuda.synchronize()
    derr = depth_check(w if args.dtype == "f32" else W.nut_bolt_workload(n_env=args.n_env),
                       cand["phi"].cpu().numpy())

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"nut-on-bolt: {w.n_env} envs x {w.meshes[0].n}-vertex hex nut (M16-like internal "
                        f"thread) vs one {'x'.join(map(str, w.grids[0].dims))} {args.dtype} bolt SDF "
                        f"(h = 0.1 mm), K = {w.K} bins; step = one-pass query + contact reduction + penalty "
                        f"adjoint (k = 1e4, shared vertex gradients)",
            "n_env": w.n_env,
            "queries_per_step": Q,
            "layout": batch.layout,
            "env_order": "spatial (locality_order)",
            "launch": launch,
        },
        "fwd_queries_per_s": Q / (f_avg * 1e-3),
        "fwd_bwd_queries_per_s": value,
        "separate_fwd_then_bwd_queries_per_s": Q / ((f_avg + b_avg) * 1e-3),
        "separate_equals_one_pass": bool(same),
        "call_ms": {"query_and_backward": o_avg, "query": f_avg, "backward": b_avg},
        "call_ms_quantiles": {"query_and_backward": quantiles(one_ms), "query": quantiles(fwd_ms),
                              "backward": quantiles(bwd_ms)},
        "kernel_ms_quantiles": {"k_query_backward": quantiles(k_one)},
        "fwd_unfused_queries_per_s": Q / (unf_ms * 1e-3),
        "kernel_ms": {"k_query_backward": kms, "k_forward": float(k_fwd.mean()), "k_backward": float(k_bwd.mean())},
        "max_depth_err_m": derr,
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "kernel_ms": kms,
            "timing": "HIP events recorded on the launch stream around this kernel alone, in each of K steps "
                      "run right after the timed ones",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "limiter": "gather: texture address/data units and L1 line traffic (most corner lines hit in "
                       "L2/MALL, so DRAM moves far fewer bytes than the algorithmic count)",
            "dram_GBps": (traffic / (kms * 1e-3) / 1e9) if traffic else None,
            "dram_frac": (traffic / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
            "alg_bytes_per_query": bpq,
            "achievable_gather": {
                "probe": "fc_gather_probe: the same kernel loop, work items and corner loads, no arithmetic",
                "probe_ms": float(k_probe.mean()),
                "probe_GBps": bpq * Q / (float(k_probe.mean()) * 1e-3) / 1e9,
                "frac": float(k_probe.mean()) / kms,
            },
        },
    }
    if not args.no_forms and args.dtype == "f32":
        res["forms"] = {"nutbolt_faces_pgd": measure_faces(batch, pose, n, args.warmup),
                        "nutbolt_patch_reduction": measure_patches(batch, pose, n, args.warmup)}
        res["forms"].update(measure_forms(w, dev, n, args.warmup))
        res["forms"]["torus64_icosphere_256_poses"] = measure_torus(dev, n, args.warmup)
        res["forms"]["nutbolt_1024_envs_fwd_bwd"] = measure_nutbolt_1024(dev, n, args.warmup)
        res["forms"]["m4_bolt_mesh_bake"] = measure_bake(n, args.warmup, 0 if args.no_cpu_baseline else 100)
    res["host"] = host_info()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, min(args.cpu_sample, w.n_env))
        if args.dtype == "f32":
            try:
                res["cpu_baseline_parallel"] = cpu_baseline_parallel(w, min(16, len(os.sched_getaffinity(0))))
            except Exception as exc:  # reported, never fatal: the GPU figures above stand
                res["cpu_baseline_parallel"] = {"skipped": f"{type(exc).__name__}: {exc}"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
