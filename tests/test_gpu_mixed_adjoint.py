"""GPU parity of the penalty adjoint on the uneven mixed batch (five part
types, five grids, meshes of 1k to 60k vertices) in FP32.

* On about three envs per part type: per-env loss, twist gradient and
  per-query vertex gradients against the FP64 oracle (each env on its own
  grid and mesh), and each mesh's shared vertex-gradient block against the
  oracle's sum over that mesh's envs; two envs per type against FP64
  central finite differences.
* On the whole 4,096-env batch, in the launch shape and schedule the step
  is timed in: the one-pass call equals the two separate calls bit for bit
  (shared and per-env vertex gradients), each shared block equals the FP64
  sum of the per-env gradients of its envs, the sampled envs of the per-env
  run match the oracle, and a hipGraph of the one-pass step replays to the
  eager results."""
import json
import os

import numpy as np
import pytest

from _adjoint_common import KP, check_fd, check_vs_oracle, run_backward, shared_blocks
from _gpu_common import ULP32, assert_same, to_np, torch_gpu
from paper_2205_03532_amd import fc
from paper_2205_03532_amd import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE_CACHE = os.path.join(ROOT, "paper_2205_03532_amd", "autotune.json")


def sample_envs(w, per_type, seed):
    rng = np.random.default_rng(seed)
    envs = []
    for t in range(len(w.meshes)):
        ids = np.nonzero(w.env_mesh == t)[0]
        envs += list(rng.choice(ids, per_type, replace=False))
    return sorted(int(e) for e in envs)


@pytest.fixture(scope="module")
def mixed():
    torch_gpu()
    return W.mixed_workload()


@pytest.fixture(scope="module")
def bench_batch(mixed):
    """The full batch as the step is timed: brick layout, spatial env order,
    the tuned launch shape of its signature."""
    fc.fc_autotune_load(TUNE_CACHE)
    b = fc.Batch.from_workload(mixed, layout="brick", env_order=fc.locality_order(mixed))
    keys = [e["key"] for e in json.load(open(TUNE_CACHE))["entries"]]
    assert b.signature() in keys, "the mixed batch has no tuned launch shape"
    return b, fc.pose_tensor(mixed.pose)


def onepass(batch, pose, per_env):
    torch = torch_gpu()
    o, g = batch.new_contacts(), batch.new_grads(per_env=per_env)
    fc.fc_sdf_query_and_backward(batch, pose, o, KP, g)
    torch.cuda.synchronize()
    return o, g


def separate(batch, pose, per_env):
    torch = torch_gpu()
    o, g = batch.new_contacts(), batch.new_grads(per_env=per_env)
    fc.fc_sdf_query(batch, pose, fused_out=o)
    fc.fc_sdf_query_backward(batch, pose, KP, g)
    torch.cuda.synchronize()
    return o, g


def same_gpu(a, b):
    torch = torch_gpu()
    for k, v in a.items():
        if hasattr(v, "dtype"):
            assert torch.equal(v.view(torch.uint8) if v.dtype != torch.uint8 else v,
                               b[k].view(torch.uint8) if b[k].dtype != torch.uint8 else b[k]), k


def test_subset_matches_oracle_per_env_and_per_mesh_blocks(mixed):
    """Three envs per type in one batch: per-env mode against the oracle; the
    shared mode's five blocks against the oracle's per-mesh sums; both
    vertex-gradient modes give the same loss and twist; one pass = two calls."""
    envs = sample_envs(mixed, 3, seed=21)
    w = W.subset(mixed, envs)
    b = fc.Batch.from_workload(w, layout="brick")
    pose = fc.pose_tensor(w.pose)
    res_env = run_backward(b, pose, per_env=True)
    shared, tol, worst = check_vs_oracle(w, res_env, range(w.n_env), True)
    print("mixed subset adjoint: worst twist |err|/bound =", worst)
    res = run_backward(b, pose, per_env=False)
    blocks = shared_blocks(w, res["d_verts"])
    for m, gv in enumerate(blocks):
        ref, t = shared[m], tol[m]
        assert np.all(np.abs(gv - ref) <= t[:, None] + 1e-6 * np.abs(ref) + 1e-9), m
        assert np.abs(ref).max() > 0, f"mesh {m}: no penetrating vertex in the sample"
    assert_same(dict(l=res["loss"], p=res["d_pose"]), dict(l=res_env["loss"], p=res_env["d_pose"]))
    for per_env in (False, True):
        o1, g1 = separate(b, pose, per_env)
        o2, g2 = onepass(b, pose, per_env)
        same_gpu(o1, o2)
        same_gpu({k: v for k, v in g1.items() if k != "per_env"}, {k: v for k, v in g2.items() if k != "per_env"})


def test_subset_matches_fp64_finite_differences(mixed):
    """Two envs per part type: twist and vertex gradients against FP64
    central differences (h = 1e-6 m / 1e-6 rad) of the oracle's loss."""
    envs = sample_envs(mixed, 2, seed=22)
    w = W.subset(mixed, envs)
    b = fc.Batch.from_workload(w, layout="brick")
    res = run_backward(b, fc.pose_tensor(w.pose), per_env=True)
    n_smooth, n_kinked = check_fd(w, res, range(w.n_env))
    print(f"mixed FD components: {n_smooth} smooth, {n_kinked} with kinks (checked within their bound)")
    assert n_smooth > 0


def test_full_batch_one_pass_equals_separate_calls(bench_batch):
    b, pose = bench_batch
    for per_env in (False, True):
        o1, g1 = separate(b, pose, per_env)
        o2, g2 = onepass(b, pose, per_env)
        same_gpu(o1, o2)
        same_gpu({k: v for k, v in g1.items() if k != "per_env"}, {k: v for k, v in g2.items() if k != "per_env"})
        del o1, g1, o2, g2


def test_full_batch_shared_blocks_sum_per_env_gradients_and_sample_matches_oracle(mixed, bench_batch):
    """Per mesh m, the shared block equals the sum over m's envs of the
    per-env vertex gradients (FP64 sum on the host; the combine is FP32 with
    compensation, so within a few ulps of the sum plus n_env ulp^2 of the
    sum of magnitudes); loss and twist do not depend on the mode; sampled
    envs of the per-env run match the oracle."""
    torch = torch_gpu()
    b, pose = bench_batch
    w = mixed
    _, g_sh = onepass(b, pose, per_env=False)
    res_sh = to_np({k: v for k, v in g_sh.items() if k != "per_env"})
    del g_sh
    _, g_env = onepass(b, pose, per_env=True)
    assert np.array_equal(g_env["loss"].cpu().numpy().view(np.uint32), res_sh["loss"].view(np.uint32))
    assert np.array_equal(g_env["d_pose"].cpu().numpy().view(np.uint32), res_sh["d_pose"].view(np.uint32))
    off = w.env_query_offsets()
    dv = g_env["d_verts"].view(3, -1)
    blocks = shared_blocks(w, res_sh["d_verts"])
    for m, mesh in enumerate(w.meshes):
        envs = np.nonzero(w.env_mesh == m)[0]
        idx = torch.from_numpy((off[envs][:, None] + np.arange(mesh.n)[None, :]).reshape(-1)).to(dv.device)
        per = dv[:, idx].double().view(3, len(envs), mesh.n)
        s = per.sum(dim=1).T.cpu().numpy()
        a = per.abs().sum(dim=1).T.cpu().numpy()
        tol = 4 * ULP32 * np.abs(s) + 4 * len(envs) * ULP32 ** 2 * a + 1e-30
        err = np.abs(blocks[m] - s)
        assert np.all(err <= tol), (m, float((err / tol).max()))
        assert a.max() > 0, m
        del idx, per
    envs = sample_envs(w, 3, seed=23)
    res = {"loss": res_sh["loss"], "d_pose": res_sh["d_pose"]}
    rows = np.concatenate([np.arange(off[e], off[e + 1]) for e in envs])
    sub_dv = dv[:, torch.from_numpy(rows).to(dv.device)].cpu().numpy()
    # check_vs_oracle reads d_verts at the env's offsets: give it a compact copy
    ws = W.subset(w, envs)
    res_sub = {"loss": res["loss"][envs], "d_pose": res["d_pose"][:, envs], "d_verts": sub_dv.reshape(-1)}
    check_vs_oracle(ws, res_sub, range(ws.n_env), True)
    del g_env, dv


def test_bench_graph_replays_equal_eager(bench_batch):
    """The hipGraph of the one-pass step, as the step is timed on this batch:
    each replay, with eager work and synchronisation between replays, equals
    the eager separate calls bit for bit; so does the forward-only graph."""
    torch = torch_gpu()
    b, pose = bench_batch
    ref_o, ref_g = separate(b, pose, per_env=False)
    ref_o, ref_g = to_np(ref_o), to_np({k: v for k, v in ref_g.items() if k != "per_env"})
    o, g = b.new_contacts(), b.new_grads(per_env=False)
    graph = fc.fc_graph_create(b, pose, fused_out=o, k=KP, grads=g)
    o_f = b.new_contacts()
    graph_f = fc.fc_graph_create(b, pose, fused_out=o_f)
    for _ in range(3):
        for t in list(o.values()) + list(o_f.values()) + [v for k, v in g.items() if k != "per_env"]:
            t.fill_(7)
        torch.cuda.synchronize()
        graph.launch()
        graph_f.launch()
        torch.cuda.synchronize()
        assert_same(to_np(o), ref_o)
        assert_same(to_np(o_f), ref_o)
        assert_same(to_np({k: v for k, v in g.items() if k != "per_env"}), ref_g)
        separate(b, pose, per_env=False)  # eager work between replays
    del graph, graph_f
