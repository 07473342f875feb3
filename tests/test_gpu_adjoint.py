"""GPU parity of the penetration-penalty adjoint (loss, twist and vertex
gradients) against the FP64 oracle and FP64 finite differences, plus the
autograd wrapper and graph replay."""
import numpy as np
import pytest

from _adjoint_common import KP, check_fd, check_vs_oracle, run_backward, shared_blocks
from _gpu_common import assert_same, to_np, torch_gpu
from paper_2205_03532_amd import fc
from paper_2205_03532_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torus16():
    torch_gpu()
    w = W.subset(W.torus_workload(), range(16))
    return w, fc.Batch.from_workload(w), fc.pose_tensor(w.pose)


@pytest.fixture(scope="module")
def nutbolt40():
    torch_gpu()
    w = W.subset(W.nut_bolt_workload(seed=1004, n_env=1024), range(40))
    return w, fc.Batch.from_workload(w), fc.pose_tensor(w.pose)


def test_torus_adjoint_matches_oracle(torus16):
    w, b, pose = torus16
    res = run_backward(b, pose, per_env=True)
    _, _, worst = check_vs_oracle(w, res, range(w.n_env), True)
    print("torus adjoint: worst |err|/bound =", worst)
    assert res["loss"].max() > 0


def test_nutbolt_adjoint_matches_oracle_and_shared_sum(nutbolt40):
    w, b, pose = nutbolt40
    res_env = run_backward(b, pose, per_env=True)
    shared, tol, worst = check_vs_oracle(w, res_env, range(w.n_env), True)
    print("nut-bolt adjoint: worst |err|/bound =", worst)
    res = run_backward(b, pose, per_env=False)
    gv = shared_blocks(w, res["d_verts"])[0]
    assert np.all(np.abs(gv - shared[0]) <= tol[0][:, None] + 1e-6 * np.abs(shared[0]) + 1e-9)
    # loss / pose outputs do not depend on the vertex-gradient mode
    assert_same(dict(l=res["loss"], p=res["d_pose"]), dict(l=res_env["loss"], p=res_env["d_pose"]))


def test_adjoint_deterministic_and_workspace_clean(nutbolt40):
    torch = torch_gpu()
    w, b, pose = nutbolt40
    r1 = run_backward(b, pose, per_env=False)
    assert int(torch.count_nonzero(b.workspace[: 256])) == 0
    r2 = run_backward(b, pose, per_env=False)
    assert_same(r1, r2)


def test_adjoint_xcd_ranges_and_env_order(nutbolt40):
    """XCD-range scheduling leaves every output bit-identical; a different env
    order changes only the shared vertex sum's rounding."""
    w, b, pose = nutbolt40
    ref = run_backward(b, pose, per_env=False)
    ref_env = run_backward(b, pose, per_env=True)
    old = b.get_launch()
    try:
        b.set_launch(**dict(old, xcd_remap=1))
        assert_same(run_backward(b, pose, per_env=False), ref)
        assert_same(run_backward(b, pose, per_env=True), ref_env)
    finally:
        b.set_launch(**old)
    bo = fc.Batch.from_workload(w, env_order=np.arange(w.n_env)[::-1].copy())
    r = run_backward(bo, pose, per_env=False)
    assert_same(dict(l=r["loss"], p=r["d_pose"]), dict(l=ref["loss"], p=ref["d_pose"]))
    assert np.allclose(r["d_verts"], ref["d_verts"], rtol=1e-5, atol=1e-6 * np.abs(ref["d_verts"]).max())


def test_upstream_scaling(torus16):
    torch = torch_gpu()
    w, b, pose = torus16
    up = torch.linspace(-2.0, 3.0, w.n_env, device="cuda")
    r1 = run_backward(b, pose, per_env=True)
    r2 = run_backward(b, pose, per_env=True, upstream=up)
    u = up.cpu().numpy()
    assert np.array_equal(r2["loss"], r1["loss"])  # the loss is the forward value
    assert np.array_equal(r2["d_pose"], (u[None, :] * r1["d_pose"]).astype(np.float32))
    off = w.env_query_offsets()
    for e in range(w.n_env):
        s = slice(off[e], off[e + 1])
        a = r2["d_verts"].reshape(3, -1)[:, s]
        c = r1["d_verts"].reshape(3, -1)[:, s]
        assert np.array_equal(a, (np.float32(u[e]) * c).astype(np.float32))


def test_gradients_match_fp64_finite_differences():
    """The 1,024-env nut-bolt set: GPU twist gradients vs FP64 central differences
    (h = 1e-6 m / 1e-6 rad) on 64 envs drawn by the seed."""
    torch_gpu()
    w = W.nut_bolt_workload(seed=1004, n_env=1024)
    rng = np.random.default_rng(1004)
    envs = np.sort(rng.choice(w.n_env, 64, replace=False))
    sub = W.subset(w, envs)
    b = fc.Batch.from_workload(sub)
    res = run_backward(b, fc.pose_tensor(sub.pose), per_env=True)
    n_smooth, n_kinked = check_fd(sub, res, range(sub.n_env))
    print(f"FD components: {n_smooth} smooth, {n_kinked} with kinks (checked within their bound)")


def test_autograd_function_matches_direct_call(torus16):
    torch = torch_gpu()
    from paper_2205_03532_amd.autograd import penalty

    w, b, pose = torus16
    for mt in b.mesh_tensors:
        mt.requires_grad_(True)
    try:
        loss, xi = penalty(b, pose, KP)
        wts = torch.arange(1, w.n_env + 1, dtype=torch.float32, device="cuda")
        (loss * wts).sum().backward()
        direct = run_backward(b, pose, per_env=False, upstream=wts)
        assert np.array_equal(loss.detach().cpu().numpy(), direct["loss"])
        assert np.array_equal(xi.grad.cpu().numpy(), direct["d_pose"].T)
        assert np.array_equal(b.mesh_tensors[0].grad.cpu().numpy().reshape(-1), direct["d_verts"])
        with pytest.raises(ValueError):
            penalty(b, pose, KP, xi=torch.ones(w.n_env, 6, device="cuda", requires_grad=True))
    finally:
        for mt in b.mesh_tensors:
            mt.requires_grad_(False)
            mt.grad = None


def test_graph_replay_matches_eager(nutbolt40):
    torch = torch_gpu()
    w, b, pose = nutbolt40
    out_e = b.new_contacts()
    g_e = b.new_grads(per_env=False)
    fc.fc_sdf_query(b, pose, fused_out=out_e)
    fc.fc_sdf_query_backward(b, pose, KP, g_e)
    torch.cuda.synchronize()
    ref_o, ref_g = to_np(out_e), to_np({k: v for k, v in g_e.items() if k != "per_env"})
    out = b.new_contacts()
    gr = b.new_grads(per_env=False)
    graph = fc.fc_graph_create(b, pose, fused_out=out, k=KP, grads=gr)
    for rep in range(4):
        for t in list(out.values()) + [v for k, v in gr.items() if k != "per_env"]:
            t.fill_(7)  # eager work between replays
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert_same(to_np(out), ref_o)
        assert_same(to_np({k: v for k, v in gr.items() if k != "per_env"}), ref_g)
        # eager calls interleaved with replays share the workspace correctly
        fc.fc_sdf_query(b, pose, fused_out=out_e)
        torch.cuda.synchronize()
        assert_same(to_np(out_e), ref_o)
    del graph
