"""GPU parity of the forward path (query + reduction) against the CPU oracle,
through the C ABI.  Tolerances are in _gpu_common."""
import math

import numpy as np
import pytest

from _gpu_common import (assert_same, check_candidates, check_points, check_reduction_exact, to_np,
                         torch_gpu)
from paper_2205_03532_amd import fc
from paper_2205_03532_amd import workloads as W

pytestmark = pytest.mark.gpu


def run(batch, pose, cand=True, fused=True):
    torch = torch_gpu()
    c = batch.new_candidates() if cand else None
    o = batch.new_contacts() if fused else None
    fc.fc_sdf_query(batch, pose, cand=c, fused_out=o)
    torch.cuda.synchronize()
    return (to_np(c) if cand else None), (to_np(o) if fused else None)


def run_unfused(batch, pose):
    torch = torch_gpu()
    c = batch.new_candidates()
    o = batch.new_contacts()
    fc.fc_sdf_query(batch, pose, cand=c)
    fc.fc_contact_reduce(batch, pose, c, o)
    torch.cuda.synchronize()
    return to_np(c), to_np(o)


@pytest.fixture(scope="module")
def torus():
    torch_gpu()
    w = W.torus_workload()
    return w, fc.Batch.from_workload(w), fc.pose_tensor(w.pose)


@pytest.fixture(scope="module")
def nutbolt24():
    torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(24))
    return w, fc.Batch.from_workload(w), fc.pose_tensor(w.pose)


def test_torus_candidates_match_oracle(torus):
    w, b, pose = torus
    c, _ = run(b, pose, fused=False)
    st = check_candidates(w, c, range(w.n_env))
    print("torus 64^3, 256 envs x 2562:", st)
    assert st["cand"] > 10000


def test_torus_reduction_exact_fused_and_unfused(torus):
    w, b, pose = torus
    c, o_unf = run_unfused(b, pose)
    _, o_fused = run(b, pose, cand=False)
    check_reduction_exact(w, c, o_unf, range(w.n_env))
    check_points(w, o_unf, range(w.n_env))
    assert_same(o_fused, o_unf)
    assert o_fused["count"].sum() > 0


def test_torus_both_outputs_in_one_launch(torus):
    w, b, pose = torus
    c1, o1 = run(b, pose, cand=True, fused=True)
    c2, _ = run(b, pose, fused=False)
    _, o2 = run(b, pose, cand=False)
    assert_same(c1, c2)
    assert_same(o1, o2)


def test_deterministic_and_workspace_returns_to_zero(torus):
    torch = torch_gpu()
    w, b, pose = torus
    _, o1 = run(b, pose, cand=False)
    assert int(torch.count_nonzero(b.workspace)) == 0
    _, o2 = run(b, pose, cand=False)
    assert_same(o1, o2)


def test_nutbolt_candidates_and_reduction(nutbolt24):
    w, b, pose = nutbolt24
    c, o = run_unfused(b, pose)
    st = check_candidates(w, c, range(w.n_env))
    print("nut-bolt 256x256x512, 24 envs x 16396:", st)
    assert st["cand"] > 1000
    check_reduction_exact(w, c, o, range(w.n_env))
    check_points(w, o, range(w.n_env))
    _, of = run(b, pose, cand=False)
    assert_same(of, o)


@pytest.mark.parametrize("shape", [
    dict(block=128, tile=128, persistent=0, grid_mult=8),
    dict(block=256, tile=512, persistent=1, grid_mult=2),
    dict(block=512, tile=2048, persistent=2, grid_mult=4),
    dict(block=128, tile=512, persistent=2, grid_mult=1),
    dict(block=256, tile=256, persistent=1, grid_mult=32),
    dict(block=256, tile=1024, persistent=0, grid_mult=8, xcd_remap=1),
    dict(block=256, tile=1024, persistent=1, grid_mult=4, xcd_remap=1),
    dict(block=256, tile=1024, persistent=2, grid_mult=8, xcd_remap=1),
    dict(block=512, tile=512, persistent=2, grid_mult=1, xcd_remap=1),
])
def test_launch_shapes_bit_identical(nutbolt24, shape):
    w, b, pose = nutbolt24
    ref_c, ref_o = run(b, pose)
    old = b.get_launch()
    try:
        b.set_launch(**shape)
        for _ in range(2):  # second run checks the persistent counters were reset
            c, o = run(b, pose)
            assert_same(c, ref_c)
            assert_same(o, ref_o)
    finally:
        b.set_launch(**old)


@pytest.mark.parametrize("xcd", [0, 1])
def test_env_chunked_forward_bit_identical(nutbolt24, torus, xcd):
    """persistent = 3: the fused forward on the adjoint's env-chunked items
    gives the contacts of the per-item kernel, bit for bit, call after call."""
    for w, b, pose in (nutbolt24, torus):
        _, ref = run(b, pose, cand=False)
        old = b.get_launch()
        try:
            b.set_launch(**dict(old, persistent=3, xcd_remap=xcd))
            for _ in range(2):
                _, o = run(b, pose, cand=False)
                assert_same(o, ref)
            c, o = run(b, pose)  # with candidates requested the per-item kernel runs
            assert_same(o, ref)
            for _ in range(2):  # candidates alone, then the reduction: per-item kernel, plain launches
                c, o = run_unfused(b, pose)
                assert_same(o, ref)
        finally:
            b.set_launch(**old)


def test_env_order_does_not_change_contacts(nutbolt24):
    w, b, pose = nutbolt24
    ref_c, ref_o = run(b, pose)
    for order in (fc.locality_order(w), np.arange(w.n_env)[::-1].copy()):
        bo = fc.Batch.from_workload(w, env_order=order)
        bo.set_launch(block=256, tile=1024, persistent=2, grid_mult=8, xcd_remap=1)
        c, o = run(bo, pose)
        assert_same(c, ref_c)
        assert_same(o, ref_o)


@pytest.mark.parametrize("layout", ["brick", "slab"])
def test_brick_layouts_bit_identical(nutbolt24, layout):
    w, b, pose = nutbolt24
    ref_c, ref_o = run(b, pose)
    bb = fc.Batch.from_workload(w, layout=layout)
    c, o = run(bb, pose)
    assert_same(c, ref_c)
    assert_same(o, ref_o)
    g_ref, g_b = b.new_grads(per_env=True), bb.new_grads(per_env=True)
    fc.fc_sdf_query_backward(b, pose, 1e4, g_ref)
    fc.fc_sdf_query_backward(bb, pose, 1e4, g_b)
    assert_same(to_np({k: v for k, v in g_b.items() if k != "per_env"}),
                to_np({k: v for k, v in g_ref.items() if k != "per_env"}))


def _sphere_grid(n=24, h=1.0 / 16):
    o = -h * (n - 1) / 2
    return W.sample_grid(lambda p: W.field_sphere(p, (0, 0, 0), 0.5), (n, n, n), (o, o, o), h)


def test_ragged_and_empty_meshes_mixed_batch():
    torch_gpu()
    rng = np.random.default_rng(5)
    grids = [_sphere_grid(), W.sample_grid(lambda p: W.field_torus(p, 0.4, 0.15), (20, 22, 18), (-0.7, -0.75, -0.6),
                                           0.07)]
    sizes = [0, 1, 63, 65, 1025, 2049]
    meshes = [W.Mesh(verts=rng.uniform(-0.7, 0.7, (n, 3)).astype(np.float32)) for n in sizes]
    n_env = 40
    eg = rng.integers(0, 2, n_env).astype(np.int32)
    em = rng.integers(0, len(sizes), n_env).astype(np.int32)
    q = W.shoemake_quat(rng, n_env)
    t = rng.uniform(-0.1, 0.1, (3, n_env))
    w = W.Workload("ragged", grids, meshes, eg, em, W.pack_pose(q, t), W.fibonacci_bins(16), 0.0)
    b = fc.Batch.from_workload(w)
    pose = fc.pose_tensor(w.pose)
    for shape in (dict(block=256, tile=1024, persistent=0, grid_mult=8),
                  dict(block=128, tile=256, persistent=2, grid_mult=2)):
        b.set_launch(**shape)
        c, o = run_unfused(b, pose)
        check_candidates(w, c, range(n_env))
        check_reduction_exact(w, c, o, range(n_env))
        _, of = run(b, pose, cand=False)
        assert_same(of, o)
        empty = [e for e in range(n_env) if sizes[em[e]] == 0]
        assert empty and all(o["count"][e] == 0 for e in empty)
        assert all(np.all(o["vidx"][e * 16:(e + 1) * 16] == -1) for e in empty)


def test_ties_go_to_lowest_vertex_index():
    """Half-space grid, vertices on a plane: every candidate has the same depth."""
    torch_gpu()
    h = 1.0 / 32
    g = W.sample_grid(lambda p: p[..., 2] - 0.25, (33, 33, 33), (-0.5, -0.5, -0.5), h)
    rng = np.random.default_rng(6)
    n = 3000
    v = np.c_[rng.uniform(-0.4, 0.4, (n, 2)), np.full(n, 0.125)].astype(np.float32)
    pose = np.zeros((7, 3), np.float32)
    pose[3] = 1.0
    w = W.Workload("ties", [g], [W.Mesh(verts=v)], np.zeros(3, np.int32), np.zeros(3, np.int32), pose,
                   W.fibonacci_bins(8), 0.0)
    b = fc.Batch.from_workload(w)
    c, o = run_unfused(b, fc.pose_tensor(pose))
    check_reduction_exact(w, c, o, range(3))
    for e in range(3):
        full = o["vidx"][e * 8:(e + 1) * 8] >= 0
        assert full.sum() == 1  # one normal direction
        assert o["vidx"][e * 8:(e + 1) * 8][full][0] == 0


def test_nan_and_outside_are_never_candidates():
    torch_gpu()
    g = _sphere_grid()
    v = np.array([[0, 0, 0], [np.nan, 0, 0], [5, 5, 5], [0.1, 0.1, 0.1]], np.float32)
    pose = np.zeros((7, 3), np.float32)
    pose[3] = 1.0
    pose[4, 1] = np.nan  # env 1 has a NaN translation
    w = W.Workload("nan", [g], [W.Mesh(verts=v)], np.zeros(3, np.int32), np.zeros(3, np.int32), pose,
                   W.fibonacci_bins(4), 0.0)
    b = fc.Batch.from_workload(w)
    c, o = run_unfused(b, fc.pose_tensor(pose))
    assert c["bin"][1] == -1 and c["bin"][2] == -1 and np.isinf(c["phi"][1]) and np.isinf(c["phi"][2])
    assert np.all(c["bin"][4:8] == -1)  # whole env 1
    assert c["bin"][0] >= 0 and c["bin"][3] >= 0
    assert o["count"][1] == 0 and o["count"][0] >= 1


@pytest.mark.parametrize("K", [1, 64])
def test_bin_count_extremes(torus, K):
    w0, _, _ = torus
    w = W.subset(w0, range(16))
    w = W.Workload(w.name, w.grids, w.meshes, w.env_grid, w.env_mesh, w.pose, W.fibonacci_bins(K), w.margin)
    b = fc.Batch.from_workload(w)
    c, o = run_unfused(b, fc.pose_tensor(w.pose))
    check_candidates(w, c, range(16))
    check_reduction_exact(w, c, o, range(16))


def test_positive_margin(torus):
    w0, _, _ = torus
    w = W.subset(w0, range(16))
    w.margin = 0.002
    b = fc.Batch.from_workload(w)
    c, o = run_unfused(b, fc.pose_tensor(w.pose))
    st = check_candidates(w, c, range(16))
    check_reduction_exact(w, c, o, range(16))
    # some winners are not penetrating (depth < 0) yet within the margin
    assert np.any((o["vidx"] >= 0) & (o["depth"] < 0))
    assert math.isfinite(st["max_depth_err"])
