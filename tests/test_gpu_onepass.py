"""GPU parity of fc_sdf_query_and_backward, the one-pass query + adjoint:
every output is bit-identical to fc_sdf_query (fused) followed by
fc_sdf_query_backward on the same inputs, across workloads, storage types,
layouts, scheduling options, vertex-gradient modes and upstream weights, and
the contacts also match the oracle's exact reduction."""
import numpy as np
import pytest

from _gpu_common import assert_same, check_candidates, check_points, check_reduction_exact, to_np, torch_gpu
from paper_2205_03532_amd import fc
from paper_2205_03532_amd import workloads as W

pytestmark = pytest.mark.gpu
KP = 1e4


def separate(batch, pose, per_env=False, upstream=None):
    torch = torch_gpu()
    o = batch.new_contacts()
    g = batch.new_grads(per_env=per_env)
    fc.fc_sdf_query(batch, pose, fused_out=o)
    fc.fc_sdf_query_backward(batch, pose, KP, g, upstream=upstream)
    torch.cuda.synchronize()
    return to_np(o), to_np({k: v for k, v in g.items() if k != "per_env"})


def onepass(batch, pose, per_env=False, upstream=None):
    torch = torch_gpu()
    o = batch.new_contacts()
    g = batch.new_grads(per_env=per_env)
    fc.fc_sdf_query_and_backward(batch, pose, o, KP, g, upstream=upstream)
    torch.cuda.synchronize()
    return to_np(o), to_np({k: v for k, v in g.items() if k != "per_env"})


def check_identical(batch, pose, per_env=False, upstream=None):
    o1, g1 = separate(batch, pose, per_env, upstream)
    o2, g2 = onepass(batch, pose, per_env, upstream)
    assert_same(o1, o2)
    assert_same(g1, g2)
    return o2, g2


def upstream_for(n_env, seed):
    torch = torch_gpu()
    u = np.random.default_rng(seed).uniform(0.25, 2.0, n_env).astype(np.float32)
    return torch.from_numpy(u).cuda()


def test_torus_identical_and_oracle_exact():
    torch_gpu()
    w = W.subset(W.torus_workload(), range(64))
    b = fc.Batch.from_workload(w)
    pose = fc.pose_tensor(w.pose)
    o, g = check_identical(b, pose)
    assert int(o["count"].sum()) > 0 and float(np.abs(g["d_pose"]).sum()) > 0
    # contacts against the oracle's reduction of the GPU's own candidates
    c = b.new_candidates()
    fc.fc_sdf_query(b, pose, cand=c)
    torch_gpu().cuda.synchronize()
    c = to_np(c)
    envs = range(w.n_env)
    check_candidates(w, c, envs)
    check_reduction_exact(w, c, o, envs)
    check_points(w, o, envs)


@pytest.mark.parametrize("layout,xcd,order", [("linear", 0, False), ("brick", 1, True), ("slab", 0, True)])
def test_nutbolt_identical(layout, xcd, order):
    torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(48))
    b = fc.Batch.from_workload(w, layout=layout, env_order=fc.locality_order(w) if order else None)
    b.set_launch(block=256, tile=1024, persistent=0, grid_mult=8, xcd_remap=xcd)
    pose = fc.pose_tensor(w.pose)
    o, g = check_identical(b, pose)
    assert int(o["count"].sum()) > 0
    check_identical(b, pose, per_env=True, upstream=upstream_for(w.n_env, 7))


def test_ragged_tail_and_upstream():
    """The full nut (16,396 vertices = 32 tiles of 512 + a 12-vertex tail),
    a chunk that is not full (40 envs = 32 + 8) and nonuniform upstream weights."""
    torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(40))
    b = fc.Batch.from_workload(w, layout="brick")
    pose = fc.pose_tensor(w.pose)
    check_identical(b, pose, upstream=upstream_for(w.n_env, 3))


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_mixed_half_identical(dtype):
    torch_gpu()
    w = W.half_storage(W.subset(W.mixed_workload(), range(0, 4096, 16)), dtype)
    b = fc.Batch.from_workload(w, layout="brick")
    pose = fc.pose_tensor(w.pose)
    o, g = check_identical(b, pose)
    assert int(o["count"].sum()) > 0
    check_identical(b, pose, per_env=True)


def test_margin_and_k64():
    """Positive margin (candidates that do not penetrate: in the contacts, not in
    the penalty) and the largest bin count."""
    torch_gpu()
    w = W.subset(W.torus_workload(), range(32))
    w.margin = np.float32(2e-4)
    w.bins = W.fibonacci_bins(64)
    b = fc.Batch.from_workload(w)
    pose = fc.pose_tensor(w.pose)
    check_identical(b, pose)


def test_repeated_calls_leave_workspace_clean():
    """The one-pass call resets the keys like the forward: alternating it with
    the separate calls on one workspace keeps giving identical results."""
    torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(16))
    b = fc.Batch.from_workload(w, layout="brick")
    pose = fc.pose_tensor(w.pose)
    ref = separate(b, pose)
    for _ in range(3):
        o, g = onepass(b, pose)
        assert_same(ref[0], o)
        assert_same(ref[1], g)
        o, g = separate(b, pose)
        assert_same(ref[0], o)
        assert_same(ref[1], g)


def test_graph_of_both_equals_eager():
    """A graph holding both outputs captures the one-pass call; each replay,
    with eager work in between, equals the eager separate calls."""
    torch = torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(24))
    b = fc.Batch.from_workload(w, layout="brick")
    pose = fc.pose_tensor(w.pose)
    ref_o, ref_g = separate(b, pose)
    o = b.new_contacts()
    g = b.new_grads()
    graph = fc.fc_graph_create(b, pose, fused_out=o, k=KP, grads=g)
    for _ in range(3):
        for t in list(o.values()) + [v for k, v in g.items() if k != "per_env"]:
            t.fill_(7)
        graph.launch()
        torch.cuda.synchronize()
        assert_same(ref_o, to_np(o))
        assert_same(ref_g, to_np({k: v for k, v in g.items() if k != "per_env"}))
        separate(b, pose)  # eager work between replays


def test_kernel_timing_records_main_kernels_only():
    """fc_batch_set_timing records one event pair per compute call, in call
    order with the kernel ids; graph replays are not recorded."""
    torch = torch_gpu()
    w = W.subset(W.torus_workload(), range(16))
    b = fc.Batch.from_workload(w)
    pose = fc.pose_tensor(w.pose)
    o = b.new_contacts()
    g = b.new_grads()
    b.set_timing(8)
    fc.fc_sdf_query_and_backward(b, pose, o, KP, g)
    fc.fc_sdf_query(b, pose, fused_out=o)
    fc.fc_sdf_query_backward(b, pose, KP, g)
    ms, kid = b.read_timing()
    assert list(kid) == [fc.FC_KERNEL_QUERY_BACKWARD, fc.FC_KERNEL_FORWARD, fc.FC_KERNEL_BACKWARD]
    assert np.all(ms > 0) and np.all(ms < 1e3)
    graph = fc.fc_graph_create(b, pose, fused_out=o, k=KP, grads=g)
    graph.launch()
    torch.cuda.synchronize()
    assert len(b.read_timing()[0]) == 0  # capture and replay record nothing
    for _ in range(10):  # more calls than slots: the first 8 are kept
        fc.fc_sdf_query(b, pose, fused_out=o)
    ms, kid = b.read_timing()
    assert len(ms) == 8 and set(kid) == {fc.FC_KERNEL_FORWARD}
    b.set_timing(0)
    fc.fc_sdf_query(b, pose, fused_out=o)
    assert len(b.read_timing()[0]) == 0


def test_gather_probe_writes_nothing_and_is_timed():
    """The gather probe (the one-pass loop without its arithmetic) leaves its
    sink and every output untouched and is recorded under its own kernel id."""
    torch = torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(24))
    b = fc.Batch.from_workload(w, layout="brick")
    pose = fc.pose_tensor(w.pose)
    sink = torch.full((4,), 7.0, device="cuda")
    ws_before = b.workspace.clone()
    b.set_timing(2)
    fc.fc_gather_probe(b, pose, sink)
    fc.fc_gather_probe(b, pose, sink)
    ms, kid = b.read_timing()
    b.set_timing(0)
    assert list(kid) == [fc.FC_KERNEL_GATHER_PROBE] * 2 and np.all(ms > 0)
    assert torch.equal(sink, torch.full((4,), 7.0, device="cuda"))
    assert torch.equal(b.workspace, ws_before)


def test_layout_tuner_steps_are_bit_identical_across_layouts():
    """The layout tuner on a mixed batch (five grids, five meshes' shared
    vertex gradients): brick, slab and linear give the same contacts, loss,
    twists and vertex gradients bit for bit (the tuner raises otherwise), and
    it records the fastest under the layout-free key."""
    torch_gpu()
    from paper_2205_03532_amd import autotune

    w = W.subset(W.mixed_workload(), range(60))
    lay, entries = autotune.tune_layouts(w, reps=3, warmup=1, shapes=[autotune.DEFAULT], log=print)
    assert set(lay["step_ms"]) == set(autotune.LAYOUTS)
    assert lay["layout"] == autotune.pick_layout(lay["step_ms"])
    assert len(entries) == len(autotune.LAYOUTS) and len({e["key"] for e in entries}) == len(autotune.LAYOUTS)
    assert {autotune.layout_key(e["key"]) for e in entries} == {lay["key"]}


@pytest.mark.parametrize("workload,layout", [("nutbolt", "brick"), ("nutbolt", "sparse"), ("mixed", "slab")])
def test_wave_priority_modes_are_bit_identical(workload, layout):
    """Every wave priority mode (none, raised while a wave issues its corner
    loads, raised while it evaluates) gives the same outputs bit for bit: the
    one-pass step (shared and per-env vertex gradients), the separate adjoint
    and the env-chunked forward."""
    torch = torch_gpu()
    w = (W.subset(W.nut_bolt_workload(), range(40)) if workload == "nutbolt"
         else W.subset(W.mixed_workload(), range(0, 4096, 32)))
    b = fc.Batch.from_workload(w, layout=layout, env_order=fc.locality_order(w))
    pose = fc.pose_tensor(w.pose)
    shape = b.get_launch()
    assert shape["wave_prio"] == 1
    ref = None
    for p in (1, 0, 2):
        b.set_launch(**dict(shape, wave_prio=p))
        assert b.get_launch()["wave_prio"] == p
        res = [*onepass(b, pose), *onepass(b, pose, per_env=True, upstream=upstream_for(w.n_env, 5)),
               *separate(b, pose)]
        b.set_launch(**dict(shape, persistent=3, wave_prio=p))
        o = b.new_contacts()
        fc.fc_sdf_query(b, pose, fused_out=o)
        torch.cuda.synchronize()
        res.append(to_np(o))
        if ref is None:
            ref = res
            assert int(res[0]["count"].sum()) > 0
        else:
            for x, y in zip(ref, res):
                assert_same(x, y)
    with pytest.raises(RuntimeError):
        b.set_launch(**dict(shape, wave_prio=3))


def test_cache_entry_sets_the_wave_priority(tmp_path):
    """A loaded cache entry's wave_prio applies to batches created afterwards
    with that signature; an entry without one gives the default (1)."""
    import json

    torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(8))
    b = fc.Batch.from_workload(w, layout="brick")
    sig = b.signature()
    del b
    p = tmp_path / "c.json"
    try:
        for entry, want in ((dict(wave_prio=2), 2), ({}, 1), (dict(wave_prio=0), 0)):
            p.write_text(json.dumps({"entries": [dict(key=sig, block=256, tile=1024, persistent=0, grid_mult=8,
                                                      xcd_remap=1, **entry)]}))
            assert fc.fc_autotune_load(str(p)) == 1
            b = fc.Batch.from_workload(w, layout="brick")
            assert b.get_launch() == dict(block=256, tile=1024, persistent=0, grid_mult=8, xcd_remap=1,
                                          wave_prio=want)
            del b
    finally:  # later batches of this signature start from the library's default again
        p.write_text(json.dumps({"entries": [dict(key=sig, block=256, tile=1024, persistent=0, grid_mult=8,
                                                  xcd_remap=0, wave_prio=1)]}))
        assert fc.fc_autotune_load(str(p)) == 1
