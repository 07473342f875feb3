"""Full-size workloads in the launch configuration bench.py times, checked
against the oracle on sampled envs and by properties that hold at any size."""
import numpy as np
import pytest

from _gpu_common import assert_same, check_candidates, check_reduction_exact, rows_of, to_np, torch_gpu
import bench
from paper_2205_03532_amd import fc
from paper_2205_03532_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    torch_gpu()
    w = W.nut_bolt_workload()
    b = bench.make_batch(w, "cuda:0")
    return w, b, fc.pose_tensor(w.pose)


def test_bench_batch_contacts_match_oracle_on_sampled_envs(full):
    torch = torch_gpu()
    w, b, pose = full
    c, o = b.new_candidates(), b.new_contacts()
    fc.fc_sdf_query(b, pose, cand=c, fused_out=o)
    torch.cuda.synchronize()
    c, o = to_np(c), to_np(o)
    rng = np.random.default_rng(7)
    envs = sorted(int(e) for e in rng.choice(w.n_env, 12, replace=False))
    st = check_candidates(w, c, envs)
    print("full nut-bolt, sampled envs:", st)
    check_reduction_exact(w, c, o, envs)
    # any size: counts equal non-empty slots, every winner is a candidate of its bin
    K = w.K
    assert np.array_equal(o["count"], (o["vidx"].reshape(-1, K) >= 0).sum(1))
    off = w.env_query_offsets()
    e_idx = np.repeat(np.arange(w.n_env), K)
    full_slots = o["vidx"] >= 0
    q = off[e_idx[full_slots]] + o["vidx"][full_slots]
    assert np.array_equal(c["bin"][q], np.tile(np.arange(K), w.n_env)[full_slots])
    d = (-c["phi"][q]).astype(np.float32)
    d[d == 0] = np.float32(0.0)
    assert np.array_equal(d.view(np.uint32), o["depth"][full_slots].view(np.uint32))

def test_bench_batch_fused_equals_unfused_and_repeats(full):
    torch = torch_gpu()
    w, b, pose = full
    o1, o2, o3 = b.new_contacts(), b.new_contacts(), b.new_contacts()
    c = b.new_candidates()
    fc.fc_sdf_query(b, pose, fused_out=o1)
    fc.fc_sdf_query(b, pose, cand=c)
    fc.fc_contact_reduce(b, pose, c, o2)
    fc.fc_sdf_query(b, pose, fused_out=o3)
    torch.cuda.synchronize()
    assert_same(to_np(o1), to_np(o2))
    assert_same(to_np(o1), to_np(o3))


def test_bench_batch_adjoint_repeats_and_matches_subset(full):
    """The shared gradient at full size is reproducible; per-env outputs equal
    a batch built from sampled envs alone (bit for bit)."""
    torch = torch_gpu()
    w, b, pose = full
    g1, g2 = b.new_grads(per_env=False), b.new_grads(per_env=False)
    fc.fc_sdf_query_backward(b, pose, 1e4, g1)
    fc.fc_sdf_query_backward(b, pose, 1e4, g2)
    torch.cuda.synchronize()
    a1 = to_np({k: v for k, v in g1.items() if k != "per_env"})
    a2 = to_np({k: v for k, v in g2.items() if k != "per_env"})
    assert_same(a1, a2)
    envs = np.arange(0, w.n_env, 97)
    sub = W.subset(w, envs)
    bs = fc.Batch.from_workload(sub)
    gs = bs.new_grads(per_env=False)
    fc.fc_sdf_query_backward(bs, fc.pose_tensor(sub.pose), 1e4, gs)
    torch.cuda.synchronize()
    # loss and twist gradients depend only on the env itself
    assert np.array_equal(gs["loss"].cpu().numpy(), a1["loss"][envs])
    assert np.array_equal(gs["d_pose"].cpu().numpy(), a1["d_pose"][:, envs])


def test_bench_step_one_pass_equals_separate_calls(full):
    """The step bench.py times (one fc_sdf_query_and_backward pass) gives the
    contacts and gradients of the separate calls, bit for bit, at full size."""
    torch = torch_gpu()
    w, b, pose = full
    o1, o2 = b.new_contacts(), b.new_contacts()
    g1, g2 = b.new_grads(per_env=False), b.new_grads(per_env=False)
    fc.fc_sdf_query(b, pose, fused_out=o1)
    fc.fc_sdf_query_backward(b, pose, 1e4, g1)
    fc.fc_sdf_query_and_backward(b, pose, o2, 1e4, g2)
    torch.cuda.synchronize()
    assert_same(to_np(o1), to_np(o2))
    assert_same(to_np({k: v for k, v in g1.items() if k != "per_env"}),
                to_np({k: v for k, v in g2.items() if k != "per_env"}))
    assert int(to_np(o2)["count"].sum()) > 0
