"""fc_sdf_query_noalloc (the forward on the library's static per-device
scratch, no workspace argument) through the C ABI: bit-identical to
fc_sdf_query on the same batch, on two calls in a row of which the second
has a smaller batch (the scratch keeps the first call's contents), in every
scheduling mode the forward has; a batch needing more than the scratch is
rejected before any launch."""
import numpy as np
import pytest

from _gpu_common import assert_same, to_np, torch_gpu
from paper_2205_03532_amd import fc
from paper_2205_03532_amd import workloads as W

pytestmark = pytest.mark.gpu


def reference(b, pose):
    torch = torch_gpu()
    c, o = b.new_candidates(), b.new_contacts()
    fc.fc_sdf_query(b, pose, cand=c)
    fc.fc_sdf_query(b, pose, fused_out=o)
    torch.cuda.synchronize()
    return to_np(c), to_np(o)


def noalloc(b, pose):
    torch = torch_gpu()
    c, o = b.new_candidates(), b.new_contacts()
    for t in list(c.values()) + list(o.values()):
        t.fill_(7)
    fc.fc_sdf_query_noalloc(b, pose, cand=c)
    fc.fc_sdf_query_noalloc(b, pose, fused_out=o)
    torch.cuda.synchronize()
    return to_np(c), to_np(o)


@pytest.mark.parametrize("launch", [
    dict(block=256, tile=1024, persistent=0, grid_mult=8, xcd_remap=0),
    dict(block=256, tile=512, persistent=2, grid_mult=4, xcd_remap=1),
    dict(block=256, tile=1024, persistent=3, grid_mult=8, xcd_remap=1),
])
def test_two_calls_second_smaller_equal_workspace_calls(launch):
    torch_gpu()
    big = W.subset(W.nut_bolt_workload(), range(0, 1000, 16))  # 63 envs x 16,396 vertices, K = 32
    small = W.subset(W.torus_workload(), range(10))  # 10 envs x 2,562 vertices, K = 16
    batches = []
    for w in (big, small):
        b = fc.Batch.from_workload(w, layout="brick")
        b.set_launch(**launch)
        batches.append((b, fc.pose_tensor(w.pose)))
    refs = [reference(b, p) for b, p in batches]
    for (b, p), (rc, ro) in zip(batches, refs):
        assert fc.lib().fc_sdf_query_noalloc_bytes(b.handle) <= fc.NOALLOC_SCRATCH_BYTES
        c, o = noalloc(b, p)
        assert_same(c, rc)
        assert_same(o, ro)
        assert int(ro["count"].sum()) > 0
    # and again, in the other order: the larger batch after the smaller one
    for (b, p), (rc, ro) in reversed(list(zip(batches, refs))):
        c, o = noalloc(b, p)
        assert_same(c, rc)
        assert_same(o, ro)


def test_batch_beyond_the_scratch_is_rejected():
    torch = torch_gpu()
    w = W.subset(W.torus_workload(), np.zeros(8200, np.int64))
    w.bins = W.fibonacci_bins(64)  # 8,200 x 64 keys x 8 B > 4 MiB
    b = fc.Batch.from_workload(w)
    assert fc.lib().fc_sdf_query_noalloc_bytes(b.handle) > fc.NOALLOC_SCRATCH_BYTES
    o = b.new_contacts()
    o["count"].fill_(-3)
    with pytest.raises(fc.FcError) as ei:
        fc.fc_sdf_query_noalloc(b, fc.pose_tensor(w.pose), fused_out=o)
    assert ei.value.status == fc.FC_ERR_SCRATCH
    torch.cuda.synchronize()
    assert int((o["count"] == -3).sum()) == w.n_env  # nothing written
