"""The Python binding checks every tensor it hands to the C ABI (device,
dtype, shape, contiguity) before the call: the library receives bare device
pointers and cannot.  CPU only: a stand-in batch on the CPU device, and
tensors on the CPU and meta devices."""
from types import SimpleNamespace

import pytest

torch = pytest.importorskip("torch")

from paper_2205_03532_amd import fc  # noqa: E402

N_ENV, K, Q, QF = 3, 4, 10, 6


def batch():
    return SimpleNamespace(device=torch.device("cpu"), n_env=N_ENV, K=K, Q=Q, Qf=QF, mesh_sizes=[2, 3],
                           handle=None, workspace=None, ws_bytes=0)


def pose():
    return torch.zeros(7, N_ENV)


def contacts(S=N_ENV * K):
    return dict(vidx=torch.zeros(S, dtype=torch.int32), depth=torch.zeros(S), point=torch.zeros(3, S),
                normal=torch.zeros(3, S), count=torch.zeros(N_ENV, dtype=torch.int32))


def candidates(n=Q, point=False):
    c = dict(phi=torch.zeros(n), normal=torch.zeros(3, n), bin=torch.zeros(n, dtype=torch.int16))
    if point:
        c["point"] = torch.zeros(3, n)
    return c


def grads(per_env=False):
    nv = Q if per_env else 5
    return dict(loss=torch.zeros(N_ENV), d_pose=torch.zeros(6, N_ENV), d_verts=torch.zeros(3 * nv), per_env=per_env)


def patches(N):
    S = N_ENV * N
    i32 = dict(dtype=torch.int32)
    return dict(count=torch.zeros(N_ENV, **i32), founder=torch.zeros(S, **i32), normal=torch.zeros(3, S),
                vidx=torch.zeros(S, **i32), depth=torch.zeros(S), point=torch.zeros(3, S),
                members=torch.zeros(S, **i32))


def test_valid_arguments_pass():
    b = batch()
    fc._check_pose(b, pose())
    fc._check_candidates(b, candidates())
    fc._check_candidates(b, candidates(QF, point=True), faces=True)
    fc._check_contacts(b, contacts())
    fc._check_grads(b, grads(), torch.ones(N_ENV))
    fc._check_grads(b, grads(per_env=True), None)
    fc._check_grads(b, dict(loss=torch.zeros(N_ENV), d_pose=None, d_verts=None), None)
    fc._check_patches(b, patches(8), 8)


@pytest.mark.parametrize("bad", [
    torch.zeros(N_ENV, 7),  # AoS pose with the right element count
    torch.zeros(7, N_ENV, dtype=torch.float64),
    torch.zeros(7, 2 * N_ENV)[:, ::2],  # strided view
    torch.zeros(7, N_ENV, device="meta"),  # another device
    [[0.0] * N_ENV] * 7,
])
def test_bad_pose_is_rejected_before_the_call(bad):
    b = batch()
    with pytest.raises((ValueError, TypeError)):
        fc.fc_sdf_query(b, bad, fused_out=contacts())
    with pytest.raises((ValueError, TypeError)):
        fc.fc_sdf_query_backward(b, bad, 1e4, grads())


def test_bad_outputs_are_rejected_before_the_call():
    b = batch()
    with pytest.raises(ValueError, match="contacts\\['count'\\]"):
        c = contacts()
        c["count"] = torch.zeros(N_ENV, dtype=torch.int64)
        fc.fc_sdf_query(b, pose(), fused_out=c)
    with pytest.raises(ValueError, match="cand\\['bin'\\]"):
        c = candidates()
        c["bin"] = torch.zeros(Q, dtype=torch.int32)
        fc.fc_contact_reduce(b, pose(), c, contacts())
    with pytest.raises(ValueError, match="grads\\['d_verts'\\]"):
        fc.fc_sdf_query_backward(b, pose(), 1e4, grads(per_env=False) | dict(per_env=True))
    with pytest.raises(ValueError, match="upstream"):
        fc.fc_sdf_query_and_backward(b, pose(), contacts(), 1e4, grads(), upstream=torch.ones(N_ENV + 1))
    with pytest.raises(ValueError, match="cand\\['point'\\]"):
        fc.fc_sdf_query_faces(b, pose(), cand=candidates(QF))
    with pytest.raises(ValueError, match="contacts\\['point'\\]"):
        c = contacts()
        c["point"] = torch.zeros(N_ENV * K, 3).t()  # right shape, not contiguous
        fc.fc_sdf_query_and_backward(b, pose(), c, 1e4, grads())


def test_patch_outputs_must_match_max_patches():
    """Outputs made for 128 patches per env with max_patches = 256 would let
    the kernel write past them: rejected."""
    b = batch()
    with pytest.raises(ValueError, match="patches"):
        fc.fc_contact_patches(b, pose(), patches(128), max_patches=256)
