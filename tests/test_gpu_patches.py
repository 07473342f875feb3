"""GPU parity of the patch reduction (fc_contact_patches, Algorithm 1)
through the C ABI.

The patch decisions compare FP32 normal dots with the threshold, so both
sides take them in FP32 on the same normals: the oracle (oracle/patches.py)
runs Algorithm 1 on the candidates fc_sdf_query returns (whose values the
other parity tests check against the FP64 oracle), and every output must
match bit for bit: patch count, founders, members, normals, deepest members
and their depths.  Points are the FP64 transform of the deepest vertex
within FP32 rounding."""
import numpy as np
import pytest

from _gpu_common import to_np, torch_gpu
from oracle import patches as OP
from oracle import query as OQ
from paper_2205_03532_amd import fc
from paper_2205_03532_amd import workloads as W

pytestmark = pytest.mark.gpu


def run(b, pose, n_max, cos_sim):
    torch = torch_gpu()
    c = b.new_candidates()
    fc.fc_sdf_query(b, pose, cand=c)
    out = b.new_patches(n_max)
    fc.fc_contact_patches(b, pose, out, max_patches=n_max, cos_sim=cos_sim)
    torch.cuda.synchronize()
    return to_np(c), to_np(out)


def check_patches(w, cand, out, n_max, cos_sim, envs):
    off = w.env_query_offsets()
    stats = dict(patches=0, members=0, dropped=0, cand=0)
    for e in envs:
        rows = np.arange(off[e], off[e + 1])
        isc = cand["bin"][rows] >= 0
        v = np.nonzero(isc)[0]
        depth = (-cand["phi"][rows][isc]).astype(np.float32)
        nrm = cand["normal"][:, rows][:, isc].T.astype(np.float32)
        patches, dropped = OP.reduce_env(v, depth, nrm, np.float32(cos_sim), n_max)
        assert out["count"][e] == len(patches), (e, out["count"][e], len(patches))
        s = slice(e * n_max, (e + 1) * n_max)
        k = len(patches)
        assert np.array_equal(out["founder"][s][:k], [p["founder"] for p in patches]), e
        assert np.array_equal(out["members"][s][:k], [p["members"] for p in patches]), e
        assert np.array_equal(out["vidx"][s][:k], [OP.key_vidx(p["key"]) for p in patches]), e
        dk = np.array([OP.key_depth(p["key"]) for p in patches], dtype=np.float32)
        assert np.array_equal(out["depth"][s][:k].view(np.uint32), dk.view(np.uint32)), e
        nk = np.array([p["normal"] for p in patches], dtype=np.float32).reshape(-1, 3)
        assert np.array_equal(out["normal"][:, s][:, :k].T.view(np.uint32), nk.view(np.uint32)), e
        assert np.all(out["founder"][s][k:] == -1) and np.all(out["vidx"][s][k:] == -1)
        assert np.all(out["members"][s][k:] == 0) and np.all(out["depth"][s][k:] == 0)
        stats["patches"] += k
        stats["members"] += int(out["members"][s][:k].sum())
        stats["dropped"] += dropped
        stats["cand"] += int(isc.sum())
        assert stats["members"] + stats["dropped"] == stats["cand"]
    # points: the FP64 transform of the deepest vertex, FP32 rounding only
    pts = dict(vidx=out["vidx"].reshape(w.n_env, n_max), point=out["point"])
    for e in envs:
        full = pts["vidx"][e] >= 0
        if full.any():
            mesh = w.meshes[int(w.env_mesh[e])]
            xb = OQ.transform(w.pose[:, e], mesh.verts[pts["vidx"][e][full]])
            got = out["point"][:, e * n_max:(e + 1) * n_max][:, full].T
            assert np.max(np.abs(got - xb)) <= 1e-7
    return stats


@pytest.mark.parametrize("layout", ["brick", "linear"])
def test_nutbolt_patches_match_oracle(layout):
    torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(0, 1000, 60))
    b = fc.Batch.from_workload(w, layout=layout)
    c, out = run(b, fc.pose_tensor(w.pose), fc.PATCH_MAX, fc.PATCH_COS)
    st = check_patches(w, c, out, fc.PATCH_MAX, fc.PATCH_COS, range(w.n_env))
    print("nut-bolt patches:", layout, st, "per env", st["patches"] / w.n_env)
    assert st["patches"] > 10 * w.n_env


def test_torus_small_cap_replaces_patches():
    """N = 6 at 25 degrees: the list fills and AddPatch replaces or drops."""
    torch_gpu()
    w = W.subset(W.torus_workload(), range(48))
    b = fc.Batch.from_workload(w)
    cs = float(np.float32(np.cos(np.radians(25.0))))
    c, out = run(b, fc.pose_tensor(w.pose), 6, cs)
    st = check_patches(w, c, out, 6, cs, range(w.n_env))
    print("torus N=6:", st)
    assert st["dropped"] > 0


def test_extreme_thresholds_and_repeat_calls():
    """cos_sim = -1: one patch per env holding every candidate, its deepest
    member the deepest candidate (the maximum over the fixed-bin contacts);
    cos_sim = 2: every candidate founds its own patch until N is reached."""
    torch = torch_gpu()
    w = W.subset(W.torus_workload(), range(16))
    b = fc.Batch.from_workload(w)
    pose = fc.pose_tensor(w.pose)
    c, out = run(b, pose, 4, -1.0)
    check_patches(w, c, out, 4, -1.0, range(w.n_env))
    o = b.new_contacts()
    fc.fc_sdf_query(b, pose, fused_out=o)
    torch.cuda.synchronize()
    o = to_np(o)
    for e in range(w.n_env):
        s = slice(e * w.K, (e + 1) * w.K)
        if o["count"][e] == 0:
            assert out["count"][e] == 0
            continue
        dv = o["depth"][s]
        best = np.lexsort((o["vidx"][s], -dv.astype(np.float64)))[0]  # deepest, then lowest index
        assert out["count"][e] == 1 and out["vidx"][e * 4] == o["vidx"][s][best]
        assert out["depth"][e * 4] == dv[best]
    c2, out2 = run(b, pose, 64, 2.0)
    check_patches(w, c2, out2, 64, 2.0, range(w.n_env))
    _, out3 = run(b, pose, 64, 2.0)
    for k in out2:
        assert np.array_equal(out2[k], out3[k]), k


def test_mixed_sparse_and_half():
    torch_gpu()
    wm = W.subset(W.mixed_workload(), range(0, 4096, 97))
    c, out = run(fc.Batch.from_workload(wm), fc.pose_tensor(wm.pose), fc.PATCH_MAX, fc.PATCH_COS)
    check_patches(wm, c, out, fc.PATCH_MAX, fc.PATCH_COS, range(wm.n_env))
    w = W.subset(W.nut_bolt_workload(), range(0, 1000, 200))
    for layout, ww in (("sparse", w), ("brick", W.half_storage(w, "f16"))):
        c, out = run(fc.Batch.from_workload(ww, layout=layout), fc.pose_tensor(ww.pose), 128, fc.PATCH_COS)
        check_patches(ww, c, out, 128, fc.PATCH_COS, range(ww.n_env))


def test_patch_kernel_timing_id():
    torch_gpu()
    w = W.subset(W.torus_workload(), range(4))
    b = fc.Batch.from_workload(w)
    b.set_timing(2)
    run(b, fc.pose_tensor(w.pose), 8, fc.PATCH_COS)  # fc_sdf_query, then fc_contact_patches
    ms, kid = b.read_timing()
    b.set_timing(0)
    assert list(kid) == [fc.FC_KERNEL_FORWARD, fc.FC_KERNEL_PATCHES] and ms[1] > 0


def test_positive_margin_gives_negative_depths():
    """margin = 1 mm: candidates include points outside B (depth < 0), whose
    keys and AddPatch values are negative; the decisions still match the
    oracle bit for bit."""
    import dataclasses

    torch_gpu()
    w = dataclasses.replace(W.subset(W.torus_workload(), range(24)), margin=1e-3)
    b = fc.Batch.from_workload(w)
    c, out = run(b, fc.pose_tensor(w.pose), 12, float(np.float32(np.cos(np.radians(20.0)))))
    st = check_patches(w, c, out, 12, float(np.float32(np.cos(np.radians(20.0)))), range(w.n_env))
    assert (c["phi"][c["bin"] >= 0] > 0).sum() > 1000  # non-penetrating candidates took part
    assert st["dropped"] > 0
