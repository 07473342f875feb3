"""GPU parity of the narrow-band sparse grid (FC_LAYOUT_SPARSE) through the
C ABI.

A query whose cell lies in a stored brick must give the brick layout's
results bit for bit (same corner values, same arithmetic).  A query in a
brick that is not stored takes the coarse interpolant of the brick's corner
nodes: its phi is compared with the FP64 oracle (oracle/sparse.py) within
the FP32 tolerance of the dense path, its normal within NORMAL_TOL_COARSE.
Queries within the FP32 position error of a brick face may fall on either
side and are left out of those two comparisons."""
import numpy as np
import pytest

from _gpu_common import (DEPTH_TOL_F32, FACE_BAND, assert_same, check_bins_exact, check_reduction_exact,
                         gradient_sensitivity, oracle_rows, position_error_voxels, rows_of, to_np, torch_gpu)
from oracle import query as OQ
from oracle import sparse as OS
from paper_2205_03532_amd import fc
from paper_2205_03532_amd import workloads as W

pytestmark = pytest.mark.gpu
NORMAL_TOL_COARSE = 1e-5  # chord: the coarse interpolant's normal, FP32 expansion and position rounding


def run(batch, pose):
    torch = torch_gpu()
    c, o = batch.new_candidates(), batch.new_contacts()
    fc.fc_sdf_query(batch, pose, cand=c)
    fc.fc_sdf_query(batch, pose, fused_out=o)
    torch.cuda.synchronize()
    return to_np(c), to_np(o)


def run_one_pass(batch, pose, k=1e4):
    torch = torch_gpu()
    o, g = batch.new_contacts(), batch.new_grads(per_env=False)
    fc.fc_sdf_query_and_backward(batch, pose, o, k, g)
    torch.cuda.synchronize()
    return to_np(o), to_np(g)


def sparse_oracle(w, envs, band):
    """Oracle rows with phi, grad, normal, bin replaced by the sparse field's,
    plus the stored flag and a flag for rows near a brick face."""
    o = oracle_rows(w, envs)
    stored = np.zeros(len(o["phi"]), bool)
    for e in envs:
        sel = o["env"] == e
        g = w.grids[int(w.env_grid[e])]
        vals = OQ.grid_values_f64(g.values, g.dtype)
        phi, grad, ins, st = OS.sample_sparse(vals, g.origin, g.h, g.dims, o["x_b"][sel], band)
        o["phi"][sel], o["grad"][sel], stored[sel] = phi, grad, st
    o["normal"], o["bin"], o["dots"] = OQ.normals_and_bins(o["grad"], w.bins)
    du = np.max(position_error_voxels(o), axis=1)
    bandv = np.maximum(FACE_BAND, 2.0 * du)[:, None]
    r = o["u"] - 3.0 * np.floor(o["u"] / 3.0)  # position inside the brick, in cells
    near_brick_face = np.any((r < bandv) | (r > 3.0 - bandv), axis=1)
    o["stored"], o["near_brick_face"] = stored, near_brick_face
    return o


def test_nutbolt_sparse_equals_brick():
    """Nut vertices near the bolt lie in stored bricks (4-voxel band); the
    others (the hex corners) lie in exterior bricks whose nodes all exceed the
    band.  So per-query candidates equal the brick layout's in stored bricks,
    the rest are never candidates in either layout, and the reduced contacts
    and the one-pass adjoint equal the brick layout's bit for bit, at a
    fraction of the memory."""
    torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(0, 1000, 10))
    envs = list(range(w.n_env))
    band = float(np.float32(4 * w.grids[0].h))
    g = w.grids[0]
    vals = OQ.grid_values_f64(g.values, g.dtype)
    o = sparse_oracle(w, envs, band)
    ins = o["inside"]
    assert np.all(o["phi"][ins & ~o["stored"]] > band)  # unstored: exterior only
    assert (ins & o["stored"]).sum() > 0.99 * ins.sum()
    b_sp = fc.Batch.from_workload(w, layout="sparse", band=band)
    b_br = fc.Batch.from_workload(w, layout="brick")
    pose = fc.pose_tensor(w.pose)
    c1, o1 = run(b_sp, pose)
    c2, o2 = run(b_br, pose)
    rows = rows_of(w, envs)
    st = ins & o["stored"] & ~o["near_brick_face"]
    for k in ("phi", "bin"):
        assert np.array_equal(c1[k][rows][st].view(np.uint8), c2[k][rows][st].view(np.uint8)), k
    assert np.array_equal(c1["normal"][:, rows][:, st].view(np.uint32), c2["normal"][:, rows][:, st].view(np.uint32))
    ex = ins & ~o["stored"]
    assert np.all(c1["bin"][rows][ex] == -1) and np.all(c1["phi"][rows][ex] > band)
    assert_same(o1, o2)
    p1, g1 = run_one_pass(b_sp, pose)
    p2, g2 = run_one_pass(b_br, pose)
    assert_same(p1, p2)
    assert_same(g1, g2)
    # the library's classification: its buffer size is the oracle's count of stored bricks
    bx, by, bz = OS.brick_counts(g.dims)
    n_stored = 0
    for k in range(bz):
        j, i = np.meshgrid(np.arange(by), np.arange(bx), indexing="ij")
        n_stored += int(OS.brick_stored(vals, band, np.stack([i.ravel(), j.ravel(), np.full(i.size, k)], -1)).sum())
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    assert b_sp.sparse_bytes == al(bx * by * bz * 4) + al((bx + 1) * (by + 1) * (bz + 1) * 4) + n_stored * 64 * 4
    brick_bytes = b_br.grid_tensors[0].numel()
    print(f"nut-bolt sparse: {b_sp.sparse_bytes / 2**20:.1f} MiB vs brick {brick_bytes / 2**20:.1f} MiB, "
          f"linear {g.values.nbytes / 2**20:.1f} MiB")
    assert b_sp.sparse_bytes < brick_bytes / 4


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_half_sparse_equals_brick(dtype):
    torch_gpu()
    w = W.half_storage(W.subset(W.nut_bolt_workload(), range(0, 1000, 40)), dtype)
    band = float(np.float32(4 * w.grids[0].h))
    pose = fc.pose_tensor(w.pose)
    c1, o1 = run(fc.Batch.from_workload(w, layout="sparse", band=band), pose)
    c2, o2 = run(fc.Batch.from_workload(w, layout="brick"), pose)
    assert_same(o1, o2)
    # |phi| <= band needs a corner within the band or corners of both signs: a stored brick
    near = np.abs(c2["phi"]) < band * (1 - 1e-6)
    assert near.sum() > 0.9 * np.isfinite(c2["phi"]).sum()
    assert np.array_equal(c1["phi"][near].view(np.uint32), c2["phi"][near].view(np.uint32))
    assert np.array_equal(c1["bin"], c2["bin"])


def test_torus_sparse_matches_oracle():
    """Icosphere vertices spread through the torus grid: with a 1.5-voxel band
    many queries fall in bricks that are not stored (coarse interpolant)."""
    torch_gpu()
    w = W.subset(W.torus_workload(), range(64))
    envs = list(range(w.n_env))
    band = float(np.float32(1.5 * w.grids[0].h))
    pose = fc.pose_tensor(w.pose)
    b_sp = fc.Batch.from_workload(w, layout="sparse", band=band)
    c_sp, o_sp = run(b_sp, pose)
    c_br, _ = run(fc.Batch.from_workload(w, layout="brick"), pose)
    o = sparse_oracle(w, envs, band)
    rows = rows_of(w, envs)
    ins = o["inside"] & np.isfinite(c_sp["phi"][rows])
    clear = ins & ~o["near_brick_face"]
    st, co = clear & o["stored"], clear & ~o["stored"]
    assert st.sum() > 10000 and co.sum() > 10000, (st.sum(), co.sum())
    # stored bricks: the brick layout's bits
    for k in ("phi", "bin"):
        assert np.array_equal(c_sp[k][rows][st].view(np.uint8), c_br[k][rows][st].view(np.uint8)), k
    assert np.array_equal(c_sp["normal"][:, rows][:, st].view(np.uint32), c_br["normal"][:, rows][:, st].view(np.uint32))
    # coarse bricks: the oracle's coarse interpolant
    phi = c_sp["phi"][rows].astype(np.float64)
    err = np.abs(phi[co] - o["phi"][co])
    assert err.max() <= DEPTH_TOL_F32, err.max()
    nrm = c_sp["normal"][:, rows].T.astype(np.float64)
    gl = np.linalg.norm(o["grad"], axis=1)
    ok = co & (gl > 0.1)
    nerr = np.linalg.norm(nrm[ok] - o["normal"][ok], axis=1)
    assert nerr.max() <= NORMAL_TOL_COARSE, nerr.max()
    # candidates, bins and the reduction, whatever the path
    m = np.float64(np.float32(w.margin))
    amb = np.abs(o["phi"] - m) <= DEPTH_TOL_F32
    g_cand = c_sp["bin"][rows] >= 0
    o_cand = ins & (o["phi"] < m)
    assert not ((g_cand != o_cand) & clear & ~amb).any()
    check_bins_exact(w, c_sp, envs)
    check_reduction_exact(w, c_sp, o_sp, envs)
    print(f"torus sparse: stored {st.sum()}, coarse {co.sum()}, max coarse depth err {err.max():.2e}, "
          f"max coarse normal err {nerr.max():.2e}, bytes {b_sp.sparse_bytes}")


def test_infinite_band_equals_brick_everywhere():
    torch_gpu()
    w = W.subset(W.torus_workload(), range(32))
    pose = fc.pose_tensor(w.pose)
    c1, o1 = run(fc.Batch.from_workload(w, layout="sparse", band=float("inf")), pose)
    c2, o2 = run(fc.Batch.from_workload(w, layout="brick"), pose)
    assert_same(c1, c2)
    assert_same(o1, o2)


def test_faces_on_sparse_equal_brick():
    torch = torch_gpu()
    w = W.subset(W.nut_bolt_workload(), range(0, 1000, 125))
    band = float(np.float32(4 * w.grids[0].h))
    pose = fc.pose_tensor(w.pose)
    outs = []
    for b in (fc.Batch.from_workload(w, layout="sparse", band=band), fc.Batch.from_workload(w, layout="brick")):
        c, o = b.new_face_candidates(), b.new_contacts()
        fc.fc_sdf_query_faces(b, pose, cand=c, fused_out=o)
        torch.cuda.synchronize()
        outs.append((to_np(c), to_np(o)))
    assert_same(outs[0][0], outs[1][0])
    assert_same(outs[0][1], outs[1][1])


def test_sparse_graph_replay_and_autograd():
    """The sparse layout under hipGraph replay (with eager work between
    replays) and behind the autograd function: the same bits as eager calls
    on the same batch, and the autograd gradients equal the brick layout's."""
    torch = torch_gpu()
    from paper_2205_03532_amd.autograd import penalty

    w = W.subset(W.nut_bolt_workload(), range(0, 1000, 25))
    band = float(np.float32(4 * w.grids[0].h))
    b = fc.Batch.from_workload(w, layout="sparse", band=band)
    pose = fc.pose_tensor(w.pose)
    ref_o, ref_g = run_one_pass(b, pose)
    out, gr = b.new_contacts(), b.new_grads(per_env=False)
    graph = fc.fc_graph_create(b, pose, fused_out=out, k=1e4, grads=gr)
    for _ in range(3):
        for t in list(out.values()) + [v for k, v in gr.items() if k != "per_env"]:
            t.fill_(7)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert_same(to_np(out), ref_o)
        assert_same(to_np({k: v for k, v in gr.items() if k != "per_env"}),
                    {k: v for k, v in ref_g.items() if k != "per_env"})
    del graph
    grads = []
    for bb in (b, fc.Batch.from_workload(w, layout="brick")):
        for mt in bb.mesh_tensors:
            mt.requires_grad_(True)
        loss, xi = penalty(bb, pose, 1e4)
        loss.sum().backward()
        grads.append((loss.detach().cpu().numpy(), xi.grad.cpu().numpy(), bb.mesh_tensors[0].grad.cpu().numpy()))
        for mt in bb.mesh_tensors:
            mt.requires_grad_(False)
            mt.grad = None
    for a_, b_ in zip(grads[0], grads[1]):
        assert np.array_equal(a_.view(np.uint32), b_.view(np.uint32))


def _sparse_cell_data(w, o, band):
    """Per row, S (largest mixed second difference) and cmax (scale of the
    FP32 rounding) of the corners the kernel interpolates: a stored brick's
    dense cell corners; in a brick that is not stored, S of the coarse
    interpolant at the fine cell's 8 corners and cmax of the brick's 8
    corner nodes, from which the kernel expands those corners in FP32."""
    import itertools

    S, cmax = gradient_sensitivity(w, o)
    g = w.grids[0]
    vals = OQ.grid_values_f64(g.values, g.dtype)
    idx = np.nonzero(o["inside"] & ~o["stored"])[0]
    cell = o["cell"][idx]
    C = {}
    for a, b, c in itertools.product((0, 1), repeat=3):
        t = np.tile(np.array([a, b, c], np.float64), (len(idx), 1))
        C[a, b, c], _ = OS.coarse_interpolant(vals, cell, t, g.h)
    m = np.zeros(len(idx))
    for k in (0, 1):
        m = np.maximum(m, np.abs(C[1, 1, k] - C[1, 0, k] - C[0, 1, k] + C[0, 0, k]))
        m = np.maximum(m, np.abs(C[1, k, 1] - C[1, k, 0] - C[0, k, 1] + C[0, k, 0]))
        m = np.maximum(m, np.abs(C[k, 1, 1] - C[k, 1, 0] - C[k, 0, 1] + C[k, 0, 0]))
    b0 = 3 * (cell // 3)
    cm = np.zeros(len(idx))
    for a, b, c in itertools.product((0, 3), repeat=3):
        cm = np.maximum(cm, np.abs(vals[b0[:, 2] + c, b0[:, 1] + b, b0[:, 0] + a]))
    S[idx], cmax[idx] = m, cm
    return S, cmax


def test_sparse_coarse_adjoint_matches_oracle_and_fd():
    """A small icosphere inside the torus's tube with a 1.5-voxel band: its
    vertices penetrate 1-3 mm, many in bricks that are not stored, so loss,
    twist and vertex gradients come partly from the coarse interpolant.
    Per-env mode against the FP64 oracle on the sparse field, the shared mode
    against the oracle's sum, and FP64 central differences of that field
    (which jumps in value across faces between stored and unstored bricks)."""
    from _adjoint_common import KP, adjoint_bounds, check_fd, check_vs_oracle, run_backward, shared_blocks
    from oracle import adjoint as OA

    torch_gpu()
    w = W.torus_tube_workload()
    g, verts = w.grids[0], w.meshes[0].verts
    envs = list(range(w.n_env))
    band = float(np.float32(1.5 * g.h))
    b = fc.Batch.from_workload(w, layout="sparse", band=band)
    pose = fc.pose_tensor(w.pose)
    res = run_backward(b, pose, per_env=True)
    o = sparse_oracle(w, envs, band)
    pen = o["inside"] & (o["phi"] < 0)
    n_coarse, n_stored = int((pen & ~o["stored"]).sum()), int((pen & o["stored"]).sum())
    assert n_coarse > 1000 and n_stored > 1000, (n_coarse, n_stored)
    S, cmax = _sparse_cell_data(w, o, band)
    vals = OQ.grid_values_f64(g.values, g.dtype)
    smp = OS.sparse_sampler(vals, g.origin, g.h, g.dims, band)
    # rows near a cell face (brick faces among them, where the field jumps
    # between a stored brick and one that is not) are allowed either side
    bounds = adjoint_bounds(w, envs, KP, o=o, S=S, cmax=cmax, extra_ulps=40.0, sampler_of=lambda e: smp)
    shared, tol, worst = check_vs_oracle(w, res, envs, True, bounds=bounds,
                                         penalty=lambda e: OA.penalty_env(g, verts, w.pose[:, e], KP, sampler=smp))
    res_sh = run_backward(b, pose, per_env=False)
    gv = shared_blocks(w, res_sh["d_verts"])[0]
    assert np.all(np.abs(gv - shared[0]) <= tol[0][:, None] + 1e-6 * np.abs(shared[0]) + 1e-9)
    n_smooth, n_kinked = check_fd(w, res, envs, bounds=bounds, sampler_of=lambda e: smp, jumps=True)
    print(f"sparse adjoint: {n_coarse} penetrating vertices in coarse bricks, {n_stored} in stored; "
          f"worst twist |err|/bound {worst:.3f}; FD {n_smooth} smooth, {n_kinked} kinked components")
    assert n_smooth > 0
