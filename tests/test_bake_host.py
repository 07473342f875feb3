"""The host half of the mesh-to-SDF bake without a GPU: fc_bake_table's
pseudonormals and corner records equal the FP64 oracle's (rounded to FP32),
its mesh checks reject open, inconsistently or inward-wound and degenerate
meshes, and fc_bake_sdf rejects invalid arguments before any HIP call."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import bake as OB
from paper_2205_03532_amd import fc
from paper_2205_03532_amd import workloads as W
from test_oracle_bake import dented_cube

FAKE = 0x100000  # never dereferenced: fc_bake_sdf validates before launching


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(fc.LIB_PATH):
        pytest.fail("libfactory_sdf.so not built (run __graft_entry__.build())")
    return fc.lib()


def meshes():
    ico = W.icosphere(2, 0.01)
    bv, bt = W.bolt_mesh(0.7e-3, 2e-3, 3e-3, 24, 12)
    return {"cube": W.cube_mesh(0.5), "tetrahedron": W.tetrahedron_mesh(0.5), "dented_cube": dented_cube(),
            "icosphere": (ico.verts, ico.tris), "bolt": (bv, bt)}


@pytest.mark.parametrize("name", ["cube", "tetrahedron", "dented_cube", "icosphere", "bolt"])
def test_table_matches_oracle(L, name):
    v, t = meshes()[name]
    v32 = np.asarray(v, dtype=np.float32)
    tab = fc.fc_bake_table(v32, t)
    m = len(t)
    nc = (m + 31) // 32
    assert tab.shape == (10 * m + 2 * nc, 4)
    pos = tab[:3 * m].reshape(m, 3, 4)
    nrm = tab[3 * m:10 * m].reshape(m, 7, 4)
    box = tab[10 * m:].reshape(nc, 2, 4)
    perm = pos[:, 0, 3].view(np.int32)
    assert np.array_equal(np.sort(perm), np.arange(m))  # every triangle once
    V = v32.astype(np.float64)
    T = np.asarray(t, dtype=np.int64)[perm]
    a = V[T[:, 0]]
    ref_pos = np.stack([a, V[T[:, 1]] - a, V[T[:, 2]] - a], axis=1)
    assert np.array_equal(pos[..., :3], ref_pos.astype(np.float32))
    N = OB.feature_normals(V, np.asarray(t, dtype=np.int64))[perm]
    # the library sums in its own order: FP64 rounding apart, then rounded to FP32
    scale = np.maximum(np.abs(N), 1.0)
    assert np.max(np.abs(nrm[..., :3] - N) / scale) < 2e-7
    assert np.all(pos[:, 1:, 3] == 0) and np.all(nrm[..., 3] == 0)
    # each run of 32 triangles lies in its box, and the box is the tightest one
    corners = v32[np.asarray(t)[perm]]  # (m, 3, 3)
    for c in range(nc):
        pts = corners[32 * c:32 * (c + 1)].reshape(-1, 3)
        assert np.array_equal(box[c, 0, :3], pts.min(0)) and np.array_equal(box[c, 1, :3], pts.max(0))
    assert box[0, 0, 3] == np.float32(np.max(np.abs(V)))
    # the order follows space: consecutive triangles are near each other
    cen = corners.mean(1)
    step = np.linalg.norm(np.diff(cen, axis=0), axis=1).mean() if m > 1 else 0.0
    ext = np.linalg.norm(v32.max(0) - v32.min(0))
    if m >= 300:
        assert step < 0.1 * ext, (step, ext)


def test_bolt_mesh_is_closed_and_outward():
    v, t = W.bolt_mesh(0.7e-3, 2e-3, 12e-3, 128, 184)
    assert len(t) == 2 * 128 * 183 + 2 * 128 == 47104
    d = {}
    for f, (i, j, k) in enumerate(t):
        for p, q in ((i, j), (j, k), (k, i)):
            assert (p, q) not in d
            d[(p, q)] = f
    assert all((q, p) in d for (p, q) in d)
    V = v.astype(np.float64)
    vol = np.sum(np.einsum("ij,ij->i", V[t[:, 0]], np.cross(V[t[:, 1]], V[t[:, 2]]))) / 6
    core, outer = np.pi * (2e-3 - 5 / 8 * np.sqrt(3) / 2 * 0.7e-3) ** 2 * 12e-3, np.pi * 2e-3 ** 2 * 12e-3
    assert core < vol < outer


def _status(L, v, t, nb=None, table=None):
    v = np.ascontiguousarray(v, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    buf = np.zeros((10 * max(len(t), 1) + 2 * (len(t) // 32 + 1), 4), dtype=np.float32) if table is None else table
    nb = buf.nbytes if nb is None else nb
    return L.fc_bake_table(v.ctypes.data_as(C.c_void_p), len(v), t.ctypes.data_as(C.c_void_p), len(t),
                           buf.ctypes.data_as(C.c_void_p), nb)


def test_table_rejects_bad_meshes(L):
    v, t = W.cube_mesh(0.5)
    t = np.asarray(t)
    assert _status(L, v, t) == fc.FC_OK
    assert _status(L, v, t[:-1]) == fc.FC_ERR_SHAPE  # open: one face missing
    flip = t.copy()
    flip[0] = flip[0][::-1]
    assert _status(L, v, flip) == fc.FC_ERR_SHAPE  # one face wound against its neighbours
    assert _status(L, v, t[:, ::-1]) == fc.FC_ERR_RANGE  # all wound inward
    bad = t.copy()
    bad[3, 1] = 8
    assert _status(L, v, bad) == fc.FC_ERR_SHAPE  # index out of range
    bad = t.copy()
    bad[3, 1] = bad[3, 0]
    assert _status(L, v, bad) == fc.FC_ERR_SHAPE  # repeated index
    dup = np.vstack([t, t[:1]])
    assert _status(L, v, dup) == fc.FC_ERR_SHAPE  # a directed edge twice
    vn = np.array(v, dtype=np.float32)
    vn[2, 0] = np.nan
    assert _status(L, vn, t) == fc.FC_ERR_RANGE
    flat = np.array(v, dtype=np.float32)
    flat[:, 2] = 0.0  # every face of the cube collapses onto z = 0: zero areas
    assert _status(L, flat, t) == fc.FC_ERR_RANGE
    assert _status(L, v, t[:3]) == fc.FC_ERR_SHAPE  # fewer than 4 faces
    assert _status(L, v, t, nb=L.fc_bake_table_bytes(len(t)) - 1) == fc.FC_ERR_WORKSPACE
    assert L.fc_bake_table(None, 8, None, 12, None, 0) == fc.FC_ERR_NULL
    assert L.fc_bake_table_bytes(3) == 0 and L.fc_bake_table_bytes(12) == 12 * 160 + 32
    assert L.fc_bake_table_bytes(33) == 33 * 160 + 2 * 32
    assert L.fc_bake_table_bytes((1 << 24) + 1) == 0


def test_bake_sdf_rejects_invalid_arguments(L):
    o = (C.c_float * 3)(0.0, 0.0, 0.0)
    fake = C.c_void_p(FAKE)
    call = L.fc_bake_sdf
    assert call(None, 12, 4, 4, 4, o, 0.1, fake, None) == fc.FC_ERR_NULL
    assert call(fake, 12, 4, 4, 4, None, 0.1, fake, None) == fc.FC_ERR_NULL
    assert call(fake, 12, 4, 4, 4, o, 0.1, None, None) == fc.FC_ERR_NULL
    assert call(fake, 3, 4, 4, 4, o, 0.1, fake, None) == fc.FC_ERR_SHAPE
    assert call(fake, 12, 0, 4, 4, o, 0.1, fake, None) == fc.FC_ERR_SHAPE
    assert call(fake, 12, 2048, 2048, 512, o, 0.1, fake, None) == fc.FC_ERR_SHAPE  # 2^31 nodes
    assert call(fake, 12, 4, 4, 4, o, 0.0, fake, None) == fc.FC_ERR_RANGE
    assert call(fake, 12, 4, 4, 4, o, float("inf"), fake, None) == fc.FC_ERR_RANGE
    onan = (C.c_float * 3)(0.0, float("nan"), 0.0)
    assert call(fake, 12, 4, 4, 4, onan, 0.1, fake, None) == fc.FC_ERR_RANGE
    assert call(C.c_void_p(FAKE + 4), 12, 4, 4, 4, o, 0.1, fake, None) == fc.FC_ERR_RANGE  # misaligned table
