"""The C ABI without a GPU: the library loads, exports every function
include/fc.h declares, and rejects invalid arguments before any HIP call."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

from paper_2205_03532_amd import fc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fc.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(fc.LIB_PATH):
        pytest.fail("libfactory_sdf.so not built (run __graft_entry__.build())")
    return fc.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s+(fc_[a-z_0-9]+)\s*\(", text, flags=re.M))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fc_sdf_query", "fc_contact_reduce", "fc_sdf_query_backward", "fc_sdf_query_and_backward",
                     "fc_graph_create",
                     "fc_workspace_bytes", "fc_autotune_load", "fc_status_str", "fc_last_hip_error"):
        assert required in names
    assert set(names) == set(fc.SIGNATURES), set(names) ^ set(fc.SIGNATURES)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name
    assert b"gfx950" in L.fc_version()


def test_status_strings(L):
    for s in range(9):
        assert L.fc_status_str(s) != b"unknown status"
    assert L.fc_status_str(0) == b"ok"


FAKE = 0x100000  # never dereferenced: validation only reads host arrays


def make_desc(n_env=2, K=16, dims=(4, 4, 4), h=0.1, dtype=0, n_verts=5, env_grid=None, mesh_null=False,
              second_grid_dtype=None, n_tris=0, tris_null=False):
    grids = (fc.fc_grid * 2)()
    grids[0] = fc.fc_grid(C.c_void_p(FAKE), dtype, 0, *dims, (C.c_float * 3)(0, 0, 0), h)
    grids[1] = fc.fc_grid(C.c_void_p(FAKE), dtype if second_grid_dtype is None else second_grid_dtype, 0, *dims,
                          (C.c_float * 3)(0, 0, 0), h)
    meshes = (fc.fc_mesh * 1)()
    p = None if mesh_null else C.c_void_p(FAKE)
    meshes[0] = fc.fc_mesh(p, p, p, n_verts, None if tris_null else C.c_void_p(FAKE), n_tris)
    eg = np.zeros(n_env, np.int32) if env_grid is None else np.asarray(env_grid, np.int32)
    em = np.zeros(n_env, np.int32)
    dirs = np.zeros((3, max(K, 1)), np.float32)
    dirs[2] = 1
    desc = fc.fc_batch_desc(n_env, grids, 2, meshes, 1, eg.ctypes.data_as(C.POINTER(C.c_int32)),
                            em.ctypes.data_as(C.POINTER(C.c_int32)), K, dirs.ctypes.data_as(C.POINTER(C.c_float)),
                            0.0)
    desc._keep = (grids, meshes, eg, em, dirs)
    return desc


@pytest.mark.parametrize("kw,status", [
    (dict(n_env=0), fc.FC_ERR_SHAPE),
    (dict(K=0), fc.FC_ERR_RANGE),
    (dict(K=65), fc.FC_ERR_RANGE),
    (dict(dims=(1, 4, 4)), fc.FC_ERR_SHAPE),
    (dict(dims=(2048, 2048, 1024)), fc.FC_ERR_SHAPE),
    (dict(h=0.0), fc.FC_ERR_RANGE),
    (dict(h=float("nan")), fc.FC_ERR_RANGE),
    (dict(dtype=7), fc.FC_ERR_DTYPE),
    (dict(second_grid_dtype=1), fc.FC_ERR_DTYPE),
    (dict(env_grid=[0, 2]), fc.FC_ERR_SHAPE),
    (dict(env_grid=[-1, 0]), fc.FC_ERR_SHAPE),
    (dict(n_verts=-1), fc.FC_ERR_SHAPE),
    (dict(mesh_null=True), fc.FC_ERR_NULL),
    (dict(n_tris=-1), fc.FC_ERR_SHAPE),
    (dict(n_tris=4, tris_null=True), fc.FC_ERR_NULL),
])
def test_batch_create_rejects(L, kw, status):
    desc = make_desc(**kw)
    h = C.c_void_p(12345)
    assert L.fc_batch_create(C.byref(desc), C.byref(h)) == status
    assert h.value is None  # nothing handed out


def test_null_arguments(L):
    h = C.c_void_p()
    assert L.fc_batch_create(None, C.byref(h)) == fc.FC_ERR_NULL
    assert L.fc_batch_create(C.byref(make_desc()), None) == fc.FC_ERR_NULL
    assert L.fc_sdf_query(None, None, None, None, None, 0, None) == fc.FC_ERR_NULL
    assert L.fc_sdf_query_noalloc(None, None, None, None, None) == fc.FC_ERR_NULL
    assert L.fc_sdf_query_noalloc_bytes(None) == 0
    assert L.fc_contact_reduce(None, None, None, None, None, 0, None) == fc.FC_ERR_NULL
    assert L.fc_sdf_query_backward(None, None, 1.0, None, None, None, 0, None) == fc.FC_ERR_NULL
    assert L.fc_sdf_query_and_backward(None, None, None, 1.0, None, None, None, 0, None) == fc.FC_ERR_NULL
    assert L.fc_graph_launch(None, None) == fc.FC_ERR_NULL
    assert L.fc_gather_probe(None, None, None, None) == fc.FC_ERR_NULL
    assert L.fc_sdf_query_faces(None, None, None, None, None, None, 0, None) == fc.FC_ERR_NULL
    assert L.fc_batch_face_queries(None) == -1
    assert L.fc_batch_set_timing(None, 4) == fc.FC_ERR_NULL
    assert L.fc_batch_read_timing(None, None, None, 0) == -1
    assert L.fc_batch_queries(None) == -1
    assert L.fc_workspace_bytes(None) == 0
    L.fc_batch_destroy(None)
    L.fc_graph_destroy(None)


def test_brick_size_query(L):
    g = fc.fc_grid(C.c_void_p(FAKE), 0, 0, 256, 256, 512, (C.c_float * 3)(0, 0, 0), 1e-4)
    bx, by, bz = -(-255 // 3), -(-255 // 3), -(-511 // 3)
    assert L.fc_grid_brick_bytes(C.byref(g), 1) == bx * by * bz * 64 * 4
    assert L.fc_grid_brick_bytes(C.byref(g), 2) == bx * by * 511 * 32 * 4  # slabs: 4x4x2 nodes, 3x3x1 cells
    assert L.fc_grid_brick_bytes(C.byref(g), 0) == 0
    g.dtype = 1
    assert L.fc_grid_brick_bytes(C.byref(g), 1) == bx * by * bz * 64 * 2
    g.nx = 1
    assert L.fc_grid_brick_bytes(C.byref(g), 1) == 0


def test_contact_patches_rejects_invalid_arguments(L):
    """Checked before anything touches the batch: no HIP call here."""
    fake = C.c_void_p(FAKE)
    ok = fc.fc_patch_params(128, 0.98)
    outs = fc.fc_patches(*([fake] * 7))
    call = L.fc_contact_patches
    assert call(None, fake, C.byref(ok), C.byref(outs), None) == fc.FC_ERR_NULL
    assert call(fake, None, C.byref(ok), C.byref(outs), None) == fc.FC_ERR_NULL
    assert call(fake, fake, None, C.byref(outs), None) == fc.FC_ERR_NULL
    assert call(fake, fake, C.byref(ok), None, None) == fc.FC_ERR_NULL
    for i in range(7):
        ptrs = [fake] * 7
        ptrs[i] = None
        assert call(fake, fake, C.byref(ok), C.byref(fc.fc_patches(*ptrs)), None) == fc.FC_ERR_NULL
    for n, cs in ((0, 0.9), (257, 0.9), (128, float("nan")), (128, float("inf"))):
        assert call(fake, fake, C.byref(fc.fc_patch_params(n, cs)), C.byref(outs), None) == fc.FC_ERR_RANGE


def test_sparse_conversion_rejects_invalid_arguments(L):
    """Every check happens before the classification kernel: no HIP call here."""
    g = fc.fc_grid(C.c_void_p(FAKE), 0, 0, 64, 64, 64, (C.c_float * 3)(0, 0, 0), 1e-3)
    nb = C.c_size_t()
    out = fc.fc_grid()
    assert L.fc_grid_sparse_bytes(None, 1e-3, C.byref(nb), None) == fc.FC_ERR_NULL
    assert L.fc_grid_sparse_bytes(C.byref(g), 1e-3, None, None) == fc.FC_ERR_NULL
    assert L.fc_grid_sparse_bytes(C.byref(g), -1e-3, C.byref(nb), None) == fc.FC_ERR_RANGE
    assert L.fc_grid_sparse_bytes(C.byref(g), float("nan"), C.byref(nb), None) == fc.FC_ERR_RANGE
    assert L.fc_grid_to_sparse(C.byref(g), 1e-3, None, 1 << 20, C.byref(out), None) == fc.FC_ERR_NULL
    assert L.fc_grid_to_sparse(C.byref(g), 1e-3, C.c_void_p(FAKE), 1 << 20, None, None) == fc.FC_ERR_NULL
    assert L.fc_grid_to_sparse(C.byref(g), 1e-3, C.c_void_p(FAKE + 16), 1 << 20, C.byref(out), None) == fc.FC_ERR_RANGE
    g.layout = 1  # only a linear grid converts
    assert L.fc_grid_sparse_bytes(C.byref(g), 1e-3, C.byref(nb), None) == fc.FC_ERR_DTYPE
    g.layout, g.nx = 0, 1
    assert L.fc_grid_sparse_bytes(C.byref(g), 1e-3, C.byref(nb), None) == fc.FC_ERR_SHAPE
    g.nx, g.h = 64, 0.0
    assert L.fc_grid_sparse_bytes(C.byref(g), 1e-3, C.byref(nb), None) == fc.FC_ERR_RANGE


def test_autotune_cache_parse(L, tmp_path):
    p = tmp_path / "tune.json"
    p.write_text(json.dumps({"entries": [
        {"key": "a", "block": 256, "tile": 1024, "persistent": 0, "grid_mult": 8},
        {"key": "b", "block": 128, "tile": 512, "persistent": 2, "grid_mult": 4},
        {"key": "c", "block": 256, "tile": 1024, "persistent": 3, "grid_mult": 8, "xcd_remap": 1},
        {"key": "d", "block": 256, "tile": 1024, "persistent": 0, "grid_mult": 8, "wave_prio": 0},
        {"key": "e", "block": 256, "tile": 1024, "persistent": 0, "grid_mult": 8, "wave_prio": 2,
         "step_ms": {"1": 0.14, "0": 0.15, "2": 0.13}},
        {"key": "bad", "block": 100, "tile": 1024, "persistent": 0, "grid_mult": 8},
        {"key": "bad2", "block": 256, "tile": 1024, "persistent": 4, "grid_mult": 8},
        {"key": "bad3", "block": 256, "tile": 1024, "persistent": 0, "grid_mult": 8, "wave_prio": 3},
        {"key": "bad4", "block": 256, "tile": 1024, "persistent": 0, "grid_mult": 8, "wave_prio": -1},
    ]}))
    assert L.fc_autotune_load(str(p).encode()) == 5
    p.write_text("{not json")
    assert L.fc_autotune_load(str(p).encode()) == -1
    assert L.fc_autotune_load(b"/nonexistent/file.json") == -1


def test_env_order_must_be_a_permutation(L):
    desc = make_desc(n_env=3)
    for bad in ([0, 0, 2], [0, 1, 3], [-1, 0, 1]):
        eo = np.asarray(bad, np.int32)
        desc.env_order = eo.ctypes.data_as(C.POINTER(C.c_int32))
        h = C.c_void_p()
        assert L.fc_batch_create(C.byref(desc), C.byref(h)) == fc.FC_ERR_SHAPE
