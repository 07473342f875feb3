"""ctypes binding of libfactory_sdf.so (include/fc.h).

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch supplies device memory (tensors) and the current stream.  The module
fails loudly when the library is not built; there is no CPU fallback.

Names follow the C ABI: ``fc_sdf_query``, ``fc_contact_reduce``,
``fc_sdf_query_backward``, ``fc_sdf_query_and_backward`` (both in one pass),
``fc_graph_create`` / ``fc_graph_launch``,
``fc_grid_to_bricks``, ``fc_bake_table`` / ``fc_bake_sdf``, ``fc_autotune_load``.  ``Batch`` owns the device copies
of a workload's grids and meshes and the opaque ``fc_batch`` handle.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

(FC_KERNEL_FORWARD, FC_KERNEL_BACKWARD, FC_KERNEL_QUERY_BACKWARD, FC_KERNEL_GATHER_PROBE, FC_KERNEL_FACES,
 FC_KERNEL_PATCHES) = range(6)

# the in-tree build; FC_LIB_PATH selects another build of the same sources
LIB_PATH = os.environ.get("FC_LIB_PATH") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                         "libfactory_sdf.so")

(FC_OK, FC_ERR_NULL, FC_ERR_SHAPE, FC_ERR_DTYPE, FC_ERR_RANGE, FC_ERR_WORKSPACE, FC_ERR_HIP, FC_ERR_UNSUPPORTED,
 FC_ERR_SCRATCH) = range(9)
NOALLOC_SCRATCH_BYTES = 4 << 20  # the static scratch of fc_sdf_query_noalloc, per device
DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
LAYOUTS = {"linear": 0, "brick": 1, "slab": 2, "sparse": 3}
SPARSE_BAND_VOXELS = 4.0  # default narrow band of the sparse layout, in voxels
MAX_TYPES = 8
MAX_BINS = 64


class fc_grid(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("layout", C.c_int32), ("nx", C.c_int32),
                ("ny", C.c_int32), ("nz", C.c_int32), ("origin", C.c_float * 3), ("h", C.c_float)]


class fc_mesh(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("n_verts", C.c_int32),
                ("tris", C.c_void_p), ("n_tris", C.c_int32)]


class fc_batch_desc(C.Structure):
    _fields_ = [("n_env", C.c_int32), ("grids", C.POINTER(fc_grid)), ("n_grids", C.c_int32),
                ("meshes", C.POINTER(fc_mesh)), ("n_meshes", C.c_int32), ("env_grid", C.POINTER(C.c_int32)),
                ("env_mesh", C.POINTER(C.c_int32)), ("n_bins", C.c_int32), ("bin_dirs", C.POINTER(C.c_float)),
                ("margin", C.c_float), ("env_order", C.POINTER(C.c_int32))]


class fc_candidates(C.Structure):
    _fields_ = [("phi", C.c_void_p), ("normal", C.c_void_p), ("bin", C.c_void_p), ("point", C.c_void_p)]


class fc_pgd(C.Structure):
    _fields_ = [("iters", C.c_int32), ("step0", C.c_float)]


class fc_patch_params(C.Structure):
    _fields_ = [("max_patches", C.c_int32), ("cos_sim", C.c_float)]


class fc_patches(C.Structure):
    _fields_ = [("count", C.c_void_p), ("founder", C.c_void_p), ("normal", C.c_void_p), ("vidx", C.c_void_p),
                ("depth", C.c_void_p), ("point", C.c_void_p), ("members", C.c_void_p)]


PATCH_MAX = 128  # N (the paper: 128 <= N <= 256)
PATCH_COS = float(np.float32(np.cos(np.radians(10.0))))  # similar normals: within 10 degrees


class fc_contacts(C.Structure):
    _fields_ = [("vidx", C.c_void_p), ("depth", C.c_void_p), ("point", C.c_void_p), ("normal", C.c_void_p),
                ("count", C.c_void_p)]


class fc_grads(C.Structure):
    _fields_ = [("loss", C.c_void_p), ("d_pose", C.c_void_p), ("d_verts", C.c_void_p),
                ("verts_per_env", C.c_int32)]


class fc_launch(C.Structure):
    _fields_ = [("block", C.c_int32), ("tile", C.c_int32), ("persistent", C.c_int32), ("grid_mult", C.c_int32),
                ("xcd_remap", C.c_int32), ("wave_prio", C.c_int32)]


# every symbol include/fc.h declares, with its ctypes signature
SIGNATURES = {
    "fc_batch_create": (C.c_int, [C.POINTER(fc_batch_desc), C.POINTER(C.c_void_p)]),
    "fc_batch_destroy": (None, [C.c_void_p]),
    "fc_batch_queries": (C.c_int64, [C.c_void_p]),
    "fc_batch_set_launch": (C.c_int, [C.c_void_p, C.POINTER(fc_launch)]),
    "fc_batch_get_launch": (C.c_int, [C.c_void_p, C.POINTER(fc_launch)]),
    "fc_workspace_bytes": (C.c_size_t, [C.c_void_p]),
    "fc_workspace_init": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "fc_sdf_query": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(fc_candidates), C.POINTER(fc_contacts),
                               C.c_void_p, C.c_size_t, C.c_void_p]),
    "fc_sdf_query_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(fc_candidates), C.POINTER(fc_contacts),
                                       C.c_void_p]),
    "fc_sdf_query_noalloc_bytes": (C.c_size_t, [C.c_void_p]),
    "fc_contact_reduce": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(fc_candidates), C.POINTER(fc_contacts),
                                    C.c_void_p, C.c_size_t, C.c_void_p]),
    "fc_sdf_query_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_float, C.c_void_p, C.POINTER(fc_grads),
                                        C.c_void_p, C.c_size_t, C.c_void_p]),
    "fc_sdf_query_and_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(fc_contacts), C.c_float, C.c_void_p,
                                            C.POINTER(fc_grads), C.c_void_p, C.c_size_t, C.c_void_p]),
    "fc_graph_create": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(fc_contacts), C.c_float, C.c_void_p,
                                  C.POINTER(fc_grads), C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]),
    "fc_graph_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fc_graph_destroy": (None, [C.c_void_p]),
    "fc_grid_brick_bytes": (C.c_size_t, [C.POINTER(fc_grid), C.c_int32]),
    "fc_grid_to_bricks": (C.c_int, [C.POINTER(fc_grid), C.c_int32, C.c_void_p, C.c_size_t, C.POINTER(fc_grid),
                                    C.c_void_p]),
    "fc_autotune_load": (C.c_int32, [C.c_char_p]),
    "fc_batch_signature": (C.c_int32, [C.c_void_p, C.c_char_p, C.c_int32]),
    "fc_batch_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "fc_batch_read_timing": (C.c_int32, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_int32), C.c_int32]),
    "fc_gather_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fc_sdf_query_faces": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(fc_pgd), C.POINTER(fc_candidates),
                                     C.POINTER(fc_contacts), C.c_void_p, C.c_size_t, C.c_void_p]),
    "fc_batch_face_queries": (C.c_int64, [C.c_void_p]),
    "fc_contact_patches": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(fc_patch_params), C.POINTER(fc_patches),
                                     C.c_void_p]),
    "fc_grid_sparse_bytes": (C.c_int, [C.POINTER(fc_grid), C.c_float, C.POINTER(C.c_size_t), C.c_void_p]),
    "fc_grid_to_sparse": (C.c_int, [C.POINTER(fc_grid), C.c_float, C.c_void_p, C.c_size_t, C.POINTER(fc_grid),
                                    C.c_void_p]),
    "fc_bake_table_bytes": (C.c_size_t, [C.c_int32]),
    "fc_bake_table": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]),
    "fc_bake_sdf": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_float),
                              C.c_float, C.c_void_p, C.c_void_p]),
    "fc_bake_sdf_unculled": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_float),
                                       C.c_float, C.c_void_p, C.c_void_p]),
    "fc_status_str": (C.c_char_p, [C.c_int]),
    "fc_last_hip_error": (C.c_int32, []),
    "fc_version": (C.c_char_p, []),
}

_LIB = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2205_03532_amd.build` "
                               "(or __graft_entry__.build()); there is no CPU fallback")
        # torch first: its HIP runtime is then already in the process and the
        # library binds to that one, so streams and device pointers pass
        # between the two (loaded the other way round, the library's first HIP
        # call has failed with hipErrorNoDevice)
        import torch  # noqa: F401

        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


class FcError(RuntimeError):
    def __init__(self, status, what):
        L = lib()
        msg = L.fc_status_str(status).decode()
        if status == FC_ERR_HIP:
            msg += f" (hipError {L.fc_last_hip_error()})"
        super().__init__(f"{what}: {msg} [status {status}]")
        self.status = status


def _check(status, what):
    if status != FC_OK:
        raise FcError(status, what)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


# ---- argument checks: the C ABI receives bare device pointers and cannot
# check what they point at, so every wrapper checks each tensor's device,
# dtype, shape and contiguity against the batch before the call.
def _need(t, what, dtype, shape, device):
    import torch

    if t is None:
        raise ValueError(f"{what} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch.Tensor, not {type(t).__name__}")
    if t.device != device:
        raise ValueError(f"{what} must be on {device}, not {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, not {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, not {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def _check_pose(batch, pose):
    import torch

    _need(pose, "pose", torch.float32, (7, batch.n_env), batch.device)


def _check_candidates(batch, cand, faces=False):
    import torch

    Q = max(batch.Qf, 1) if faces else batch.Q
    d = batch.device
    _need(cand["phi"], "cand['phi']", torch.float32, (Q,), d)
    _need(cand["normal"], "cand['normal']", torch.float32, (3, Q), d)
    _need(cand["bin"], "cand['bin']", torch.int16, (Q,), d)
    if faces or cand.get("point") is not None:
        _need(cand.get("point"), "cand['point']", torch.float32, (3, Q), d)


def _check_contacts(batch, out):
    import torch

    S, d = batch.n_env * batch.K, batch.device
    _need(out["vidx"], "contacts['vidx']", torch.int32, (S,), d)
    _need(out["depth"], "contacts['depth']", torch.float32, (S,), d)
    _need(out["point"], "contacts['point']", torch.float32, (3, S), d)
    _need(out["normal"], "contacts['normal']", torch.float32, (3, S), d)
    _need(out["count"], "contacts['count']", torch.int32, (batch.n_env,), d)


def _check_grads(batch, grads, upstream):
    import torch

    d, n = batch.device, batch.n_env
    nv = batch.Q if grads.get("per_env") else sum(batch.mesh_sizes)
    if grads.get("loss") is not None:
        _need(grads["loss"], "grads['loss']", torch.float32, (n,), d)
    if grads.get("d_pose") is not None:
        _need(grads["d_pose"], "grads['d_pose']", torch.float32, (6, n), d)
    if grads.get("d_verts") is not None:
        _need(grads["d_verts"], "grads['d_verts']", torch.float32, (3 * nv,), d)
    if upstream is not None:
        _need(upstream, "upstream", torch.float32, (n,), d)


def _check_patches(batch, out, max_patches):
    import torch

    S, d = batch.n_env * int(max_patches), batch.device
    _need(out["count"], "patches['count']", torch.int32, (batch.n_env,), d)
    for k in ("founder", "vidx", "members"):
        _need(out[k], f"patches['{k}']", torch.int32, (S,), d)
    _need(out["depth"], "patches['depth']", torch.float32, (S,), d)
    for k in ("normal", "point"):
        _need(out[k], f"patches['{k}']", torch.float32, (3, S), d)


class Batch:
    """A batch of environments resident on one GPU.

    Holds device tensors of the grids and meshes (SoA), the bin table, the
    opaque fc_batch, and a zero-initialised workspace.
    """

    def __init__(self, grids, meshes, env_grid, env_mesh, bins, margin, device="cuda", layout="linear",
                 env_order=None, band=None):
        import torch

        L = lib()
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.layout = layout
        self.n_env = int(len(env_grid))
        self.K = int(bins.shape[1])
        self._keep = []
        gdesc = (fc_grid * len(grids))()
        self.grid_tensors = []
        for i, g in enumerate(grids):
            vals = np.ascontiguousarray(g.values)
            if g.dtype == "f32":
                t = torch.from_numpy(vals.astype(np.float32, copy=False)).to(self.device)
            else:
                t = torch.from_numpy(vals.view(np.int16)).to(self.device)
            nz, ny, nx = vals.shape
            d = fc_grid(C.c_void_p(t.data_ptr()), DTYPES[g.dtype], 0, nx, ny, nz,
                        (C.c_float * 3)(*[float(np.float32(o)) for o in g.origin]), float(np.float32(g.h)))
            if layout == "sparse":
                bnd = float(np.float32(SPARSE_BAND_VOXELS * g.h if band is None else band))
                t, d = self._to_sparse(t, d, bnd)
            elif layout != "linear":
                lay = LAYOUTS[layout]
                nb = L.fc_grid_brick_bytes(C.byref(d), lay)
                if nb == 0:
                    raise ValueError(f"grid cannot be stored as {layout}")
                bt = torch.empty(nb, dtype=torch.uint8, device=self.device)
                out = fc_grid()
                _check(L.fc_grid_to_bricks(C.byref(d), lay, C.c_void_p(bt.data_ptr()), nb, C.byref(out),
                                           _stream(None)), "fc_grid_to_bricks")
                torch.cuda.synchronize(self.device)
                self._keep.append(t)
                t, d = bt, out
            gdesc[i] = d
            self.grid_tensors.append(t)
        mdesc = (fc_mesh * len(meshes))()
        self.mesh_tensors = []
        self.tri_tensors = []
        for i, m in enumerate(meshes):
            v = np.ascontiguousarray(np.asarray(m.verts, dtype=np.float32).T)  # (3, n)
            t = torch.from_numpy(v).to(self.device)
            n = v.shape[1]
            tris = getattr(m, "tris", None)
            tt, nt = None, 0
            if tris is not None and len(tris):
                tt = torch.from_numpy(np.ascontiguousarray(np.asarray(tris, dtype=np.int32).T)).to(self.device)
                nt = int(tt.shape[1])  # (3, n_tris): corner a of every face, then b, then c
            if n:
                mdesc[i] = fc_mesh(C.c_void_p(t[0].data_ptr()), C.c_void_p(t[1].data_ptr()),
                                   C.c_void_p(t[2].data_ptr()), n, None if tt is None else C.c_void_p(tt.data_ptr()),
                                   nt)
            else:
                mdesc[i] = fc_mesh(None, None, None, 0, None, 0)
            self.mesh_tensors.append(t)
            self.tri_tensors.append(tt)
        self.mesh_sizes = [int(m.verts.shape[0]) for m in meshes]
        eg = np.ascontiguousarray(env_grid, dtype=np.int32)
        em = np.ascontiguousarray(env_mesh, dtype=np.int32)
        self.env_mesh = em
        dirs = np.ascontiguousarray(bins, dtype=np.float32)
        eo = None if env_order is None else np.ascontiguousarray(env_order, dtype=np.int32)
        desc = fc_batch_desc(self.n_env, gdesc, len(grids), mdesc, len(meshes),
                             eg.ctypes.data_as(C.POINTER(C.c_int32)), em.ctypes.data_as(C.POINTER(C.c_int32)),
                             self.K, dirs.ctypes.data_as(C.POINTER(C.c_float)), float(np.float32(margin)),
                             None if eo is None else eo.ctypes.data_as(C.POINTER(C.c_int32)))
        h = C.c_void_p()
        _check(L.fc_batch_create(C.byref(desc), C.byref(h)), "fc_batch_create")
        self.handle = h
        self.Q = int(L.fc_batch_queries(h))
        self.Qf = int(L.fc_batch_face_queries(h))
        self.ws_bytes = int(L.fc_workspace_bytes(h))
        self.workspace = torch.zeros(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")

    def _to_sparse(self, t, d, band):
        """fc_grid_to_sparse of the linear grid tensor t (descriptor d)."""
        import torch

        L = lib()
        nb = C.c_size_t()
        _check(L.fc_grid_sparse_bytes(C.byref(d), band, C.byref(nb), _stream(None)), "fc_grid_sparse_bytes")
        bt = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)
        out = fc_grid()
        _check(L.fc_grid_to_sparse(C.byref(d), band, C.c_void_p(bt.data_ptr()), int(nb.value), C.byref(out),
                                   _stream(None)), "fc_grid_to_sparse")
        self.sparse_bytes = getattr(self, "sparse_bytes", 0) + int(nb.value)
        return bt, out

    @classmethod
    def from_workload(cls, w, device="cuda", layout="linear", env_order=None, band=None):
        return cls(w.grids, w.meshes, w.env_grid, w.env_mesh, w.bins, w.margin, device=device, layout=layout,
                   env_order=env_order, band=band)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.fc_batch_destroy(h)
            self.handle = None

    # ---- output allocation
    def new_candidates(self):
        import torch

        return dict(phi=torch.empty(self.Q, dtype=torch.float32, device=self.device),
                    normal=torch.empty(3, self.Q, dtype=torch.float32, device=self.device),
                    bin=torch.empty(self.Q, dtype=torch.int16, device=self.device))

    def new_face_candidates(self):
        """Per-face candidates: phi, normal [3][Qf], bin, point [3][Qf]."""
        import torch

        Q = max(self.Qf, 1)
        return dict(phi=torch.empty(Q, dtype=torch.float32, device=self.device),
                    normal=torch.empty(3, Q, dtype=torch.float32, device=self.device),
                    bin=torch.empty(Q, dtype=torch.int16, device=self.device),
                    point=torch.empty(3, Q, dtype=torch.float32, device=self.device))

    def new_patches(self, max_patches=PATCH_MAX):
        """Outputs of fc_contact_patches: slot e * N + p."""
        import torch

        S = self.n_env * max_patches
        i32 = dict(dtype=torch.int32, device=self.device)
        f32 = dict(dtype=torch.float32, device=self.device)
        return dict(count=torch.empty(self.n_env, **i32), founder=torch.empty(S, **i32),
                    normal=torch.empty(3, S, **f32), vidx=torch.empty(S, **i32), depth=torch.empty(S, **f32),
                    point=torch.empty(3, S, **f32), members=torch.empty(S, **i32))

    def new_contacts(self):
        import torch

        S = self.n_env * self.K
        return dict(vidx=torch.empty(S, dtype=torch.int32, device=self.device),
                    depth=torch.empty(S, dtype=torch.float32, device=self.device),
                    point=torch.empty(3, S, dtype=torch.float32, device=self.device),
                    normal=torch.empty(3, S, dtype=torch.float32, device=self.device),
                    count=torch.empty(self.n_env, dtype=torch.int32, device=self.device))

    def new_grads(self, per_env=False, loss=True, d_pose=True, d_verts=True):
        import torch

        nv = self.Q if per_env else sum(self.mesh_sizes)
        return dict(loss=torch.empty(self.n_env, dtype=torch.float32, device=self.device) if loss else None,
                    d_pose=torch.empty(6, self.n_env, dtype=torch.float32, device=self.device) if d_pose else None,
                    d_verts=(torch.empty(3 * nv, dtype=torch.float32, device=self.device) if d_verts else None),
                    per_env=bool(per_env))

    def set_timing(self, max_records):
        """Record the main kernel's duration for the next max_records calls (0: off)."""
        _check(lib().fc_batch_set_timing(self.handle, int(max_records)), "fc_batch_set_timing")
        self._timing_cap = int(max_records)

    def read_timing(self):
        """(durations in ms, kernel ids) of the calls recorded since set_timing or the last read."""
        cap = max(getattr(self, "_timing_cap", 0), 1)
        ms = (C.c_float * cap)()
        kid = (C.c_int32 * cap)()
        n = lib().fc_batch_read_timing(self.handle, ms, kid, cap)
        if n < 0:
            raise RuntimeError(f"fc_batch_read_timing failed (hip error {lib().fc_last_hip_error()})")
        return np.array(ms[:n], dtype=np.float64), np.array(kid[:n], dtype=np.int32)

    def set_launch(self, block=256, tile=1024, persistent=0, grid_mult=8, xcd_remap=0, wave_prio=1):
        l = fc_launch(block, tile, persistent, grid_mult, xcd_remap, wave_prio)
        _check(lib().fc_batch_set_launch(self.handle, C.byref(l)), "fc_batch_set_launch")

    def get_launch(self):
        l = fc_launch()
        _check(lib().fc_batch_get_launch(self.handle, C.byref(l)), "fc_batch_get_launch")
        return dict(block=l.block, tile=l.tile, persistent=l.persistent, grid_mult=l.grid_mult,
                    xcd_remap=l.xcd_remap, wave_prio=l.wave_prio)

    def signature(self):
        buf = C.create_string_buffer(1024)
        lib().fc_batch_signature(self.handle, buf, 1024)
        return buf.value.decode()

    def reset_workspace(self):
        _check(lib().fc_workspace_init(self.handle, C.c_void_p(self.workspace.data_ptr()), self.ws_bytes,
                                       _stream(None)), "fc_workspace_init")


def _cand_struct(c):
    return None if c is None else fc_candidates(_ptr(c["phi"]), _ptr(c["normal"]), _ptr(c["bin"]),
                                                _ptr(c.get("point")))


def _contacts_struct(o):
    return None if o is None else fc_contacts(_ptr(o["vidx"]), _ptr(o["depth"]), _ptr(o["point"]),
                                              _ptr(o["normal"]), _ptr(o["count"]))


def _grads_struct(g):
    return fc_grads(_ptr(g.get("loss")), _ptr(g.get("d_pose")), _ptr(g.get("d_verts")),
                    1 if g.get("per_env") else 0)


def _byref(s):
    return None if s is None else C.byref(s)


def fc_sdf_query(batch: Batch, pose, cand=None, fused_out=None, stream=None):
    _check_pose(batch, pose)
    if cand is not None:
        _check_candidates(batch, cand)
    if fused_out is not None:
        _check_contacts(batch, fused_out)
    cs, os_ = _cand_struct(cand), _contacts_struct(fused_out)
    _check(lib().fc_sdf_query(batch.handle, _ptr(pose), _byref(cs), _byref(os_),
                              C.c_void_p(batch.workspace.data_ptr()), batch.ws_bytes, _stream(stream)),
           "fc_sdf_query")


def fc_sdf_query_noalloc(batch: Batch, pose, cand=None, fused_out=None, stream=None):
    """fc_sdf_query on the library's static per-device scratch instead of the
    batch's workspace (no allocation by the call; calls on one device must
    not overlap)."""
    _check_pose(batch, pose)
    if cand is not None:
        _check_candidates(batch, cand)
    if fused_out is not None:
        _check_contacts(batch, fused_out)
    cs, os_ = _cand_struct(cand), _contacts_struct(fused_out)
    _check(lib().fc_sdf_query_noalloc(batch.handle, _ptr(pose), _byref(cs), _byref(os_), _stream(stream)),
           "fc_sdf_query_noalloc")


def fc_contact_reduce(batch: Batch, pose, cand, out, stream=None):
    _check_pose(batch, pose)
    _check_candidates(batch, cand)
    _check_contacts(batch, out)
    _check(lib().fc_contact_reduce(batch.handle, _ptr(pose), C.byref(_cand_struct(cand)),
                                   C.byref(_contacts_struct(out)), C.c_void_p(batch.workspace.data_ptr()),
                                   batch.ws_bytes, _stream(stream)), "fc_contact_reduce")


def fc_sdf_query_backward(batch: Batch, pose, k, grads, upstream=None, stream=None):
    _check_pose(batch, pose)
    _check_grads(batch, grads, upstream)
    _check(lib().fc_sdf_query_backward(batch.handle, _ptr(pose), float(k), _ptr(upstream),
                                       C.byref(_grads_struct(grads)), C.c_void_p(batch.workspace.data_ptr()),
                                       batch.ws_bytes, _stream(stream)), "fc_sdf_query_backward")


def fc_sdf_query_and_backward(batch: Batch, pose, fused_out, k, grads, upstream=None, stream=None):
    _check_pose(batch, pose)
    _check_contacts(batch, fused_out)
    _check_grads(batch, grads, upstream)
    _check(lib().fc_sdf_query_and_backward(batch.handle, _ptr(pose), C.byref(_contacts_struct(fused_out)), float(k),
                                           _ptr(upstream), C.byref(_grads_struct(grads)),
                                           C.c_void_p(batch.workspace.data_ptr()), batch.ws_bytes,
                                           _stream(stream)), "fc_sdf_query_and_backward")


PGD_ITERS, PGD_STEP0 = 8, 0.5  # per-face descent defaults (trials, first step in face sizes)


def fc_sdf_query_faces(batch: Batch, pose, cand=None, fused_out=None, iters=PGD_ITERS, step0=PGD_STEP0,
                       stream=None):
    _check_pose(batch, pose)
    if cand is not None:
        _check_candidates(batch, cand, faces=True)
    if fused_out is not None:
        _check_contacts(batch, fused_out)
    cs, os_ = _cand_struct(cand), _contacts_struct(fused_out)
    p = fc_pgd(int(iters), float(step0))
    _check(lib().fc_sdf_query_faces(batch.handle, _ptr(pose), C.byref(p), _byref(cs), _byref(os_),
                                    C.c_void_p(batch.workspace.data_ptr()), batch.ws_bytes, _stream(stream)),
           "fc_sdf_query_faces")


def fc_contact_patches(batch: Batch, pose, out, max_patches=PATCH_MAX, cos_sim=PATCH_COS, stream=None):
    """Patch reduction (Algorithm 1) of every environment into ``out``
    (Batch.new_patches(max_patches))."""
    _check_pose(batch, pose)
    _check_patches(batch, out, max_patches)
    prm = fc_patch_params(int(max_patches), float(cos_sim))
    ps = fc_patches(*[_ptr(out[k]) for k in ("count", "founder", "normal", "vidx", "depth", "point", "members")])
    _check(lib().fc_contact_patches(batch.handle, _ptr(pose), C.byref(prm), C.byref(ps), _stream(stream)),
           "fc_contact_patches")


def fc_gather_probe(batch: Batch, pose, sink, stream=None):
    """The one-pass kernel's loads without its arithmetic (a measurement aid)."""
    import torch

    _check_pose(batch, pose)
    _need(sink, "sink", torch.float32, tuple(sink.shape), batch.device)
    _check(lib().fc_gather_probe(batch.handle, _ptr(pose), _ptr(sink), _stream(stream)), "fc_gather_probe")


def fc_bake_table(verts, tris) -> np.ndarray:
    """Host table of a closed, outward-wound mesh for fc_bake_sdf: verts
    (n, 3), tris (m, 3) -> float32 array (rows, 4) in the library's layout
    (see fc_bake_table in include/fc.h)."""
    v = np.ascontiguousarray(verts, dtype=np.float32)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
        raise ValueError("verts and tris must be (n, 3) and (m, 3)")
    nb = int(lib().fc_bake_table_bytes(len(t)))
    out = np.zeros((max(nb, 16) // 16, 4), dtype=np.float32)
    _check(lib().fc_bake_table(v.ctypes.data_as(C.c_void_p), len(v), t.ctypes.data_as(C.c_void_p), len(t),
                               out.ctypes.data_as(C.c_void_p), nb), "fc_bake_table")
    return out


class BakeTable:
    """A bake table resident on one GPU (the host table, copied once)."""

    def __init__(self, verts, tris, device="cuda"):
        import torch

        self.n_tris = int(np.asarray(tris).shape[0])
        self.table = torch.from_numpy(fc_bake_table(verts, tris)).to(device)


def fc_bake_sdf(table: BakeTable, dims, origin, h, out=None, stream=None, cull=True):
    """Signed distance of the table's mesh at every node: a float32 tensor
    [nz][ny][nx] (``out`` if given).  ``cull=False`` calls
    fc_bake_sdf_unculled (every node against every triangle)."""
    import torch

    nx, ny, nz = (int(d) for d in dims)
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=table.table.device)
    elif (out.dtype != torch.float32 or out.numel() != nx * ny * nz or not out.is_contiguous()
          or out.device != table.table.device):
        raise ValueError("out must be a contiguous float32 tensor of nx*ny*nz elements")
    o = (C.c_float * 3)(*[float(x) for x in origin])
    name = "fc_bake_sdf" if cull else "fc_bake_sdf_unculled"
    _check(getattr(lib(), name)(_ptr(table.table), table.n_tris, nx, ny, nz, o, float(h), _ptr(out), _stream(stream)),
           name)
    return out


class Graph:
    """An instantiated hipGraph of one step (fused forward and/or backward)."""

    def __init__(self, batch: Batch, pose, fused_out=None, k=0.0, grads=None, upstream=None):
        _check_pose(batch, pose)
        if fused_out is not None:
            _check_contacts(batch, fused_out)
        if grads is not None:
            _check_grads(batch, grads, upstream)
        h = C.c_void_p()
        os_ = _contacts_struct(fused_out)
        gs = None if grads is None else _grads_struct(grads)
        _check(lib().fc_graph_create(batch.handle, _ptr(pose), _byref(os_), float(k), _ptr(upstream),
                                     _byref(gs), C.c_void_p(batch.workspace.data_ptr()), batch.ws_bytes,
                                     C.byref(h)), "fc_graph_create")
        self.handle = h
        self._refs = (batch, pose, fused_out, grads, upstream)

    def launch(self, stream=None):
        _check(lib().fc_graph_launch(self.handle, _stream(stream)), "fc_graph_launch")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.fc_graph_destroy(h)
            self.handle = None


def fc_graph_create(batch, pose, fused_out=None, k=0.0, grads=None, upstream=None) -> Graph:
    return Graph(batch, pose, fused_out, k, grads, upstream)


def fc_autotune_load(path: str) -> int:
    return int(lib().fc_autotune_load(path.encode()))


def locality_order(w):
    """A scheduling order for ``fc_batch_desc.env_order``: envs grouped by
    part type, then sorted along a Z-order curve of their translation, so that
    consecutive envs sit near each other in B's frame.  Host-side, from the
    poses the caller already has."""
    t = np.asarray(w.pose[4:7], dtype=np.float64).T
    lo = t.min(axis=0)
    span = float(np.max(t.max(axis=0) - lo))  # one scale for all axes: the curve follows the real extent
    span = span if span > 0 else 1.0
    q = np.clip(((t - lo) / span * 1023).astype(np.int64), 0, 1023)
    code = np.zeros(len(t), dtype=np.int64)
    for bit in range(10):
        for a in range(3):
            code |= ((q[:, a] >> bit) & 1) << (3 * bit + a)
    return np.lexsort((code, np.asarray(w.env_mesh), np.asarray(w.env_grid))).astype(np.int32)


def pose_tensor(pose_np, device="cuda"):
    import torch

    return torch.from_numpy(np.ascontiguousarray(pose_np, dtype=np.float32)).to(device)
