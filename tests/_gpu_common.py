"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the CPU oracle on the same seeded inputs."""
import math

import numpy as np
import pytest

from oracle import query as OQ
from oracle import reduce as ORD

# Tolerances (stated once, used by every parity test).
DEPTH_TOL_F32 = 1e-6  # m: |phi_gpu - phi_fp64| for FP32 grids
NORMAL_TOL = 1e-6  # rad (chord): FP32 normalisation and gradient rounding
FACE_BAND = 1e-4  # voxels: a point this close to a cell face may take either cell
BOUND_BAND = 1e-4  # voxels: this close to the grid boundary the inside test may differ
ULP32 = 2.0 ** -23


def position_error_voxels(o):
    """Bound on |u_fp32 - u_fp64| per query, in voxels.

    x_B = R v + t is three chained FP32 fmas per coordinate (<= 3 roundings of
    |x_B|-sized values, plus R's own rounding times |v|), u = (x - o) * (1/h)
    adds a subtraction and a product rounding and 1/h's rounding.
    """
    xb = np.abs(o["x_b"])
    scale = np.maximum(xb, np.abs(o["u"]) * o["h"][:, None]) + 1e-30
    return (6.0 * ULP32 * scale) / o["h"][:, None] + 2.0 * ULP32 * np.abs(o["u"]) + 1e-7


def gradient_sensitivity(w, o, cells=None):
    """Per query: S = max |mixed second difference| of the cell's corners
    (value units), which bounds |d grad / d t| of the trilinear interpolant
    inside the cell; and cmax = max |corner value| (the scale of the FP32
    rounding in the nested lerps).  ``cells`` overrides o["cell"]."""
    cells = o["cell"] if cells is None else cells
    S = np.zeros(len(cells))
    cmax = np.zeros(len(cells))
    for e in np.unique(o["env"]):
        sel = np.nonzero(o["env"] == e)[0]
        g = w.grids[int(w.env_grid[e])]
        vals = OQ.grid_values_f64(g.values, g.dtype)
        c = cells[sel]
        ix, iy, iz = c[:, 0], c[:, 1], c[:, 2]
        C = {(a, b, d): vals[iz + d, iy + b, ix + a] for a in (0, 1) for b in (0, 1) for d in (0, 1)}
        m = np.zeros(len(sel))
        for k in (0, 1):
            m = np.maximum(m, np.abs(C[1, 1, k] - C[1, 0, k] - C[0, 1, k] + C[0, 0, k]))  # xy plane
            m = np.maximum(m, np.abs(C[1, k, 1] - C[1, k, 0] - C[0, k, 1] + C[0, k, 0]))  # xz plane
            m = np.maximum(m, np.abs(C[k, 1, 1] - C[k, 1, 0] - C[k, 0, 1] + C[k, 0, 0]))  # yz plane
        S[sel] = m
        cmax[sel] = np.max(np.abs(np.stack(list(C.values()))), axis=0)
    return S, cmax


def _round_fraction_f32(x):
    """Round an exact rational to float32, nearest-even."""
    from fractions import Fraction

    r0 = np.float32(float(x))
    cands = [r0, np.nextafter(r0, np.float32(np.inf)), np.nextafter(r0, np.float32(-np.inf))]
    best = None
    for c in cands:
        d = abs(Fraction(float(c)) - x)
        even = (int(np.asarray(c, np.float32).view(np.uint32)) & 1) == 0
        key = (d, 0 if even else 1)
        if best is None or key < best[0]:
            best = (key, c)
    return best[1]


def fma32(a, b, c):
    """float32 fma(a, b, c) with a single rounding, exactly.

    a*b is exact in float64 (24 x 24 bits); a*b + c is rounded once to float64
    and then to float32.  That double rounding can only differ from the single
    rounding when the float64 sum lies within a few float64 ulps of a float32
    midpoint; those elements are redone in exact rational arithmetic."""
    from fractions import Fraction

    a64, b64, c64 = np.broadcast_arrays(*(np.asarray(x, np.float32).astype(np.float64) for x in (a, b, c)))
    s = a64 * b64 + c64
    r = s.astype(np.float32)
    r64 = r.astype(np.float64)
    up = np.nextafter(r, np.float32(np.inf)).astype(np.float64)
    dn = np.nextafter(r, np.float32(-np.inf)).astype(np.float64)
    d = np.minimum(np.abs(s - (r64 + up) / 2), np.abs(s - (r64 + dn) / 2))
    risky = np.nonzero(d <= 4 * np.spacing(np.abs(s)))[0]
    for i in risky:
        r[i] = _round_fraction_f32(Fraction(float(a64[i])) * Fraction(float(b64[i])) + Fraction(float(c64[i])))
    return r


def bins_fp32(normal, dirs):
    """The kernels' bin rule on given float32 normals: d_k = fma(nz, dz, fma(ny, dy, nx*dx)),
    lowest k with the largest d_k (strict >), evaluated exactly in float32."""
    nx, ny, nz = (np.asarray(v, np.float32) for v in normal)
    D = np.asarray(dirs, np.float32)
    K = D.shape[1]
    best = fma32(nz, D[2, 0], fma32(ny, D[1, 0], nx * D[0, 0]))
    b = np.zeros(len(nx), np.int64)
    for k in range(1, K):
        v = fma32(nz, D[2, k], fma32(ny, D[1, k], nx * D[0, k]))
        better = v > best
        best = np.where(better, v, best)
        b = np.where(better, k, b)
    return b


def check_bins_exact(w, cand, envs):
    """Every candidate's bin equals the kernels' rule re-evaluated on the CPU
    from the GPU's own normal (bit-exact: catches any omission in the bin
    search table)."""
    rows = rows_of(w, envs)
    b = cand["bin"][rows].astype(np.int64)
    sel = np.nonzero(b >= 0)[0]
    nrm = cand["normal"][:, rows[sel]]
    ref = bins_fp32(nrm, w.bins)
    bad = ref != b[sel]
    assert not bad.any(), f"bin differs from the FP32 rule at rows {rows[sel][bad][:10]}"
    return int(len(sel))


def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    return torch


def to_np(d):
    out = {}
    for k, v in d.items():
        if hasattr(v, "detach"):
            out[k] = v.detach().cpu().numpy()
        else:
            out[k] = v
    return out


def rows_of(w, envs):
    off = w.env_query_offsets()
    return np.concatenate([np.arange(off[e], off[e + 1]) for e in envs]).astype(np.int64)


def oracle_rows(w, envs):
    """Oracle results for the envs, plus grid coordinates u and the grid dims per row."""
    o = OQ.query_workload(w, envs)
    u = np.empty_like(o["x_b"])
    dims = np.empty_like(o["x_b"])
    hh = np.empty(len(u))
    for e in envs:
        g = w.grids[int(w.env_grid[e])]
        sel = o["env"] == e
        u[sel] = (o["x_b"][sel] - np.asarray(g.origin)) / g.h
        dims[sel] = g.dims
        hh[sel] = g.h
    o["u"], o["dims"], o["h"] = u, dims, hh
    return o


def normal_bound(w, o, du, cells=None, grads=None):
    """|n_fp32 - n_fp64| bound per query: 2 (sqrt(3) S du + 8 ulp cmax) / |g| (+ NORMAL_TOL)."""
    grads = o["grad"] if grads is None else grads
    S, cmax = gradient_sensitivity(w, o, cells)
    gvox = np.linalg.norm(grads, axis=1) * o["h"]
    return NORMAL_TOL + 2.0 * (math.sqrt(3.0) * S * du + 8.0 * ULP32 * cmax) / np.maximum(gvox, 1e-30)


def _alt_normals(w, o, idx, band):
    """Oracle normals, with their own error bounds, at points nudged across
    nearby cell faces on every combination of the near axes (within the FP32
    position error either neighbouring cell is valid)."""
    import itertools

    alts = []
    sub = {k: (v[idx] if hasattr(v, "__len__") and len(v) == len(o["phi"]) else v) for k, v in o.items()}
    t = sub["u"] - np.floor(sub["u"])
    bnd = band[idx][:, None]
    near = (t < bnd) | (t > 1 - bnd)
    du = np.max(position_error_voxels(sub), axis=1)
    for sgn in itertools.product((-1.0, 0.0, 1.0), repeat=3):
        if sgn == (0.0, 0.0, 0.0):
            continue
        step = np.asarray(sgn)[None, :] * near * (2.0 * bnd * sub["h"][:, None])
        x = sub["x_b"] + step
        n = np.zeros_like(x)
        grads = np.zeros_like(x)
        cells = np.zeros_like(sub["cell"])
        for e in np.unique(sub["env"]):
            sel = sub["env"] == e
            g = w.grids[int(w.env_grid[e])]
            vals = OQ.grid_values_f64(g.values, g.dtype)
            _, grads[sel], _, cells[sel] = OQ.sample(vals, g.origin, g.h, g.dims, x[sel])
            n[sel], _, _ = OQ.normals_and_bins(grads[sel], w.bins)
        tol = normal_bound(w, sub, du, cells, grads)
        alts.append((n, tol))
    return alts


def check_candidates(w, cand, envs, depth_tol=DEPTH_TOL_F32, o=None):
    """Element-wise parity of per-query candidates against the FP64 oracle.

    Returns a dict of counts of the legitimately ambiguous cases.
    """
    if o is None:
        o = oracle_rows(w, envs)
    rows = rows_of(w, envs)
    phi = cand["phi"][rows].astype(np.float64)
    nrm = cand["normal"][:, rows].T.astype(np.float64)
    b = cand["bin"][rows].astype(np.int64)
    stats = {}
    # inside decision
    u, dims = o["u"], o["dims"]
    with np.errstate(invalid="ignore"):
        near_bound = np.any((np.abs(u) < BOUND_BAND) | (np.abs(u - (dims - 1)) < BOUND_BAND), axis=1)
    g_inside = np.isfinite(phi)
    bad = (g_inside != o["inside"]) & ~near_bound
    assert not bad.any(), f"inside mismatch at rows {rows[bad][:10]}"
    both = g_inside & o["inside"]
    stats["boundary_band"] = int(((g_inside != o["inside"]) & near_bound).sum())
    # value
    err = np.abs(phi[both] - o["phi"][both])
    stats["max_depth_err"] = float(err.max()) if err.size else 0.0
    assert stats["max_depth_err"] <= depth_tol, stats["max_depth_err"]
    # candidate decision
    m = np.float64(np.float32(w.margin))
    g_cand = b >= 0
    amb = both & (np.abs(o["phi"] - m) <= depth_tol)
    bad = (g_cand != o["cand"]) & ~amb & both
    assert not bad.any(), f"candidate mismatch at rows {rows[bad][:10]}"
    assert not (g_cand & ~g_inside).any()
    # normals: within the FP32 bound; within the FP32 position error of a cell
    # face either cell's normal is valid.
    du3 = position_error_voxels(o)
    du = np.max(du3, axis=1)
    tol = normal_bound(w, o, du)
    band = np.maximum(FACE_BAND, 2.0 * du)
    t = o["u"] - np.floor(o["u"])
    near_face = np.any((t < band[:, None]) | (t > 1 - band[:, None]), axis=1) & both
    nerr = np.linalg.norm(nrm - o["normal"], axis=1)
    bad = (nerr > tol) & both & ~near_face
    assert not bad.any(), f"normal mismatch at rows {rows[bad][:10]} err {nerr[bad][:5]} tol {tol[bad][:5]}"
    far = both & ~near_face
    stats["max_normal_err"] = float(nerr[far].max()) if far.any() else 0.0
    stats["max_normal_err_over_bound"] = float((nerr / tol)[far].max()) if far.any() else 0.0
    nf = np.nonzero(near_face & (nerr > tol))[0]
    stats["face_band"] = int(near_face.sum())
    alts = _alt_normals(w, o, nf, band) if len(nf) else []
    if len(nf):
        ok = np.zeros(len(nf), bool)
        for a, ta in alts:
            ok |= np.linalg.norm(nrm[nf] - a, axis=1) <= ta
        assert ok.all(), f"near-face normal mismatch at rows {rows[nf[~ok]][:10]}"
    # bins, where both sides call it a candidate: the GPU's bin must be an
    # argmax of the FP64 dots up to the normal error bound
    cc = g_cand & o["cand"]
    dmax = o["dots"].max(axis=1)
    bsafe = np.clip(b, 0, o["dots"].shape[1] - 1)
    dgpu = np.take_along_axis(o["dots"], bsafe[:, None], axis=1)[:, 0]
    okb = (b == o["bin"]) | (dgpu >= dmax - 2.0 * tol - 1e-7)
    if len(nf):
        dirs = np.asarray(w.bins, np.float32).astype(np.float64)
        for a, ta in alts:
            da = a @ dirs
            dg = np.take_along_axis(da, np.clip(b[nf], 0, da.shape[1] - 1)[:, None], axis=1)[:, 0]
            okb[nf] |= dg >= da.max(axis=1) - 2.0 * ta - 1e-7
    bad = cc & ~okb
    assert not bad.any(), f"bin mismatch at rows {rows[bad][:10]}"
    stats["bin_near_tie"] = int((cc & (b != o["bin"])).sum())
    stats["bins_checked_exact"] = check_bins_exact(w, cand, envs)
    stats["n"] = int(len(rows))
    stats["cand"] = int(g_cand.sum())
    return stats


def check_reduction_exact(w, cand, out, envs):
    """Reduced contacts == the oracle's exact reduction of the GPU's own candidates, bit for bit."""
    rows = rows_of(w, envs)
    off = w.env_query_offsets()
    env = np.concatenate([np.full(off[e + 1] - off[e], e) for e in envs])
    vidx = rows - off[env]
    phi = cand["phi"][rows]
    depth = (-phi).astype(np.float32)
    b = cand["bin"][rows].astype(np.int64)
    wv, wd, wrow = ORD.reduce_contacts(env, vidx, depth, b, b >= 0, w.n_env, w.K)
    K = w.K
    for e in envs:
        s = slice(e * K, (e + 1) * K)
        assert np.array_equal(out["vidx"][s], wv[e]), e
        assert np.array_equal(out["depth"][s].view(np.uint32), wd[e].view(np.uint32)), e
        assert out["count"][e] == int((wv[e] >= 0).sum()), e
        full = wv[e] >= 0
        # winner normal is the candidate's normal, bit for bit
        q = off[e] + wv[e][full]
        assert np.array_equal(out["normal"][:, s][:, full].view(np.uint32), cand["normal"][:, q].view(np.uint32)), e
        assert np.all(out["normal"][:, s][:, ~full] == 0) and np.all(out["point"][:, s][:, ~full] == 0)
    return wv, wd


def check_points(w, out, envs, tol=1e-7):
    """Winner points equal the FP64 transform of the winning vertex (FP32 rounding only)."""
    K = w.K
    for e in envs:
        s = slice(e * K, (e + 1) * K)
        v = out["vidx"][s]
        full = v >= 0
        if not full.any():
            continue
        mesh = w.meshes[int(w.env_mesh[e])]
        xb = OQ.transform(w.pose[:, e], mesh.verts[v[full]])
        assert np.max(np.abs(out["point"][:, s][:, full].T - xb)) <= tol


def assert_same(a, b, keys=None):
    keys = keys or a.keys()
    for k in keys:
        if a[k] is None:
            continue
        x, y = np.asarray(a[k]), np.asarray(b[k])
        assert x.shape == y.shape, k
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), f"{k} differs"
