"""FP64 reference of the per-vertex SDF query (test infrastructure only).

Follows Section III-A of the paper (an SDF maps a point to its signed
distance; the sign tells inside from outside; the gradient gives the contact
normal that pushes the colliding body out; the SDF is a sampled grid read
with trilinear filtering) and the Generate step of Algorithm 1 (Section
III-C: candidate contacts of a mesh queried against the other body's SDF).
A contact record holds a point, a normal and a distance (Section III-B).

Readings where the paper is silent (each also listed in the design notes):
  * grid samples are node-centred: node (i, j, k) at origin + h (i, j, k),
    stored [nz][ny][nx] with x fastest; no half-voxel offset;
  * a point is inside the grid iff 0 <= u_a <= n_a - 1 on every axis, with
    u = (x - origin) / h; outside points are never candidates;
  * the cell is i_a = min(floor(u_a), n_a - 2), local coordinate
    t_a = u_a - i_a in [0, 1] (a point on a shared face uses the upper cell,
    one on the far boundary the last cell);
  * the gradient is the exact derivative of the trilinear interpolant inside
    that cell (the paper differences the field numerically; the interpolant's
    derivative is the analytic counterpart);
  * candidate iff phi < margin (strict); depth = -phi; point = x_B in B's
    frame; normal = grad / |grad|, or 0 when the gradient vanishes;
  * bin = the lowest k maximising normal . d_k over the given direction
    table (fixed normal-direction bins stand in for the paper's
    normal-similarity patches); a zero normal lands in bin 0;
  * quaternions are (x, y, z, w) and are not renormalised:
    R = I + 2 w [v]x + 2 [v]x^2.
"""
from __future__ import annotations

import numpy as np


def grid_values_f64(values: np.ndarray, dtype: str) -> np.ndarray:
    """Exact promotion of stored samples to FP64 ([nz][ny][nx])."""
    if dtype == "f64":  # FP64 samples: used by the pin tests for exact fields
        return np.asarray(values, dtype=np.float64)
    if dtype == "f32":
        return np.asarray(values, dtype=np.float32).astype(np.float64)
    if dtype == "f16":
        return np.asarray(values, dtype=np.uint16).view(np.float16).astype(np.float64)
    if dtype == "bf16":
        u = np.asarray(values, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
        return u.view(np.float32).astype(np.float64)
    raise ValueError(f"unknown grid dtype {dtype!r}")


def skew(v):
    """[v]x, the cross-product matrix: skew(a) @ b == a x b."""
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def rotation_from_quaternion(q):
    """R(q) = I + 2 w [v]x + 2 [v]x^2 for q = (x, y, z, w), no renormalisation."""
    q = np.asarray(q, dtype=np.float64)
    V = skew(q[:3])
    return np.eye(3) + 2.0 * q[3] * V + 2.0 * (V @ V)


def transform(pose, verts):
    """x_B = R v + t for every vertex (pose = qx qy qz qw tx ty tz)."""
    pose = np.asarray(pose, dtype=np.float64)
    R = rotation_from_quaternion(pose[:4])
    v = np.asarray(verts, dtype=np.float64)
    return v @ R.T + pose[4:7]


def locate(x, origin, h, dims):
    """Grid coordinates, in-grid test, cell index and local coordinates."""
    o = np.asarray(origin, dtype=np.float64)
    n = np.asarray(dims, dtype=np.float64)  # (nx, ny, nz)
    u = (np.asarray(x, dtype=np.float64) - o) / np.float64(h)
    with np.errstate(invalid="ignore"):
        inside = np.all((u >= 0.0) & (u <= n - 1.0), axis=-1)
    us = np.where(inside[..., None], u, 0.0)
    cell = np.minimum(np.floor(us), n - 2.0)
    t = us - cell
    return inside, cell.astype(np.int64), t


def trilinear_value_grad(vals64, cell, t, h):
    """phi and its exact gradient inside the cell.

    phi = sum_{a,b,c in {0,1}} W_a(tx) W_b(ty) W_c(tz) C[a,b,c],
    W_0(s) = 1 - s, W_1(s) = s, C[a,b,c] = value at node cell + (a, b, c);
    d phi / dx = (1/h) sum_{b,c} W_b(ty) W_c(tz) (C[1,b,c] - C[0,b,c]), and
    the same for y and z.
    """
    ix, iy, iz = cell[..., 0], cell[..., 1], cell[..., 2]
    tx, ty, tz = t[..., 0], t[..., 1], t[..., 2]
    W = {0: (1.0 - tx, 1.0 - ty, 1.0 - tz), 1: (tx, ty, tz)}
    C = {}
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                C[a, b, c] = vals64[iz + c, iy + b, ix + a]
    phi = np.zeros(np.shape(tx))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                phi = phi + W[a][0] * W[b][1] * W[c][2] * C[a, b, c]
    gx = np.zeros_like(phi)
    gy = np.zeros_like(phi)
    gz = np.zeros_like(phi)
    for p in (0, 1):
        for q in (0, 1):
            gx = gx + W[p][1] * W[q][2] * (C[1, p, q] - C[0, p, q])
            gy = gy + W[p][0] * W[q][2] * (C[p, 1, q] - C[p, 0, q])
            gz = gz + W[p][0] * W[q][1] * (C[p, q, 1] - C[p, q, 0])
    grad = np.stack([gx, gy, gz], axis=-1) / np.float64(h)
    return phi, grad


def sample(grid_vals64, origin, h, dims, x):
    """phi, grad, inside, cell at arbitrary B-frame points (NaN phi outside)."""
    inside, cell, t = locate(x, origin, h, dims)
    phi, grad = trilinear_value_grad(grid_vals64, cell, t, h)
    phi = np.where(inside, phi, np.nan)
    grad = np.where(inside[..., None], grad, 0.0)
    return phi, grad, inside, cell


def normals_and_bins(grad, bins):
    """Unit normal (0 for a zero gradient) and lowest-k argmax bin."""
    nrm = np.sqrt(np.sum(grad * grad, axis=-1))
    safe = np.where(nrm > 0.0, nrm, 1.0)
    n = np.where((nrm > 0.0)[..., None], grad / safe[..., None], 0.0)
    d = np.asarray(bins, dtype=np.float32).astype(np.float64)  # [3][K]
    dots = n @ d
    return n, np.argmax(dots, axis=-1).astype(np.int64), dots


def query_env(grid, verts, pose, margin, bins, vals64=None):
    """All per-vertex quantities for one environment.

    ``grid`` has .values/.dtype/.origin/.h/.dims; ``verts`` (n,3) float32;
    ``pose`` the env's 7 pose values; ``bins`` float32 [3][K].
    """
    if vals64 is None:
        vals64 = grid_values_f64(grid.values, grid.dtype)
    xb = transform(pose, verts)
    phi, grad, inside, cell = sample(vals64, grid.origin, grid.h, grid.dims, xb)
    with np.errstate(invalid="ignore"):
        cand = inside & (phi < np.float64(np.float32(margin)))
    n, b, dots = normals_and_bins(grad, bins)
    return dict(x_b=xb, phi=phi, grad=grad, inside=inside, cell=cell, cand=cand,
                depth=-phi, normal=n, bin=b, dots=dots)


def query_workload(w, envs=None):
    """Concatenated per-query results over environments (default: all).

    Adds ``env`` and ``vidx`` columns; rows follow q = offset[e] + v.
    """
    envs = range(w.n_env) if envs is None else envs
    cache = {}
    parts = []
    for e in envs:
        gi, mi = int(w.env_grid[e]), int(w.env_mesh[e])
        if gi not in cache:
            g = w.grids[gi]
            cache[gi] = grid_values_f64(g.values, g.dtype)
        r = query_env(w.grids[gi], w.meshes[mi].verts, w.pose[:, e], w.margin, w.bins, cache[gi])
        n = len(r["phi"])
        r["env"] = np.full(n, e, dtype=np.int64)
        r["vidx"] = np.arange(n, dtype=np.int64)
        parts.append(r)
    out = {}
    for k in parts[0]:
        out[k] = np.concatenate([p[k] for p in parts], axis=0)
    return out
