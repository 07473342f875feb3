"""FP64 reference of baking a signed-distance grid from a closed triangle
mesh (test infrastructure only).

Section III-A: the SDF of a body is generated from its triangle mesh ahead
of time, by sampling.  Here every grid node takes the distance to the
nearest triangle, signed by the angle-weighted pseudonormal of the closest
feature (Baerentzen and Aanaes 2005: the face normal, the sum of the two
adjacent face normals for an edge, the angle-weighted sum of the incident
face normals for a vertex), negative inside.  The closest point on a
triangle is Ericson's Voronoi-region classification (Real-Time Collision
Detection, 2005, Sec. 5.1.5).

The same definition as ``meshdist.MeshSDF`` (pure Python, tiny meshes),
vectorised over grid nodes for moderate sizes.  Readings (also in the
design notes): node (i, j, k) at origin + h (i, j, k), stored [nz][ny][nx];
the nearest triangle is the one with the smallest distance, the lowest
triangle index among exact ties; the mesh is closed and consistently wound
(outward normals by the right-hand rule).
"""
from __future__ import annotations

import math

import numpy as np

FACE, EDGE_AB, EDGE_AC, EDGE_BC, VERT_A, VERT_B, VERT_C = range(7)


def closest_on_triangle(P, a, b, c):
    """Closest point of triangle (a, b, c) to each row of P (n, 3) and the
    feature it lies on (FACE, EDGE_*, VERT_*), by Ericson's region tests."""
    ab, ac = b - a, c - a
    ap = P - a
    d1, d2 = ap @ ab, ap @ ac
    bp = P - b
    d3, d4 = bp @ ab, bp @ ac
    cp = P - c
    d5, d6 = cp @ ab, cp @ ac
    vc = d1 * d4 - d3 * d2
    vb = d5 * d2 - d1 * d6
    va = d3 * d6 - d5 * d4
    n = len(P)
    q = np.empty((n, 3))
    feat = np.full(n, -1, dtype=np.int64)
    done = np.zeros(n, dtype=bool)

    def take(mask, pts, code):
        m = mask & ~done
        q[m] = pts[m] if pts.ndim == 2 else pts
        feat[m] = code
        done[m] = True

    with np.errstate(divide="ignore", invalid="ignore"):
        take((d1 <= 0) & (d2 <= 0), a, VERT_A)
        take((d3 >= 0) & (d4 <= d3), b, VERT_B)
        take((vc <= 0) & (d1 >= 0) & (d3 <= 0), a + (d1 / (d1 - d3))[:, None] * ab, EDGE_AB)
        take((d6 >= 0) & (d5 <= d6), c, VERT_C)
        take((vb <= 0) & (d2 >= 0) & (d6 <= 0), a + (d2 / (d2 - d6))[:, None] * ac, EDGE_AC)
        w = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        take((va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0), b + w[:, None] * (c - b), EDGE_BC)
        den = 1.0 / (va + vb + vc)
        take(np.ones(n, dtype=bool), a + (vb * den)[:, None] * ab + (vc * den)[:, None] * ac, FACE)
    return q, feat


def pseudonormals(V, T):
    """Face normals (m, 3), per-face edge pseudonormals (m, 3, 3) for edges
    (ab, ac, bc), per-vertex angle-weighted pseudonormals (n, 3)."""
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    fn = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    fn /= np.linalg.norm(fn, axis=1, keepdims=True)
    vn = np.zeros_like(V)
    edge = {}
    for f, (i, j, k) in enumerate(T):
        for p, q, r in ((i, j, k), (j, k, i), (k, i, j)):
            u, v = V[q] - V[p], V[r] - V[p]
            ang = math.acos(max(-1.0, min(1.0, (u @ v) / (np.linalg.norm(u) * np.linalg.norm(v)))))
            vn[p] += ang * fn[f]
        for p, q in ((i, j), (j, k), (k, i)):
            key = (min(p, q), max(p, q))
            edge[key] = edge.get(key, np.zeros(3)) + fn[f]
    en = np.zeros((len(T), 3, 3))
    for f, (i, j, k) in enumerate(T):
        for slot, (p, q) in enumerate(((i, j), (i, k), (j, k))):
            en[f, slot] = edge[(min(p, q), max(p, q))]
    return fn, en, vn


def bake(V, T, dims, origin, h):
    """Signed distance at every node of the grid, [nz][ny][nx] float64."""
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    P = np.stack([origin[0] + h * x, origin[1] + h * y, origin[2] + h * z], -1).reshape(-1, 3)
    fn, en, vn = pseudonormals(V, T)
    best = np.full(len(P), np.inf)
    nrm = np.zeros((len(P), 3))
    qbest = np.zeros((len(P), 3))
    for f, (i, j, k) in enumerate(T):
        q, feat = closest_on_triangle(P, V[i], V[j], V[k])
        d = np.sqrt(np.sum((P - q) ** 2, axis=1))
        closer = d < best  # strict: the lowest index keeps exact ties
        if not closer.any():
            continue
        n = np.empty((len(P), 3))
        n[feat == FACE] = fn[f]
        for code, slot in ((EDGE_AB, 0), (EDGE_AC, 1), (EDGE_BC, 2)):
            n[feat == code] = en[f, slot]
        for code, vi in ((VERT_A, i), (VERT_B, j), (VERT_C, k)):
            n[feat == code] = vn[vi]
        best = np.where(closer, d, best)
        nrm = np.where(closer[:, None], n, nrm)
        qbest = np.where(closer[:, None], q, qbest)
    sign = np.where(np.sum((P - qbest) * nrm, axis=1) < 0.0, -1.0, 1.0)
    return (sign * best).reshape(nz, ny, nx)
