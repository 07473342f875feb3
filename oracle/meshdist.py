"""Brute-force signed distance to a closed triangle mesh (test infrastructure).

Used only to pin ``query`` on tiny meshes: a grid sampled from this distance
must be reproduced exactly at its nodes, and within the Lipschitz bound in
between.  The paper bakes its SDFs from triangle meshes (Section III-A).

Unsigned distance: the closest point on each triangle by the Voronoi-region
classification of Ericson, *Real-Time Collision Detection* (2005), Sec. 5.1.5,
minimised over triangles.  Sign: the angle-weighted pseudonormal of the
closest feature (face, edge or vertex), Baerentzen and Aanaes, IEEE TVCG 2005;
negative inside.  Pure Python loops: tiny inputs only.
"""
from __future__ import annotations

import math

import numpy as np


def _closest_on_triangle(p, a, b, c):
    """Closest point and feature: ('v', i), ('e', (i, j)) or ('f', None)."""
    ab, ac, ap = b - a, c - a, p - a
    d1, d2 = ab @ ap, ac @ ap
    if d1 <= 0.0 and d2 <= 0.0:
        return a, ("v", 0)
    bp = p - b
    d3, d4 = ab @ bp, ac @ bp
    if d3 >= 0.0 and d4 <= d3:
        return b, ("v", 1)
    vc = d1 * d4 - d3 * d2
    if vc <= 0.0 and d1 >= 0.0 and d3 <= 0.0:
        return a + (d1 / (d1 - d3)) * ab, ("e", (0, 1))
    cp = p - c
    d5, d6 = ab @ cp, ac @ cp
    if d6 >= 0.0 and d5 <= d6:
        return c, ("v", 2)
    vb = d5 * d2 - d1 * d6
    if vb <= 0.0 and d2 >= 0.0 and d6 <= 0.0:
        return a + (d2 / (d2 - d6)) * ac, ("e", (0, 2))
    va = d3 * d6 - d5 * d4
    if va <= 0.0 and (d4 - d3) >= 0.0 and (d5 - d6) >= 0.0:
        w = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        return b + w * (c - b), ("e", (1, 2))
    den = 1.0 / (va + vb + vc)
    return a + ab * (vb * den) + ac * (vc * den), ("f", None)


class MeshSDF:
    def __init__(self, verts, tris):
        self.V = np.asarray(verts, dtype=np.float64)
        self.T = np.asarray(tris, dtype=np.int64)
        fn = []
        vn = np.zeros_like(self.V)
        en = {}
        for f, (i, j, k) in enumerate(self.T):
            a, b, c = self.V[i], self.V[j], self.V[k]
            n = np.cross(b - a, c - a)
            n = n / np.linalg.norm(n)
            fn.append(n)
            for (p, q, r) in ((i, j, k), (j, k, i), (k, i, j)):
                u, v = self.V[q] - self.V[p], self.V[r] - self.V[p]
                ang = math.acos(max(-1.0, min(1.0, (u @ v) / (np.linalg.norm(u) * np.linalg.norm(v)))))
                vn[p] += ang * n
            for (p, q) in ((i, j), (j, k), (k, i)):
                key = (min(p, q), max(p, q))
                en[key] = en.get(key, np.zeros(3)) + n
        self.fn = np.asarray(fn)
        self.vn = vn
        self.en = en

    def __call__(self, p):
        p = np.asarray(p, dtype=np.float64)
        best, sign = np.inf, 1.0
        for f, tri in enumerate(self.T):
            a, b, c = self.V[tri[0]], self.V[tri[1]], self.V[tri[2]]
            q, feat = _closest_on_triangle(p, a, b, c)
            d = float(np.linalg.norm(p - q))
            if d < best:
                if feat[0] == "f":
                    n = self.fn[f]
                elif feat[0] == "v":
                    n = self.vn[tri[feat[1]]]
                else:
                    i, j = tri[feat[1][0]], tri[feat[1][1]]
                    n = self.en[(min(i, j), max(i, j))]
                best = d
                sign = -1.0 if (p - q) @ n < 0.0 else 1.0
        return sign * best

    def many(self, P):
        P = np.asarray(P, dtype=np.float64)
        return np.array([self(p) for p in P.reshape(-1, 3)]).reshape(P.shape[:-1])
