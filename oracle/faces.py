"""FP64 reference of per-face contact generation (test infrastructure only).

Section III-A: besides testing vertices, a contact can be generated for each
triangle of A's mesh, at the point of the face closest to body B, found by
iterative local minimisation of B's signed distance over the face with
projected gradient descent and an adaptive step; the face's contact is then
recorded and reduced like a vertex's (Section III-B record, Algorithm 1).

The paper names the method but not its constants or details.  Readings
(listed with the others in the design notes):
  * the face is parametrised by barycentric coordinates b in the simplex
    {b >= 0, b_a + b_b + b_c = 1}; x(b) = b_a x_a + b_b x_b + b_c x_c with
    the corners in B's frame (x_i = R v_i + t); phi and its gradient are the
    trilinear interpolant and its exact derivative (as for vertices);
  * descent starts at the centroid b = (1/3, 1/3, 1/3);
  * the gradient with respect to b is d_i = grad phi(x) . x_i; a trial is
    b' = P(b - alpha d), P the Euclidean projection onto the simplex (adding
    a constant to all of d does not change b', so no tangential projection
    is needed; it is evaluated as (0, g.e1, g.e2) with e1, e2 the edges from
    the first corner, which keeps a tiny or point-like face well scaled);
  * adaptive step: the trial is accepted iff phi(x(b')) < phi(x(b)) (a trial
    outside the grid counts as +infinity); alpha doubles after an accepted
    trial and halves after a rejected one; a fixed number of trials (iters);
  * the first step is alpha_0 = step0 / sqrt(S), S = sum_i |x_i - centroid|^2
    (alpha_0 = 0 for a degenerate face), so a unit gradient moves the point by
    about step0 times the face's size;
  * the contact is the final point: candidate iff it is inside the grid and
    phi < margin; depth = -phi, normal and bin as for vertices, and the
    reduction's tie-break index is the face index.
"""
from __future__ import annotations

import numpy as np

from .query import grid_values_f64, normals_and_bins, sample, transform


def project_simplex(y):
    """Euclidean projection of each row of y (n, 3) onto the probability
    simplex: the sort-and-threshold rule (Held, Wolfe and Crowder 1974)."""
    y = np.asarray(y, dtype=np.float64)
    u = -np.sort(-y, axis=1)  # descending
    css = np.cumsum(u, axis=1) - 1.0
    j = np.arange(1, y.shape[1] + 1, dtype=np.float64)
    positive = (u - css / j) > 0.0
    rho = positive.sum(axis=1)  # the positive entries form a prefix
    theta = css[np.arange(len(y)), rho - 1] / rho
    return np.maximum(y - theta[:, None], 0.0)


def trial_point(b, alpha, d):
    """One projected step: P(b - alpha d)."""
    return project_simplex(b - alpha[:, None] * d)


def accept(phi_trial, phi):
    """A trial is kept iff it strictly lowers phi."""
    return phi_trial < phi


def pgd_faces(vals64, origin, h, dims, X, iters, step0):
    """Projected gradient descent of phi over each face.

    X: (F, 3, 3) face corners in B's frame.  The face is written from its
    first corner, x(b) = x_a + b_b e1 + b_c e2 with e1 = x_b - x_a,
    e2 = x_c - x_a, and the b-gradient as (0, g.e1, g.e2) (the same trial
    points as (g.x_a, g.x_b, g.x_c), whose common part the projection
    ignores); S = (|e1|^2 + |e2|^2 + |e2 - e1|^2) / 3 is the sum of squared
    corner distances to the centroid.  Returns the final barycentric
    coordinates, point, phi (+inf outside the grid), gradient, and the phi of
    the starting point."""
    X = np.asarray(X, dtype=np.float64)
    F = X.shape[0]
    xa = X[:, 0]
    e1, e2 = X[:, 1] - xa, X[:, 2] - xa

    def point(b):
        return xa + b[:, 1:2] * e1 + b[:, 2:3] * e2

    b = np.full((F, 3), 1.0 / 3.0)
    x = point(b)
    phi, g, inside, _ = sample(vals64, origin, h, dims, x)
    phi = np.where(inside, phi, np.inf)
    phi0 = phi.copy()
    S = (np.sum(e1 * e1, 1) + np.sum(e2 * e2, 1) + np.sum((e2 - e1) ** 2, 1)) / 3.0
    alpha = np.where(S > 0.0, step0 / np.sqrt(np.where(S > 0.0, S, 1.0)), 0.0)
    for _ in range(iters):
        d = np.stack([np.zeros(F), np.sum(g * e1, 1), np.sum(g * e2, 1)], axis=1)
        bt = trial_point(b, alpha, d)
        xt = point(bt)
        pt, gt, it, _ = sample(vals64, origin, h, dims, xt)
        pt = np.where(it, pt, np.inf)
        acc = accept(pt, phi)
        b = np.where(acc[:, None], bt, b)
        x = np.where(acc[:, None], xt, x)
        phi = np.where(acc, pt, phi)
        g = np.where(acc[:, None], gt, g)
        alpha = np.where(acc, 2.0 * alpha, 0.5 * alpha)
    return b, x, phi, g, phi0


def face_corners(pose, verts, tris):
    """(F, 3, 3) corners of every face in B's frame."""
    xb = transform(pose, verts)
    t = np.asarray(tris, dtype=np.int64)
    return np.stack([xb[t[:, 0]], xb[t[:, 1]], xb[t[:, 2]]], axis=1)


def query_faces_env(grid, verts, tris, pose, margin, bins, iters, step0, vals64=None):
    """All per-face quantities for one environment."""
    if vals64 is None:
        vals64 = grid_values_f64(grid.values, grid.dtype)
    X = face_corners(pose, verts, tris)
    b, x, phi, g, phi0 = pgd_faces(vals64, grid.origin, grid.h, grid.dims, X, iters, step0)
    inside = np.isfinite(phi)
    with np.errstate(invalid="ignore"):
        cand = inside & (phi < np.float64(np.float32(margin)))
    n, bn, dots = normals_and_bins(g, bins)
    return dict(bary=b, x_b=x, phi=phi, grad=g, phi0=phi0, inside=inside, cand=cand, depth=-phi, normal=n,
                bin=bn, dots=dots, corners=X)


def query_faces_workload(w, iters, step0, envs=None):
    """Concatenated per-face results over environments (default: all); adds
    ``env`` and ``fidx`` columns; rows follow q = face_offset[e] + f."""
    envs = range(w.n_env) if envs is None else envs
    cache = {}
    parts = []
    for e in envs:
        gi, mi = int(w.env_grid[e]), int(w.env_mesh[e])
        if gi not in cache:
            g = w.grids[gi]
            cache[gi] = grid_values_f64(g.values, g.dtype)
        m = w.meshes[mi]
        r = query_faces_env(w.grids[gi], m.verts, m.tris, w.pose[:, e], w.margin, w.bins, iters, step0, cache[gi])
        n = len(r["phi"])
        r["env"] = np.full(n, e, dtype=np.int64)
        r["fidx"] = np.arange(n, dtype=np.int64)
        parts.append(r)
    return {k: np.concatenate([p[k] for p in parts], axis=0) for k in parts[0]}
