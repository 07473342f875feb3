"""Penetration-penalty loss, its analytic gradients and finite differences.

Test infrastructure only.  Per environment e with pose T = (R, t):

    L_e = sum over vertices v with x_B = R v + t inside the grid and
          phi(x_B) < 0 of  0.5 k phi(x_B)^2 .

The paper's SDF gradient pushes a colliding body out of the surface
(Section III-A); the penalty turns that push into a differentiable objective.
With w = k phi grad(phi) at each penetrating vertex:

    dL/dv         = R^T w                       (vertex in A's frame)
    dL/d rho      = sum w                       (translation part of the twist)
    dL/d omega    = sum x_B x w                 (rotation part of the twist)

for a left (B-frame) perturbation T <- exp(xi^) T, xi = (rho, omega),
evaluated at xi = 0.  ``fd_*`` difference the same loss in FP64: translations
move x_B by +-h e_i; rotations turn x_B about B's origin by +-h about e_i.
Where a perturbed vertex leaves its trilinear cell the loss has a kink; such
components are flagged and an error bound for them is returned.

Every function samples the dense grid unless given ``sampler``, a callable
x -> (phi, grad, inside, cell) over B-frame points, such as the narrow-band
sparse grid's field (``oracle.sparse.sparse_sampler``).  That field is the
dense interpolant in stored bricks and a coarse trilinear interpolant in the
others; its kinks lie on fine cell faces (coarse cell faces are fine cell
faces too), so the fine cell still flags every kink, and a few smooth
crossings besides, which only widens the bound.
"""
from __future__ import annotations

import numpy as np

from . import query as Q


def dense_sampler(grid, vals64=None):
    """x -> (phi, grad, inside, cell) of the grid's trilinear interpolant."""
    if vals64 is None:
        vals64 = Q.grid_values_f64(grid.values, grid.dtype)
    return lambda x: Q.sample(vals64, grid.origin, grid.h, grid.dims, x)


def _terms(sampler, x, k):
    phi, grad, inside, cell = sampler(x)
    with np.errstate(invalid="ignore"):
        act = inside & (phi < 0.0)
    term = np.where(act, 0.5 * k * np.where(act, phi, 0.0) ** 2, 0.0)
    return term, phi, grad, act, cell


def penalty_env(grid, verts, pose, k, vals64=None, sampler=None):
    """(loss, d_twist (6,), d_verts (n,3)) for one environment, FP64."""
    sampler = sampler or dense_sampler(grid, vals64)
    pose = np.asarray(pose, dtype=np.float64)
    R = Q.rotation_from_quaternion(pose[:4])
    xb = Q.transform(pose, verts)
    term, phi, grad, act, _ = _terms(sampler, xb, k)
    w = np.where(act[:, None], k * np.where(act, phi, 0.0)[:, None] * grad, 0.0)
    d_rho = w.sum(axis=0)
    d_omega = np.cross(xb, w).sum(axis=0)
    d_verts = w @ R  # row v: R^T w_v
    return term.sum(), np.concatenate([d_rho, d_omega]), d_verts


def penalty_terms_abs(grid, verts, pose, k, vals64=None, sampler=None):
    """Sums of absolute per-vertex terms (scale for FP32 tolerances)."""
    sampler = sampler or dense_sampler(grid, vals64)
    pose = np.asarray(pose, dtype=np.float64)
    xb = Q.transform(pose, verts)
    term, phi, grad, act, _ = _terms(sampler, xb, k)
    w = np.where(act[:, None], k * np.where(act, phi, 0.0)[:, None] * grad, 0.0)
    return term.sum(), np.concatenate([np.abs(w).sum(0), np.abs(np.cross(xb, w)).sum(0)])


def rodrigues(axis_angle):
    """Rotation matrix exp([a]x) by the Rodrigues formula."""
    a = np.asarray(axis_angle, dtype=np.float64)
    th = np.linalg.norm(a)
    if th == 0.0:
        return np.eye(3)
    K = Q.skew(a / th)
    return np.eye(3) + np.sin(th) * K + (1.0 - np.cos(th)) * (K @ K)


def _perturb(xb, i, s):
    if i < 3:
        out = xb.copy()
        out[:, i] += s
        return out, np.tile(np.eye(3)[i], (len(xb), 1))
    e = np.zeros(3)
    e[i - 3] = 1.0
    Rr = rodrigues(s * e)
    return xb @ Rr.T, np.cross(e, xb)  # d x / d eps = e x x_B


def fd_twist(grid, verts, pose, k, h=1e-6, vals64=None, sampler=None, jumps=False):
    """Central differences of L_e over the 6 twist components.

    Returns (g_fd (6,), crossings (6,) int, bound (6,)).  ``crossings``
    counts vertices where the loss term is not smooth over the stencil:
      * the vertex is penetrating at +h or -h and sits in different cells
        there (the gradient jumps at a cell face): its share of the error is
        at most k |phi| |grad+ - grad-| |dx/d eps|;
      * the vertex enters or leaves the penetrating set within the stencil
        (0.5 k phi^2 is only C^1 at phi = 0, its second derivative jumps by
        k |grad . dx/d eps|^2): the central difference is then off by at
        most h k (|grad| |dx/d eps|)^2.
    ``bound`` is the sum of those shares.

    ``jumps``: the field may also jump in value across a cell face (the
    narrow-band sparse grid does, between a stored brick and one that is
    not); a vertex that changes cells then adds its whole difference
    quotient and its whole analytic term, |(t+ - t-)/2h| + |w . dx/d eps|,
    to the bound instead of the gradient-jump share.
    """
    sampler = sampler or dense_sampler(grid, vals64)
    xb = Q.transform(pose, verts)
    _, phi0, grad0, a0, _ = _terms(sampler, xb, k)
    w0 = np.where(a0[:, None], k * np.where(a0, phi0, 0.0)[:, None] * grad0, 0.0)
    g = np.zeros(6)
    cross = np.zeros(6, dtype=np.int64)
    bound = np.zeros(6)
    for i in range(6):
        xp, dx = _perturb(xb, i, +h)
        xm, _ = _perturb(xb, i, -h)
        tp, php, gp, ap, cp = _terms(sampler, xp, k)
        tm, phm, gm, am, cm = _terms(sampler, xm, k)
        g[i] = (tp.sum() - tm.sum()) / (2.0 * h)
        dxn = np.linalg.norm(dx, axis=1)
        moved = np.any(cp != cm, axis=1) & (ap | am)
        flips = (ap != am) | (ap != a0)
        cross[i] = int((moved | flips).sum())
        if moved.any() and jumps:
            fd_v = np.abs(tp[moved] - tm[moved]) / (2.0 * h)
            an_v = np.abs(np.sum(w0[moved] * dx[moved], axis=1))
            bound[i] += float(np.sum(fd_v + an_v))
        elif moved.any():
            phi_abs = np.maximum(np.abs(np.nan_to_num(php[moved])), np.abs(np.nan_to_num(phm[moved])))
            jump = np.linalg.norm(gp[moved] - gm[moved], axis=1)
            bound[i] += float(np.sum(k * phi_abs * jump * dxn[moved]))
        if flips.any():
            gmax = np.maximum(np.linalg.norm(gp[flips], axis=1), np.linalg.norm(gm[flips], axis=1))
            bound[i] += float(np.sum(h * k * (gmax * dxn[flips]) ** 2))
    return g, cross, bound


def fd_verts(grid, verts, pose, k, h=1e-6, vals64=None, sampler=None):
    """Central differences of L_e with respect to every vertex coordinate.

    Returns (g_fd (n,3), crossed (n,3) bool): a vertex coordinate is
    ``crossed`` when its term is not smooth over the stencil (the +-h
    evaluations sit in different cells, or the vertex enters or leaves the
    penetrating set).
    """
    sampler = sampler or dense_sampler(grid, vals64)
    pose = np.asarray(pose, dtype=np.float64)
    R = Q.rotation_from_quaternion(pose[:4])
    xb = Q.transform(pose, verts)
    _, _, _, a0, _ = _terms(sampler, xb, k)
    g = np.zeros((len(xb), 3))
    crossed = np.zeros((len(xb), 3), dtype=bool)
    for a in range(3):
        step = h * R[:, a]
        tp, _, _, ap, cp = _terms(sampler, xb + step, k)
        tm, _, _, am, cm = _terms(sampler, xb - step, k)
        g[:, a] = (tp - tm) / (2.0 * h)
        crossed[:, a] = (np.any(cp != cm, axis=1) & (ap | am)) | (ap != am) | (ap != a0)
    return g, crossed
