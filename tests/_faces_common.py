"""Branches of the per-face descent (test infrastructure).

The descent's accept test compares two phi values; an FP32 run and the FP64
oracle can decide it differently only where the two values lie within the
FP32 evaluation error of each other, or where a trial point lies within the
FP32 position error of the grid's boundary (inside on one side, outside, so
+infinity, on the other).  ``descent_leaves`` re-runs the oracle's descent of
one face in FP64 and, at every such decision, follows both outcomes; its
leaves are every end state a correct FP32 run can reach.  A GPU face whose
result differs from the FP64 descent must end at one of them.
"""
import numpy as np

from oracle import faces as OF
from oracle import query as OQ

ULP32 = 2.0 ** -23


def decision_tolerance(X, origin, h, dims):
    """Largest difference between the phi an FP32 run and the FP64 descent
    compare at the same decision, on the same branch: the FP32 trial point
    is off by a few roundings of the coordinates (corners R v + t, the
    barycentric combination, u = (x - o) / h), i.e. about 8 ulp of the
    largest coordinate L; phi moves by at most |grad phi| <= 1.5 per unit
    of that; sampling rounding is far smaller.  Taken with a factor 3."""
    far = np.abs(np.asarray(origin, np.float64)) + h * (np.asarray(dims, np.float64) - 1.0)
    L = max(float(np.max(np.abs(X))), float(np.max(far)))
    return 3.0 * 8.0 * ULP32 * L * 1.5


def point_tolerance(X, origin, h, dims):
    """Largest distance between the end point of an FP32 run and that of the
    FP64 descent on the same branch: the FP32 point carries the rounding of
    its corners (R v + t) and of the barycentric combination, a few ulp of
    the largest coordinate L each; 8 ulp of L, taken with a factor 3 as in
    decision_tolerance."""
    far = np.abs(np.asarray(origin, np.float64)) + h * (np.asarray(dims, np.float64) - 1.0)
    L = max(float(np.max(np.abs(X))), float(np.max(far)))
    return 3.0 * 8.0 * ULP32 * L


def _sample(vals, origin, h, dims, x, band):
    """phi (+inf outside), grad, and a flag for points within ``band`` voxels
    of the grid's boundary, where an FP32 run may call the point inside (with
    the field at the nearest boundary point) or outside."""
    n = np.asarray(dims, np.float64)
    u = (x - np.asarray(origin, np.float64)) / h
    near = np.any((np.abs(u) <= band) | (np.abs(u - (n - 1.0)) <= band), axis=-1)
    phi, g, inside, _ = OQ.sample(vals, origin, h, dims, x)
    phi = np.where(inside, phi, np.inf)
    xc = np.asarray(origin, np.float64) + h * np.clip(u, 0.0, n - 1.0)
    pc, gc, _, _ = OQ.sample(vals, origin, h, dims, xc)
    return phi, g, near, pc, gc


def alt_grads(vals, origin, h, dims, x, band):
    """The other gradients an FP32 run may take at the inside point x: within
    ``band`` voxels of an interior cell face it may place x in the cell on
    the other side, where the interpolant has the same value (it is
    continuous) but another gradient.  One per combination of such faces."""
    n = np.asarray(dims, np.int64)
    u = (np.asarray(x, np.float64) - np.asarray(origin, np.float64)) / h
    cell = np.clip(np.floor(u), 0, n - 2).astype(np.int64)
    t = u - cell
    opts = []
    for ax in range(3):
        o = [0]
        if t[ax] < band and cell[ax] > 0:
            o.append(-1)
        if t[ax] > 1.0 - band and cell[ax] < n[ax] - 2:
            o.append(1)
        opts.append(o)
    out = []
    for sx in opts[0]:
        for sy in opts[1]:
            for sz in opts[2]:
                if sx == 0 and sy == 0 and sz == 0:
                    continue
                c2 = cell + np.array([sx, sy, sz])
                _, g2 = OQ.trilinear_value_grad(vals, c2[None], (u - c2)[None], h)
                out.append(g2[0])
    return out


def descent_leaves(vals, origin, h, dims, X, iters, step0, tau, band=1e-4, face_band=None):
    """End states (x (m, 3), phi (m,)) of the FP64 descent of one face
    (corners X (3, 3) in B's frame) over every branch of its ambiguous
    decisions; phi is +inf for an end point outside the grid.  An accepted
    point within ``face_band`` voxels of a cell face (default: the position
    error bound of point_tolerance) also branches on the gradient of each
    cell it may be placed in, which steers the next trial."""
    if face_band is None:
        face_band = max(band, point_tolerance(X, origin, h, dims) / h)
    X = np.asarray(X, np.float64)
    xa, e1, e2 = X[0], X[1] - X[0], X[2] - X[0]
    S = (e1 @ e1 + e2 @ e2 + (e2 - e1) @ (e2 - e1)) / 3.0
    a0 = step0 / np.sqrt(S) if S > 0.0 else 0.0

    def point(b):
        return xa + b[:, 1:2] * e1 + b[:, 2:3] * e2

    b = np.full((1, 3), 1.0 / 3.0)
    x = point(b)
    phi, g, near, pc, gc = _sample(vals, origin, h, dims, x, band)
    alpha = np.array([a0])
    if near[0]:  # the start itself may be taken as inside or outside
        b = np.repeat(b, 2, 0)
        x = np.repeat(x, 2, 0)
        alt_phi = pc if not np.isfinite(phi[0]) else np.array([np.inf])
        alt_g = gc if not np.isfinite(phi[0]) else np.zeros((1, 3))
        phi = np.concatenate([phi, alt_phi])
        g = np.concatenate([g, alt_g])
        alpha = np.repeat(alpha, 2)

    def with_cell_gradients(rows, b, x, phi, g, alpha):
        """Adds, for each listed state, copies with the other cells' gradients."""
        extra = [(b[i], x[i], phi[i], ga, alpha[i]) for i in rows if np.isfinite(phi[i])
                 for ga in alt_grads(vals, origin, h, dims, x[i], face_band)]
        if not extra:
            return b, x, phi, g, alpha
        eb, ex, ep, eg, ea = (np.asarray(v) for v in zip(*extra))
        return (np.concatenate([b, eb]), np.concatenate([x, ex]), np.concatenate([phi, ep]),
                np.concatenate([g, eg]), np.concatenate([alpha, ea]))

    b, x, phi, g, alpha = with_cell_gradients(range(len(b)), b, x, phi, g, alpha)
    for _ in range(iters):
        d = np.stack([np.zeros(len(b)), g @ e1, g @ e2], axis=1)
        bt = OF.trial_point(b, alpha, d)
        xt = point(bt)
        pt, gt, nt, pct, gct = _sample(vals, origin, h, dims, xt, band)
        # the trial's phi as an FP32 run may see it: its own, or across the boundary
        alt = np.where(np.isfinite(pt), np.inf, pct)
        alt_g = np.where(np.isfinite(pt)[:, None], 0.0, gct)
        rows_b, rows_acc, rows_pt, rows_gt = [], [], [], []
        for i in range(len(b)):
            opts = [(pt[i], gt[i])]
            if nt[i]:
                opts.append((alt[i], alt_g[i]))
            seen = set()
            for p_i, g_i in opts:
                if np.isinf(p_i) and np.isinf(phi[i]):
                    decs = (False,)
                elif p_i < phi[i] - tau:
                    decs = (True,)
                elif p_i > phi[i] + tau:
                    decs = (False,)
                else:
                    decs = (True, False)
                for acc in decs:
                    key = (acc, float(p_i) if acc else None)
                    if key in seen:
                        continue
                    seen.add(key)
                    rows_b.append(i)
                    rows_acc.append(acc)
                    rows_pt.append(p_i)
                    rows_gt.append(g_i)
        idx = np.asarray(rows_b)
        acc = np.asarray(rows_acc)
        b = np.where(acc[:, None], bt[idx], b[idx])
        x = np.where(acc[:, None], xt[idx], x[idx])
        phi = np.where(acc, np.asarray(rows_pt), phi[idx])
        g = np.where(acc[:, None], np.asarray(rows_gt), g[idx])
        alpha = np.where(acc, 2.0 * alpha[idx], 0.5 * alpha[idx])
        b, x, phi, g, alpha = with_cell_gradients(np.nonzero(acc)[0], b, x, phi, g, alpha)
        if len(b) > 4096:
            raise RuntimeError("too many ambiguous decisions on one face")
    return x, phi


def matches_a_leaf(gx, gphi, leaves_x, leaves_phi, phi_tol, x_tol):
    """Whether the GPU's end state (point gx, phi gphi; inf outside) is one
    of the leaves: both outside, or phi within phi_tol and the point within
    x_tol."""
    if not np.isfinite(gphi):
        return bool(np.any(~np.isfinite(leaves_phi)))
    fin = np.isfinite(leaves_phi)
    ok = fin & (np.abs(leaves_phi - gphi) <= phi_tol) & (np.linalg.norm(leaves_x - gx, axis=1) <= x_tol)
    return bool(ok.any())
