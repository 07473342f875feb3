"""The branch explorer of the per-face descent (tests/_faces_common.py),
pinned on the CPU: the FP64 descent's own end state is always a leaf; a run
that takes the other side of an ambiguous decision ends at a leaf; a run that
takes the other side of a clear decision does not."""
import numpy as np

from _faces_common import descent_leaves, matches_a_leaf
from oracle import faces as OF
from oracle import query as OQ
from paper_2205_03532_amd import workloads as W

ITERS, STEP0 = 8, 0.5


def forced_descent(vals, g0, X, iters, step0, flip):
    """The FP64 descent of one face with the decisions at the listed
    iterations inverted; also returns each decision's |phi_trial - phi|."""
    X = np.asarray(X, np.float64)
    xa, e1, e2 = X[0], X[1] - X[0], X[2] - X[0]
    S = (e1 @ e1 + e2 @ e2 + (e2 - e1) @ (e2 - e1)) / 3.0
    alpha = step0 / np.sqrt(S)
    b = np.full((1, 3), 1.0 / 3.0)
    x = xa + b[:, 1:2] * e1 + b[:, 2:3] * e2
    phi, g, ins, _ = OQ.sample(vals, g0.origin, g0.h, g0.dims, x)
    phi = np.where(ins, phi, np.inf)
    gaps = []
    for it in range(iters):
        d = np.stack([np.zeros(1), g @ e1, g @ e2], axis=1)
        bt = OF.trial_point(b, np.array([alpha]), d)
        xt = xa + bt[:, 1:2] * e1 + bt[:, 2:3] * e2
        pt, gt, it_in, _ = OQ.sample(vals, g0.origin, g0.h, g0.dims, xt)
        pt = np.where(it_in, pt, np.inf)
        gaps.append(abs(float(pt[0] - phi[0])) if np.isfinite(pt[0]) and np.isfinite(phi[0]) else np.inf)
        acc = bool(OF.accept(pt, phi)[0]) != (it in flip)
        if acc:
            b, x, phi, g = bt, xt, pt, gt
            alpha *= 2.0
        else:
            alpha *= 0.5
    return x[0], float(phi[0]), gaps


def faces_of_torus(n_faces=40):
    w = W.subset(W.torus_workload(), range(2))
    g0 = w.grids[0]
    vals = OQ.grid_values_f64(g0.values, g0.dtype)
    m = w.meshes[0]
    X = OF.face_corners(w.pose[:, 0], m.verts, m.tris)
    rng = np.random.default_rng(5)
    return g0, vals, X[rng.choice(len(X), n_faces, replace=False)]


def test_fp64_descent_is_a_leaf():
    g0, vals, X = faces_of_torus()
    r_b, r_x, r_phi, _, _ = OF.pgd_faces(vals, g0.origin, g0.h, g0.dims, X, ITERS, STEP0)
    for f in range(len(X)):
        lx, lp = descent_leaves(vals, g0.origin, g0.h, g0.dims, X[f], ITERS, STEP0, tau=1e-7)
        assert matches_a_leaf(r_x[f], r_phi[f], lx, lp, 1e-12, 1e-12), f


def test_flipped_ambiguous_decision_is_a_leaf_and_a_clear_one_is_not():
    """With a wide tolerance tau every decision whose gap is below it is
    ambiguous: flipping one of those ends at a leaf; flipping a decision with
    a gap well above tau ends elsewhere (whenever the end state changes)."""
    g0, vals, X = faces_of_torus()
    tau = 2e-5
    n_amb = n_clear = 0
    for f in range(len(X)):
        _, _, gaps = forced_descent(vals, g0, X[f], ITERS, STEP0, set())
        lx, lp = descent_leaves(vals, g0.origin, g0.h, g0.dims, X[f], ITERS, STEP0, tau=tau)
        for it, gap in enumerate(gaps):
            if gap <= 0.5 * tau:
                x, p, _ = forced_descent(vals, g0, X[f], ITERS, STEP0, {it})
                assert matches_a_leaf(x, p, lx, lp, 1e-12, 1e-12), (f, it)
                n_amb += 1
            elif gap >= 4 * tau and np.isfinite(gap):
                x0, p0, _ = forced_descent(vals, g0, X[f], ITERS, STEP0, set())
                x, p, _ = forced_descent(vals, g0, X[f], ITERS, STEP0, {it})
                if abs(p - p0) > 1e-9:
                    assert not matches_a_leaf(x, p, lx, lp, 1e-12, 1e-12), (f, it)
                    n_clear += 1
    assert n_amb > 0 and n_clear > 0, (n_amb, n_clear)


def descent_from(vals, g0, X, iters, step0, g_start):
    """The FP64 descent of one face started with the given gradient at the
    centroid instead of the one its own cell gives."""
    X = np.asarray(X, np.float64)
    xa, e1, e2 = X[0], X[1] - X[0], X[2] - X[0]
    S = (e1 @ e1 + e2 @ e2 + (e2 - e1) @ (e2 - e1)) / 3.0
    alpha = step0 / np.sqrt(S)
    b = np.full((1, 3), 1.0 / 3.0)
    x = xa + b[:, 1:2] * e1 + b[:, 2:3] * e2
    phi, _, _, _ = OQ.sample(vals, g0.origin, g0.h, g0.dims, x)
    g = np.asarray(g_start, np.float64)[None]
    for _ in range(iters):
        d = np.stack([np.zeros(1), g @ e1, g @ e2], axis=1)
        bt = OF.trial_point(b, np.array([alpha]), d)
        xt = xa + bt[:, 1:2] * e1 + bt[:, 2:3] * e2
        pt, gt, it_in, _ = OQ.sample(vals, g0.origin, g0.h, g0.dims, xt)
        pt = np.where(it_in, pt, np.inf)
        if OF.accept(pt, phi)[0]:
            b, x, phi, g = bt, xt, pt, gt
            alpha *= 2.0
        else:
            alpha *= 0.5
    return x[0], float(phi[0])


def test_gradient_of_the_neighbouring_cell_is_a_branch():
    """A face whose centroid lies on a cell face (z = a node plane): an FP32
    run may place it in either cell and step along either cell's gradient,
    so both descents end at leaves; a descent steered by the gradient of a
    cell two planes away (no FP32 run can take it) ends elsewhere."""
    w = W.subset(W.torus_workload(), range(1))
    g0 = w.grids[0]
    vals = OQ.grid_values_f64(g0.values, g0.dtype)
    o, h = np.asarray(g0.origin, np.float64), float(g0.h)
    # a triangle about two voxels across, centred on node plane k = 34 inside the tube
    c = np.array([0.021887, 0.002337, o[2] + 34 * h])
    X = c + 1.98 * h * np.array([[-0.0701, 0.6516, -1.5858], [0.6598, 0.5041, 0.4546], [-0.5897, -1.1557, 1.1313]])
    X -= X.mean(0) - c
    u = (X.mean(0) - o) / h
    assert abs(u[2] - 34.0) < 1e-9
    lx, lp = descent_leaves(vals, g0.origin, g0.h, g0.dims, X, ITERS, STEP0, tau=1e-9)
    cell = np.floor(u).astype(np.int64)
    ends = []
    grads = {}
    for cz in (33, 34, 35):
        c2 = np.array([cell[0], cell[1], cz])
        _, gr = OQ.trilinear_value_grad(vals, c2[None], (u - c2)[None], h)
        grads[cz] = gr[0]
    assert np.linalg.norm(grads[33] - grads[34]) > 1e-3  # the gradient does jump at the plane
    for cz in (33, 34):
        x, p = descent_from(vals, g0, X, ITERS, STEP0, grads[cz])
        assert matches_a_leaf(x, p, lx, lp, 1e-12, 1e-12), cz
        ends.append((x, p))
    assert np.linalg.norm(ends[0][0] - ends[1][0]) > 1e-6  # the two sides do end apart
    x, p = descent_from(vals, g0, X, ITERS, STEP0, grads[35])
    assert min(np.linalg.norm(x - e[0]) for e in ends) > 1e-6
    assert not matches_a_leaf(x, p, lx, lp, 1e-12, 1e-12)
