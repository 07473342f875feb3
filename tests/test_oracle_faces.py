"""Pins of the per-face oracle (projected gradient descent over each face) to
facts outside itself (CPU only): the simplex projection against an exhaustive
active-set search, affine fields whose minimum over a face sits at a corner,
a sampled sphere whose minimum over a face is the point-to-triangle distance
(Ericson's closest point) minus the radius, and the invariants of the descent
(never above the start, always on the face)."""
import itertools

import numpy as np
import pytest

from oracle import faces as OF
from oracle import meshdist as MD
from oracle import query as Q
from paper_2205_03532_amd import workloads as W
from test_oracle_pins import node_positions, sample_fp64


def simplex_bruteforce(y):
    """Nearest point of the simplex: try every face of it (each subset of
    coordinates left free, the rest zero), keep the feasible projections onto
    that face's affine hull, take the nearest."""
    best, bd = None, np.inf
    for k in range(1, 4):
        for free in itertools.combinations(range(3), k):
            x = np.zeros(3)
            f = list(free)
            x[f] = y[f] - (y[f].sum() - 1.0) / k
            if np.all(x >= -1e-15):
                d = np.sum((x - y) ** 2)
                if d < bd:
                    best, bd = np.maximum(x, 0.0), d
    return best


def test_project_simplex_matches_active_set_search():
    rng = np.random.default_rng(0)
    y = np.concatenate([rng.normal(0.3, 1.0, (400, 3)), rng.normal(0.0, 20.0, (100, 3)),
                        rng.dirichlet((1, 1, 1), 50)])  # the last rows already lie in the simplex
    p = OF.project_simplex(y)
    ref = np.array([simplex_bruteforce(r) for r in y])
    assert np.max(np.abs(p - ref)) < 1e-12
    assert np.allclose(p.sum(1), 1.0) and np.all(p >= 0)
    assert np.allclose(p[-50:], y[-50:], atol=1e-15)


def random_faces(rng, n, centre, spread, size):
    c = centre + rng.uniform(-spread, spread, (n, 1, 3))
    return c + rng.normal(0.0, size, (n, 3, 3))


def test_affine_field_minimum_is_reached_at_the_lowest_corner():
    """phi = a.x + c is reproduced exactly by trilinear interpolation, so its
    minimum over a face is the corner with the lowest value; the descent lands
    exactly there (the projection maps overshoots onto the corner)."""
    rng = np.random.default_rng(1)
    a = np.array([0.3, -0.5, 0.81])
    a /= np.linalg.norm(a)
    g = sample_fp64(lambda p: p @ a - 0.01, (24, 24, 24), (0.0, 0.0, 0.0), 1e-3)
    vals = Q.grid_values_f64(g.values, g.dtype)
    X = random_faces(rng, 2000, np.full(3, 0.0115), 0.004, 0.002)
    b, x, phi, grad, phi0 = OF.pgd_faces(vals, g.origin, g.h, g.dims, X, 16, 0.5)
    corner = X @ a - 0.01
    lo = np.sort(corner, axis=1)
    clear = (lo[:, 1] - lo[:, 0]) > 1e-6  # a unique lowest corner
    hit = np.abs(phi - lo[:, 0]) < 1e-12
    assert clear.sum() > 1500
    assert hit[clear].mean() > 0.99, hit[clear].mean()
    assert np.all(phi <= phi0)
    assert np.all(phi >= lo[:, 0] - 1e-12)  # never below the true minimum over the face


def test_sphere_minimum_is_point_to_triangle_distance():
    """phi = |x - c| - r sampled at h = 1 mm: the minimum over a face is
    dist(c, face) - r, within the interpolation bound h^2/(4 rho) (rho the
    distance to c) and the descent's stopping slack."""
    rng = np.random.default_rng(2)
    c = np.array([0.016, 0.016, 0.016])
    r = 0.010
    g = sample_fp64(lambda p: W.field_sphere(p, c, r), (33, 33, 33), (0.0, 0.0, 0.0), 1e-3)
    vals = Q.grid_values_f64(g.values, g.dtype)
    # faces near the sphere surface: centres at radius r +- 1 mm, size ~1.5 mm
    dirs = rng.normal(size=(500, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    centres = c + dirs * (r + rng.uniform(-1e-3, 1e-3, (500, 1)))
    X = centres[:, None, :] + rng.normal(0.0, 1.5e-3, (500, 3, 3))
    b, x, phi, grad, phi0 = OF.pgd_faces(vals, g.origin, g.h, g.dims, X, 40, 0.5)
    exact = np.array([np.linalg.norm(MD._closest_on_triangle(c, *f)[0] - c) for f in X]) - r
    rho = np.maximum(exact + r - 2e-3, 1e-3)
    bound = (1e-3) ** 2 / (4 * rho) + 2e-6
    err = phi - exact
    assert np.all(np.abs(err) <= bound), np.max(np.abs(err) / bound)
    assert np.all(phi <= phi0)
    assert np.all(np.abs(b.sum(1) - 1) < 1e-12) and np.all(b >= 0)
    assert np.allclose(np.einsum("fi,fij->fj", b, X), x, atol=1e-15)


def test_degenerate_and_outside_faces():
    g = sample_fp64(lambda p: p[..., 2] - 0.005, (12, 12, 12), (0.0, 0.0, 0.0), 1e-3)
    vals = Q.grid_values_f64(g.values, g.dtype)
    X = np.array([
        [[0.004, 0.004, 0.003]] * 3,  # all corners equal
        [[0.02, 0.02, 0.02], [0.021, 0.02, 0.02], [0.02, 0.021, 0.02]],  # outside the grid
        [[0.002, 0.002, 0.002], [0.004, 0.002, 0.006], [0.002, 0.004, 0.004]],
    ])
    b, x, phi, grad, phi0 = OF.pgd_faces(vals, g.origin, g.h, g.dims, X, 8, 0.5)
    assert np.allclose(x[0], X[0, 0]) and abs(phi[0] - (0.003 - 0.005)) < 1e-15
    assert np.isinf(phi[1]) and np.all(grad[1] == 0)
    assert abs(phi[2] - (0.002 - 0.005)) < 1e-15 and np.allclose(b[2], [1, 0, 0])


def test_faces_workload_columns_and_record():
    """Per-face records of a small torus batch: candidates are inside with
    phi < margin, normals unit or zero, bins the lowest argmax, and each face's
    point is the barycentric combination of its corners."""
    w = W.subset(W.torus_workload(), range(3))
    r = OF.query_faces_workload(w, 8, 0.5)
    F = len(w.meshes[0].tris)
    assert len(r["phi"]) == 3 * F and np.array_equal(r["fidx"][:F], np.arange(F))
    assert np.all(r["cand"] == (np.isfinite(r["phi"]) & (r["phi"] < 0)))
    nn = np.linalg.norm(r["normal"], axis=1)
    assert np.all((np.abs(nn - 1) < 1e-12) | (nn == 0))
    assert np.allclose(np.einsum("fi,fij->fj", r["bary"], r["corners"]), r["x_b"], atol=1e-15)
    assert r["cand"].sum() > 100


def test_zero_iterations_is_the_centroid():
    rng = np.random.default_rng(3)
    g = sample_fp64(lambda p: p[..., 0] - 0.004, (12, 12, 12), (0.0, 0.0, 0.0), 1e-3)
    vals = Q.grid_values_f64(g.values, g.dtype)
    X = random_faces(rng, 20, np.full(3, 0.005), 0.002, 0.001)
    b, x, phi, grad, phi0 = OF.pgd_faces(vals, g.origin, g.h, g.dims, X, 0, 0.5)
    assert np.allclose(b, 1.0 / 3.0) and np.allclose(x, X.mean(1), atol=1e-15) and np.array_equal(phi, phi0)


# ------------------------------------------------------------ planted mistakes

FACE_PINS = [test_project_simplex_matches_active_set_search, test_affine_field_minimum_is_reached_at_the_lowest_corner,
             test_sphere_minimum_is_point_to_triangle_distance, test_degenerate_and_outside_faces,
             test_zero_iterations_is_the_centroid]


def _some_face_pin_fails():
    for pin in FACE_PINS:
        try:
            pin()
        except Exception:  # an assertion or a crash: caught
            return True
    return False


def _clip_renormalise(y):
    c = np.maximum(np.asarray(y, dtype=np.float64), 0.0)
    s = c.sum(1, keepdims=True)
    return np.where(s > 0, c / np.where(s > 0, s, 1.0), 1.0 / 3.0)


@pytest.mark.parametrize("name,fn", [
    ("project_simplex", _clip_renormalise),
    ("trial_point", lambda b, alpha, d: OF.project_simplex(b + alpha[:, None] * d)),  # ascent
    ("accept", lambda pt, phi: pt <= phi + 1e-3),  # keeps worse trials
])
def test_planted_face_mistake_is_caught(monkeypatch, name, fn):
    assert not _some_face_pin_fails()
    monkeypatch.setattr(OF, name, fn)
    assert _some_face_pin_fails(), name
