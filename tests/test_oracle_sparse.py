"""Pins of the sparse-grid oracle (CPU only): the brick classification
against an explicit per-brick enumeration, an infinite band reproducing the
dense interpolant, multilinear fields reproduced exactly by the coarse
interpolant, a sphere within the coarse interpolation bound away from its
band, the penalty adjoint on the sparse field (an infinite band gives the
dense adjoint; a half-space whose deep vertices take the coarse path gives
the closed-form loss and gradients; analytic against central differences),
and planted mistakes caught."""
import itertools

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import adjoint as A
from oracle import query as Q
from oracle import sparse as OS
from paper_2205_03532_amd import workloads as W
from test_oracle_pins import node_positions, sample_fp64


def classify_bruteforce(vals, band):
    """Every brick, every node, by loops."""
    nz, ny, nx = vals.shape
    bx, by, bz = OS.brick_counts((nx, ny, nz))
    out = np.zeros((bz, by, bx), dtype=bool)
    for k, j, i in itertools.product(range(bz), range(by), range(bx)):
        if 3 * i + 3 > nx - 1 or 3 * j + 3 > ny - 1 or 3 * k + 3 > nz - 1:
            out[k, j, i] = True
            continue
        vs = [vals[3 * k + c, 3 * j + b, 3 * i + a] for a in range(4) for b in range(4) for c in range(4)]
        out[k, j, i] = min(abs(v) for v in vs) <= band or (any(v < 0 for v in vs) and any(v >= 0 for v in vs))
    return out


def all_bricks(dims):
    bx, by, bz = OS.brick_counts(dims)
    k, j, i = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    return np.stack([i, j, k], -1).reshape(-1, 3), (bz, by, bx)


def sphere_grid(dims=(23, 20, 26), h=1e-3, r=6e-3):
    c = np.array([11e-3, 9.5e-3, 12.5e-3])
    return sample_fp64(lambda p: W.field_sphere(p, c, r), dims, (0.0, 0.0, 0.0), h), c, r


def test_classification_matches_enumeration():
    g, _, _ = sphere_grid()
    vals = Q.grid_values_f64(g.values, g.dtype)
    bricks, shape = all_bricks(g.dims)
    for band in (0.0, 1e-3, 2.5e-3, np.inf):
        got = OS.brick_stored(vals, np.float32(band), bricks).reshape(shape)
        ref = classify_bruteforce(vals, np.float32(band))
        assert np.array_equal(got, ref), band
    # a band of 0 keeps the surface bricks (mixed signs) and the partial ones, not more
    st0 = OS.brick_stored(vals, 0.0, bricks)
    assert 0 < st0.sum() < len(bricks)


def test_infinite_band_is_the_dense_interpolant():
    g, _, _ = sphere_grid()
    vals = Q.grid_values_f64(g.values, g.dtype)
    rng = np.random.default_rng(0)
    X = rng.uniform(-1e-3, 27e-3, (3000, 3))
    p1, g1, i1, st = OS.sample_sparse(vals, g.origin, g.h, g.dims, X, np.inf)
    p0, g0, i0, _ = Q.sample(vals, g.origin, g.h, g.dims, X)
    assert np.all(st) and np.array_equal(i0, i1)
    assert np.array_equal(p0[i0], p1[i1]) and np.array_equal(g0, g1)


@pytest.mark.parametrize("coef", [(0.3, -0.2, 0.5, 0.1, 0.0, 0.0, 0.0, 0.0),
                                  (0.0, 0.4, -0.3, 0.2, 30.0, -20.0, 15.0, 900.0)])
def test_multilinear_fields_are_exact_everywhere(coef):
    """A field in span{1, x, y, z, xy, yz, zx, xyz} is reproduced exactly by
    trilinear interpolation at any spacing, so the coarse and the dense
    interpolants agree with it and with each other."""
    c0, cx, cy, cz, cxy, cyz, czx, cxyz = coef
    o = np.array([-2e-3, 1e-3, 0.5e-3])

    def f(p):
        x, y, z = p[..., 0] - o[0], p[..., 1] - o[1], p[..., 2] - o[2]
        return c0 + cx * x + cy * y + cz * z + cxy * x * y + cyz * y * z + czx * z * x + cxyz * x * y * z

    def grad(p):
        x, y, z = p[..., 0] - o[0], p[..., 1] - o[1], p[..., 2] - o[2]
        return np.stack([cx + cxy * y + czx * z + cxyz * y * z, cy + cxy * x + cyz * z + cxyz * x * z,
                         cz + cyz * y + czx * x + cxyz * x * y], -1)

    dims, h = (17, 14, 20), 1e-3
    g = sample_fp64(f, dims, tuple(o), h)
    vals = g.values.astype(np.float64)  # exact samples would need FP64 storage: compare against the stored grid
    rng = np.random.default_rng(1)
    X = o + rng.uniform(0.0, h * (np.array(dims) - 1), (4000, 3))
    ps, gs, ins, st = OS.sample_sparse(vals, g.origin, g.h, g.dims, X, 0.0)
    assert np.all(ins) and (~st).sum() > 1000  # most points take the coarse path
    # the grid holds FP32 roundings of f: compare with the interpolant of those samples
    pd, gd, _, _ = Q.sample(vals, g.origin, g.h, g.dims, X)
    scale = np.max(np.abs(vals))
    assert np.max(np.abs(ps - pd)) <= 1e-6 * scale + 1e-12 or cxyz == 0.0 and cxy == 0.0
    if cxy == cyz == czx == cxyz == 0.0:  # affine: exact to rounding against the field
        assert np.max(np.abs(ps - f(X))) < 1e-7 * max(1.0, scale)
        assert np.max(np.abs(gs - grad(X))) < 1e-5
    # with FP64 samples the coarse and dense interpolants are the field itself
    vals64 = f(node_positions(dims, tuple(o), h))
    ps2, gs2, _, st2 = OS.sample_sparse(vals64, tuple(o), h, dims, X, 0.0)
    assert np.max(np.abs(ps2 - f(X))) < 1e-12 and np.max(np.abs(gs2 - grad(X))) < 1e-9
    assert (~st2).sum() > 1000


def test_sphere_within_coarse_bound_off_band():
    """Off the band the value is the coarse interpolant of the samples:
    within (3h)^2/8 * sum max|f_aa| (plus the FP32 sampling) of the sphere's
    SDF at a distance rho >= band from the surface, where |f_aa| <= 1/rho'."""
    g, c, r = sphere_grid(dims=(40, 40, 40), h=0.5e-3, r=4e-3)
    vals = Q.grid_values_f64(g.values, g.dtype)
    band = np.float32(1.5e-3)
    rng = np.random.default_rng(2)
    X = rng.uniform(0.0, 19.5e-3, (6000, 3))
    p, gr, ins, st = OS.sample_sparse(vals, g.origin, g.h, g.dims, X, band)
    off = ins & ~st
    assert off.sum() > 2000
    exact = W.field_sphere(X[off], c, r)
    rho = np.linalg.norm(X[off] - c, axis=1)
    # curvature of |x - c| is 1/rho; the coarse cell reaches 3h*sqrt(3) closer to c
    rmin = np.maximum(rho - 3 * g.h * np.sqrt(3), 1e-4)
    bound = (3 * g.h) ** 2 / 8 * 3 / rmin + 1e-7
    assert np.all(np.abs(p[off] - exact) <= bound)
    # each gradient component is a convex combination of difference quotients
    # of a 1-Lipschitz field over 3h, so at most 1 (plus the FP32 sampling)
    assert np.all(np.abs(gr[off]) <= 1.0 + 1e-5)
    away = rho > 2 * 3 * g.h * np.sqrt(3)  # cells clear of the centre, where the SDF has its kink
    assert np.all(np.linalg.norm(gr[off][away], axis=1) > 0.8) and away.sum() > 2000


# ------------------------------------------------------------ penalty adjoint on the sparse field


def _sampler(g, band):
    vals = Q.grid_values_f64(g.values, g.dtype)
    return OS.sparse_sampler(vals, g.origin, g.h, g.dims, band)


def test_sparse_penalty_infinite_band_is_the_dense_adjoint():
    """Every brick stored: loss, twist gradient, vertex gradients and the
    finite differences equal the dense oracle's, bit for bit."""
    w = W.torus_workload(n_env=4)
    g = w.grids[0]
    verts = w.meshes[0].verts
    sp = _sampler(g, np.inf)
    for e in range(w.n_env):
        L0, x0, v0 = A.penalty_env(g, verts, w.pose[:, e], 1e4)
        L1, x1, v1 = A.penalty_env(g, verts, w.pose[:, e], 1e4, sampler=sp)
        assert L0 == L1 and np.array_equal(x0, x1) and np.array_equal(v0, v1)
    f0 = A.fd_twist(g, verts, w.pose[:, 0], 1e4)
    f1 = A.fd_twist(g, verts, w.pose[:, 0], 1e4, sampler=sp)
    assert all(np.array_equal(a, b) for a, b in zip(f0, f1))


def test_sparse_penalty_halfspace_closed_form():
    """phi = n.x - d sampled in FP64 with a 1.5-voxel band: the bricks deep
    below the plane are not stored, yet the coarse interpolant of an affine
    field is the field, so the penalty and its gradients are the half-space's
    closed forms: L = sum 0.5 k phi^2, dL/drho = sum k phi n,
    dL/domega = sum x_B x (k phi n), dL/dv = R^T (k phi n)."""
    rng = np.random.default_rng(5)
    nrm = np.array([0.3, -0.2, 0.9])
    nrm /= np.linalg.norm(nrm)
    d, k, h = 0.004, 1e4, 1e-3
    g = sample_fp64(lambda p: p @ nrm - d, (31, 31, 31), (-0.015,) * 3, h)
    band = 1.5 * h
    dirs = rng.normal(size=(3000, 3))
    verts = (dirs / np.linalg.norm(dirs, axis=1)[:, None] * 0.0125 * rng.uniform(0, 1, (3000, 1)) ** (1 / 3))
    verts = verts.astype(np.float32)  # a ball that stays inside the grid under any rotation
    pose = np.r_[W.shoemake_quat(rng, 1)[:, 0], [0.001, -0.001, 0.0]].astype(np.float32)
    L, dxi, dv = A.penalty_env(g, verts, pose, k, sampler=_sampler(g, band))
    q = pose[:4].astype(np.float64)
    R = (q @ q) * Rotation.from_quat(q).as_matrix() + (1.0 - q @ q) * np.eye(3)
    xb = verts.astype(np.float64) @ R.T + pose[4:].astype(np.float64)
    phi = np.minimum(xb @ nrm - d, 0.0)
    wv = k * phi[:, None] * nrm[None, :]
    _, _, ins, stored = OS.sample_sparse(g.values, g.origin, g.h, g.dims, xb, band)
    assert np.all(ins) and ((phi < 0) & ~stored).sum() > 300  # many penetrating vertices take the coarse path
    scale = np.abs(wv).sum()
    assert abs(L - np.sum(0.5 * k * phi ** 2)) <= 1e-12 * max(L, 1e-30) + 1e-15
    assert np.allclose(dxi[:3], wv.sum(0), rtol=0, atol=1e-12 * scale)
    assert np.allclose(dxi[3:], np.cross(xb, wv).sum(0), rtol=0, atol=1e-12 * scale)
    assert np.allclose(dv, wv @ R, rtol=0, atol=1e-12 * np.abs(wv).max())


def test_sparse_penalty_matches_finite_differences():
    """A sphere with a 1.5-voxel band, vertices throughout the ball: the
    analytic twist and vertex gradients of the sparse field against its own
    central differences (h = 1e-7 m), within the kink bounds (the field jumps
    in value across a face between a stored brick and one that is not)."""
    g, c, r = sphere_grid(dims=(40, 40, 40), h=0.5e-3, r=7e-3)
    band = np.float32(0.75e-3)
    sp = _sampler(g, band)
    rng = np.random.default_rng(3)
    verts = (rng.uniform(-1, 1, (1500, 3)) * 6e-3).astype(np.float32)
    checked_coarse = 0
    for i in range(3):
        pose = np.r_[W.shoemake_quat(rng, 1)[:, 0], c + rng.uniform(-1e-3, 1e-3, 3)].astype(np.float32)
        L, dxi, dv = A.penalty_env(g, verts, pose, 1e4, sampler=sp)
        gfd, cross, bound = A.fd_twist(g, verts, pose, 1e4, 1e-7, sampler=sp, jumps=True)
        scale = max(np.max(np.abs(gfd)), 1e-12)
        for j in range(6):
            assert abs(dxi[j] - gfd[j]) <= 1e-5 * scale + 1e-9 + bound[j], (i, j, dxi[j], gfd[j], cross[j])
        gv, crossed = A.fd_verts(g, verts, pose, 1e4, 1e-7, sampler=sp)
        ok = ~crossed
        assert np.allclose(dv[ok], gv[ok], rtol=1e-4, atol=1e-8 * scale)
        xb = Q.transform(pose, verts)
        _, _, ins, st = OS.sample_sparse(Q.grid_values_f64(g.values, g.dtype), g.origin, g.h, g.dims, xb, band)
        checked_coarse += int((ins & ~st & np.all(ok, axis=1)).sum())
    assert checked_coarse > 1000


# ------------------------------------------------------------ planted mistakes

SPARSE_PINS = [test_classification_matches_enumeration, test_infinite_band_is_the_dense_interpolant,
               test_sphere_within_coarse_bound_off_band, test_sparse_penalty_halfspace_closed_form,
               test_sparse_penalty_matches_finite_differences,
               lambda: test_multilinear_fields_are_exact_everywhere((0.3, -0.2, 0.5, 0.1, 0.0, 0.0, 0.0, 0.0))]


def _some_pin_fails():
    for pin in SPARSE_PINS:
        try:
            pin()
        except Exception:
            return True
    return False


def test_planted_sparse_mistakes_are_caught(monkeypatch):
    assert not _some_pin_fails()
    orig_stored = OS.brick_stored

    def no_mixed(vals64, band, bricks):  # forgets the both-signs rule
        b = np.asarray(bricks, dtype=np.int64).reshape(-1, 3)
        nz, ny, nx = vals64.shape
        partial = np.any(3 * b + 3 > np.array([nx, ny, nz]) - 1, axis=1)
        k = np.arange(4)
        x = np.minimum(3 * b[:, 0, None] + k, nx - 1)
        y = np.minimum(3 * b[:, 1, None] + k, ny - 1)
        z = np.minimum(3 * b[:, 2, None] + k, nz - 1)
        blk = vals64[z[:, :, None, None], y[:, None, :, None], x[:, None, None, :]].reshape(len(b), -1)
        return partial | (np.min(np.abs(blk), axis=1) <= band)

    monkeypatch.setattr(OS, "brick_stored", no_mixed)
    assert _some_pin_fails(), "no_mixed"
    monkeypatch.setattr(OS, "brick_stored", orig_stored)

    orig_coarse = OS.coarse_interpolant

    def coarse_t_unscaled(vals64, cell, t, h):  # local coordinates not divided by 3
        b = cell // 3
        coarse = vals64[::3, ::3, ::3]
        cz, cy, cx = coarse.shape
        bc = np.maximum(np.minimum(b, np.array([cx - 2, cy - 2, cz - 2])), 0)
        tc = np.clip((cell + t) - 3.0 * bc, 0.0, 1.0)
        return Q.trilinear_value_grad(coarse, bc, tc, 3.0 * h)

    def coarse_grad_fine_spacing(vals64, cell, t, h):  # gradient per h instead of per 3h
        p, g = orig_coarse(vals64, cell, t, h)
        return p, 3.0 * g

    for name, fn in (("coarse_t_unscaled", coarse_t_unscaled), ("coarse_grad_fine_spacing", coarse_grad_fine_spacing)):
        monkeypatch.setattr(OS, "coarse_interpolant", fn)
        assert _some_pin_fails(), name
        monkeypatch.setattr(OS, "coarse_interpolant", orig_coarse)
