"""Pins of the CPU oracle to facts outside itself (CPU only).

Each test checks the oracle against something the mathematics or an
independent routine fixes: a library rotation, fields that trilinear
interpolation reproduces exactly, closed-form SDFs within the interpolation
error bound, brute-force mesh distances, a half-space whose contacts,
normals, bins and penalty gradients have closed forms, and an exhaustive
reduction.  A dropped term, a sign flip, a transposed axis or a wrong cell
choice in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import adjoint as A
from oracle import meshdist as MD
from oracle import query as Q
from oracle import reduce as RD
from paper_2205_03532_amd import workloads as W


class G:  # minimal grid record for FP64 test fields
    def __init__(self, values, dtype, origin, h):
        self.values, self.dtype, self.origin, self.h = values, dtype, origin, h

    @property
    def dims(self):
        nz, ny, nx = self.values.shape
        return (nx, ny, nz)


def node_positions(dims, origin, h):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([origin[0] + h * x, origin[1] + h * y, origin[2] + h * z], -1)


def sample_fp64(fn, dims, origin, h):
    return G(fn(node_positions(dims, origin, h)), "f64", origin, h)


def rot_unnormalised(q):
    """Rotation the pose reading applies to a float32 quaternion of norm s != 1.

    I + 2w[v]x + 2[v]x^2 is quadratic in q, so for q = s q_hat it equals
    s^2 R(q_hat) + (1 - s^2) I; R(q_hat) comes from scipy.
    """
    q = np.asarray(q, dtype=np.float64)
    s2 = float(q @ q)
    return s2 * Rotation.from_quat(q).as_matrix() + (1.0 - s2) * np.eye(3)


# ---------------------------------------------------------------- rotation


def test_rotation_matches_scipy():
    rng = np.random.default_rng(0)
    q = W.shoemake_quat(rng, 50).T
    for qi in q:
        R = Q.rotation_from_quaternion(qi)
        Rs = Rotation.from_quat(qi).as_matrix()  # scalar-last (x, y, z, w)
        assert np.allclose(R, Rs, atol=1e-14)


def test_rotation_not_renormalised():
    q = np.array([0.1, -0.2, 0.3, 0.9]) * 1.01
    assert np.allclose(Q.rotation_from_quaternion(q), rot_unnormalised(q), atol=1e-14)


def test_rotation_quarter_turn_about_z():
    q = (0.0, 0.0, math.sin(math.pi / 4), math.cos(math.pi / 4))
    R = Q.rotation_from_quaternion(q)
    assert np.allclose(R @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    assert np.allclose(R @ [0, 1, 0], [-1, 0, 0], atol=1e-15)
    assert np.allclose(R @ [0, 0, 1], [0, 0, 1], atol=1e-15)


def test_transform_identity_and_translation_exact():
    rng = np.random.default_rng(1)
    v = (rng.integers(-512, 512, (100, 3)) / 1024.0).astype(np.float32)
    ident = np.array([0, 0, 0, 1, 0, 0, 0], np.float32)
    assert np.array_equal(Q.transform(ident, v), v.astype(np.float64))
    pose = np.array([0, 0, 0, 1, 0.25, -0.125, 0.5], np.float32)
    assert np.array_equal(Q.transform(pose, v), v.astype(np.float64) + [0.25, -0.125, 0.5])


def test_rigid_equivariance():
    rng = np.random.default_rng(2)
    v = rng.normal(size=(40, 3))
    qa = W.shoemake_quat(rng, 1)[:, 0]
    qs = W.shoemake_quat(rng, 1)[:, 0]
    S = Q.rotation_from_quaternion(qs)
    Ra = Q.rotation_from_quaternion(qa)
    t = rng.normal(size=3)
    # rotating the mesh by S and using pose Ra S^T gives the same points
    comp = Rotation.from_matrix(Ra @ S.T).as_quat()
    x1 = Q.transform(np.r_[qa, t], v)
    x2 = Q.transform(np.r_[comp, t], v @ S.T)
    assert np.allclose(x1, x2, atol=1e-13)


# ---------------------------------------------------------------- trilinear


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_trilinear_reproduces_q1_fields(seed):
    """span{1,x,y,z,xy,yz,zx,xyz} is reproduced exactly, value and gradient."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=8)
    dims = (5, 6, 7)
    origin = tuple(rng.normal(size=3))
    h = 0.37

    def f(p):
        x, y, z = p[..., 0], p[..., 1], p[..., 2]
        return a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * y + a[5] * y * z + a[6] * z * x + a[7] * x * y * z

    def grad(p):
        x, y, z = p[..., 0], p[..., 1], p[..., 2]
        return np.stack([a[1] + a[4] * y + a[6] * z + a[7] * y * z,
                         a[2] + a[4] * x + a[5] * z + a[7] * x * z,
                         a[3] + a[5] * y + a[6] * x + a[7] * x * y], -1)

    g = sample_fp64(f, dims, origin, h)
    lo = np.asarray(origin)
    hi = lo + h * (np.asarray(dims) - 1)
    x = lo + rng.random((500, 3)) * (hi - lo)
    phi, gr, inside, _ = Q.sample(g.values, g.origin, g.h, g.dims, x)
    assert inside.all()
    assert np.allclose(phi, f(x), rtol=0, atol=1e-11)
    assert np.allclose(gr, grad(x), rtol=0, atol=1e-10)


def test_node_reproduction_and_far_boundary():
    rng = np.random.default_rng(3)
    vals = rng.normal(size=(4, 5, 6)).astype(np.float32)
    g = G(vals, "f32", (0.5, -1.0, 2.0), 0.25)
    P = node_positions(g.dims, g.origin, g.h).reshape(-1, 3)
    phi, _, inside, cell = Q.sample(Q.grid_values_f64(vals, "f32"), g.origin, g.h, g.dims, P)
    assert inside.all()
    assert np.array_equal(phi, vals.reshape(-1).astype(np.float64))
    # the far corner node uses the last cell (cell index n - 2)
    far = np.asarray(g.origin) + g.h * (np.asarray(g.dims) - 1)
    _, _, _, c = Q.sample(Q.grid_values_f64(vals, "f32"), g.origin, g.h, g.dims, far[None])
    assert tuple(c[0]) == tuple(np.asarray(g.dims) - 2)


def test_outside_points_are_not_inside():
    vals = np.zeros((4, 4, 4), np.float32)
    o, h = (0.0, 0.0, 0.0), 1.0
    pts = np.array([[-1e-9, 1, 1], [3 + 1e-9, 1, 1], [1, 1, 3.0000001], [np.nan, 1, 1], [0, 0, 0], [3, 3, 3]])
    _, _, inside, _ = Q.sample(vals.astype(np.float64), o, h, (4, 4, 4), pts)
    assert inside.tolist() == [False, False, False, False, True, True]


def test_upper_cell_on_shared_face():
    vals = np.zeros((4, 4, 4))
    _, _, _, cell = Q.sample(vals, (0, 0, 0), 1.0, (4, 4, 4), np.array([[1.0, 2.0, 0.5]]))
    assert tuple(cell[0]) == (1, 2, 0)


def _interp_bound(h, hess_max):
    # tensor-product linear interpolation error: (h^2 / 8) * sum_a max |f_aa|
    return h * h / 8.0 * 3.0 * hess_max


def test_sphere_within_interpolation_bound():
    h = 1e-3
    g = sample_fp64(lambda p: W.field_sphere(p, (0, 0, 0), 0.01), (41, 41, 41), (-0.02,) * 3, h)
    rng = np.random.default_rng(4)
    x = rng.uniform(-0.0195, 0.0195, (4000, 3))
    rho = np.linalg.norm(x, axis=1)
    ok = rho > 4 * h
    x, rho = x[ok], rho[ok]
    phi, gr, _, _ = Q.sample(g.values, g.origin, g.h, g.dims, x)
    f = W.field_sphere(x, (0, 0, 0), 0.01)
    bound = _interp_bound(h, 1.0 / (rho - math.sqrt(3) * h))
    assert np.all(np.abs(phi - f) <= bound + 1e-15)
    # the bound is tight enough to matter: errors reach a good fraction of it
    assert np.max(np.abs(phi - f) / bound) > 0.2
    n_true = x / rho[:, None]
    err = np.linalg.norm(gr - n_true, axis=1)
    assert np.all(err <= 2.0 * math.sqrt(3) * h / (rho - math.sqrt(3) * h))


def test_torus_within_interpolation_bound():
    R, r, h = 0.02, 0.005, 1e-3
    g = W.sample_grid(lambda p: W.field_torus(p, R, r), (64, 64, 64), (-0.0315,) * 3, h)
    vals = Q.grid_values_f64(g.values, g.dtype)
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.03, 0.03, (6000, 3))
    rho = np.hypot(x[:, 0], x[:, 1])
    dcore = np.hypot(rho - R, x[:, 2])
    dmin = np.minimum(rho, dcore) - math.sqrt(3) * h
    ok = dmin > 2 * h
    x, dmin = x[ok], dmin[ok]
    phi, _, inside, _ = Q.sample(vals, g.origin, g.h, g.dims, x)
    assert inside.all()
    f = W.field_torus(x, R, r)
    # |f_aa| <= 1/d_core + 1/rho (two principal curvatures of the level sets)
    bound = _interp_bound(h, 2.0 / dmin) + 6e-10  # + float32 rounding of corners
    assert np.all(np.abs(phi - f) <= bound)


def test_box_exact_in_face_regions():
    half = np.array([0.3, 0.2, 0.25])
    h = 0.0625
    g = sample_fp64(lambda p: W.field_box(p, half), (17, 17, 17), (-0.5,) * 3, h)
    rng = np.random.default_rng(6)
    # outside +x face, away from edges: field = x - hx, affine
    x = np.c_[rng.uniform(0.3 + 2 * h, 0.48, 300), rng.uniform(-0.2 + 2 * h, 0.2 - 2 * h, 300),
              rng.uniform(-0.25 + 2 * h, 0.25 - 2 * h, 300)]
    phi, gr, _, _ = Q.sample(g.values, g.origin, g.h, g.dims, x)
    assert np.allclose(phi, x[:, 0] - 0.3, atol=1e-14)
    assert np.allclose(gr, [1, 0, 0], atol=1e-12)


def test_thread_field_within_lipschitz_bound():
    spec = W.M4_128
    g = W.bolt_grid(spec)
    vals = Q.grid_values_f64(g.values, g.dtype)
    rng = np.random.default_rng(7)
    lo = np.asarray(g.origin)
    hi = lo + g.h * (np.asarray(g.dims) - 1)
    x = lo + rng.random((3000, 3)) * (hi - lo)
    phi, _, _, _ = Q.sample(vals, g.origin, g.h, g.dims, x)
    f = W.field_bolt(x, spec.P, spec.Rmaj, spec.L)
    # max-composition of distance-like fields: Lipschitz constant ~1 (helix tilt < 10%)
    assert np.all(np.abs(phi - f) <= 1.1 * math.sqrt(3) * g.h + 1e-9)


# ---------------------------------------------------------------- meshes


def test_meshdist_cube_matches_box():
    v, t = W.cube_mesh(0.5)
    sdf = MD.MeshSDF(v, t)
    rng = np.random.default_rng(8)
    P = rng.uniform(-1.0, 1.0, (400, 3))
    assert np.allclose(sdf.many(P), W.field_box(P, (0.5, 0.5, 0.5)), atol=1e-12)


def test_oracle_on_tetrahedron_sdf_grid():
    v, t = W.tetrahedron_mesh(0.5)
    sdf = MD.MeshSDF(v, t)
    dims, origin, h = (9, 9, 9), (-1.0, -1.0, -1.0), 0.25
    P = node_positions(dims, origin, h)
    g = G(sdf.many(P), "f64", origin, h)
    # at nodes: exact
    phi, _, _, _ = Q.sample(g.values, origin, h, dims, P.reshape(-1, 3))
    assert np.array_equal(phi, g.values.reshape(-1))
    # in between: within the 1-Lipschitz bound sqrt(3) h
    rng = np.random.default_rng(9)
    x = rng.uniform(-0.99, 0.99, (300, 3))
    phi, _, _, _ = Q.sample(g.values, origin, h, dims, x)
    assert np.all(np.abs(phi - sdf.many(x)) <= math.sqrt(3) * h)


# ---------------------------------------------------------------- contacts, normals, bins


def test_fibonacci_table():
    for K in (16, 32, 64):
        d = W.fibonacci_bins(K).astype(np.float64)
        assert d.shape == (3, K)
        assert np.allclose(np.linalg.norm(d, axis=0), 1.0, atol=1e-6)
        assert np.all(np.diff(d[2]) < 0)
        assert d[2, 0] == np.float32(1.0 - 1.0 / K)
        # golden angle between successive azimuths
        az = np.arctan2(d[1], d[0])
        dd = np.mod(np.diff(az), 2 * np.pi)
        assert np.allclose(dd, np.mod(np.pi * (3 - np.sqrt(5)), 2 * np.pi), atol=1e-5)


def test_halfspace_contacts_closed_form():
    """Tilted half-space phi = n.x - c (affine -> exact): candidates, depth, normal, bin."""
    rng = np.random.default_rng(10)
    n = np.array([0.3, -0.4, 0.866])
    n /= np.linalg.norm(n)
    c = 0.05
    h = 1.0 / 64
    g = sample_fp64(lambda p: p @ n - c, (33, 33, 33), (-0.25,) * 3, h)
    bins = W.fibonacci_bins(32)
    verts = rng.uniform(-0.05, 0.05, (500, 3)).astype(np.float32)
    for _ in range(5):
        pose = np.r_[W.shoemake_quat(rng, 1)[:, 0], rng.uniform(-0.1, 0.1, 3)].astype(np.float32)
        r = Q.query_env(g, verts, pose, 0.0, bins)
        R = rot_unnormalised(pose[:4])
        xb = verts.astype(np.float64) @ R.T + pose[4:].astype(np.float64)
        phi_true = xb @ n - c
        assert r["inside"].all()
        assert np.allclose(r["phi"], phi_true, atol=1e-14)
        assert np.array_equal(r["cand"], phi_true < 0)
        assert np.allclose(r["depth"], -phi_true, atol=1e-14)
        assert np.allclose(r["normal"], n, atol=1e-12)
        expect_bin = int(np.argmax(n @ bins.astype(np.float64)))
        assert np.all(r["bin"] == expect_bin)


def test_bin_tie_goes_to_lowest_k_and_zero_normal_to_bin0():
    d = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 1, 0]], np.float32).T
    _, b, _ = Q.normals_and_bins(np.array([[0.0, 2.0, 0.0], [0.0, 0.0, 0.0]]), d)
    assert b.tolist() == [1, 0]
    # a constant field has zero gradient: normal 0, bin 0, still a candidate
    g = G(np.full((3, 3, 3), -1.0), "f64", (0, 0, 0), 1.0)
    r = Q.query_env(g, np.array([[0.5, 0.5, 0.5]], np.float32), np.array([0, 0, 0, 1, 0, 0, 0], np.float32),
                    0.0, W.fibonacci_bins(16))
    assert r["cand"][0] and np.all(r["normal"][0] == 0) and r["bin"][0] == 0


# ---------------------------------------------------------------- reduction


@pytest.mark.parametrize("seed", range(5))
def test_reduce_matches_bruteforce_and_is_order_free(seed):
    rng = np.random.default_rng(seed)
    n, n_env, K = 600, 5, 8
    env = rng.integers(0, n_env, n)
    vidx = rng.permutation(n)  # unique per row (like real vertex ids per env)
    depth = rng.choice(np.array([0.0, -0.0, 1e-5, 2e-5, -3e-6], np.float32), n)
    b = rng.integers(0, K, n)
    cand = rng.random(n) < 0.7
    wv, wd, _ = RD.reduce_contacts(env, vidx, depth, b, cand, n_env, K)
    bv, bd = RD.reduce_contacts_bruteforce(env, vidx, depth, b, cand, n_env, K)
    assert np.array_equal(wv, bv)
    assert np.array_equal(wd.view(np.uint32), bd.view(np.uint32))
    perm = rng.permutation(n)
    pv, pd, _ = RD.reduce_contacts(env[perm], vidx[perm], depth[perm], b[perm], cand[perm], n_env, K)
    assert np.array_equal(pv, wv) and np.array_equal(pd.view(np.uint32), wd.view(np.uint32))


def test_reduce_signed_zero_and_empty():
    env = np.array([0, 0, 0])
    vidx = np.array([7, 3, 9])
    depth = np.array([-0.0, 0.0, -1.0], np.float32)
    b = np.array([1, 1, 1])
    wv, wd, _ = RD.reduce_contacts(env, vidx, depth, b, np.array([True, True, True]), 1, 3)
    assert wv.tolist() == [[-1, 3, -1]]
    assert wd[0, 1] == 0.0 and not np.signbit(wd[0, 1])


# ---------------------------------------------------------------- adjoint


def test_penalty_halfspace_closed_form():
    """phi = z - z0: L = sum 0.5 k min(0, z_B - z0)^2; dL/dt = sum k phi e_z; dL/dw = sum x_B x (k phi e_z)."""
    rng = np.random.default_rng(11)
    z0, k, h = 0.01, 1e4, 1.0 / 128
    g = sample_fp64(lambda p: p[..., 2] - z0, (33, 33, 33), (-0.125,) * 3, h)
    verts = rng.uniform(-0.03, 0.03, (400, 3)).astype(np.float32)
    pose = np.r_[W.shoemake_quat(rng, 1)[:, 0], [0.0, 0.0, 0.005]].astype(np.float32)
    L, dxi, dv = A.penalty_env(g, verts, pose, k)
    R = rot_unnormalised(pose[:4])
    xb = verts.astype(np.float64) @ R.T + pose[4:].astype(np.float64)
    phi = np.minimum(xb[:, 2] - z0, 0.0)
    w = np.zeros_like(xb)
    w[:, 2] = k * phi
    assert np.isclose(L, np.sum(0.5 * k * phi ** 2), rtol=1e-12)
    assert np.allclose(dxi[:3], [0.0, 0.0, np.sum(k * phi)], atol=1e-9)
    assert np.allclose(dxi[3:], np.cross(xb, w).sum(0), atol=1e-9)
    assert np.allclose(dv, w @ R, atol=1e-9)


def test_penalty_gradient_matches_finite_differences():
    w = W.torus_workload(n_env=6)
    g = w.grids[0]
    vals = Q.grid_values_f64(g.values, g.dtype)
    verts = w.meshes[0].verts
    k = 1e4
    checked = 0
    for e in range(w.n_env):
        L, dxi, dv = A.penalty_env(g, verts, w.pose[:, e], k, vals)
        if L == 0.0:
            continue
        gfd, cross, bound = A.fd_twist(g, verts, w.pose[:, e], k, 1e-6, vals)
        scale = max(np.max(np.abs(gfd)), 1e-12)
        for i in range(6):
            tol = 1e-6 * scale + 1e-9 + bound[i]
            assert abs(dxi[i] - gfd[i]) <= tol, (e, i, dxi[i], gfd[i], cross[i], bound[i])
        gv, crossed = A.fd_verts(g, verts, w.pose[:, e], k, 1e-6, vals)
        ok = ~crossed
        assert np.allclose(dv[ok], gv[ok], rtol=1e-5, atol=1e-9 * scale)
        checked += 1
    assert checked >= 2


def test_fd_bound_covers_a_value_jump():
    """A field with a step: phi = z - z0 plus 1e-4 m where x > xs, cells of
    1 mm.  One penetrating vertex straddles the step within the stencil of a
    translation along x.  The central difference then carries the step
    (|FD - analytic| = k |phi| 1e-4 / 2h, huge); the gradient-jump share
    (no gradient jump here) does not cover it, the value-jump share of
    jumps=True does, and the other components stay exact."""
    xs, z0, k, h, step = 0.0, 0.01, 1e4, 1e-6, 1e-4

    def sampler(x):
        phi = x[:, 2] - z0 + np.where(x[:, 0] > xs, step, 0.0)
        grad = np.tile([0.0, 0.0, 1.0], (len(x), 1))
        cell = np.floor(x / 1e-3).astype(np.int64)
        return phi, grad, np.ones(len(x), bool), cell

    verts = np.array([[0.0, 0.0, 0.0], [0.0035, 0.0015, 0.0025], [-0.0045, 0.0025, 0.0015]], np.float32)
    pose = np.array([0, 0, 0, 1, 0.0, 0.0, 0.0], np.float32)
    L, dxi, _ = A.penalty_env(None, verts, pose, k, sampler=sampler)
    g0, cross0, b0 = A.fd_twist(None, verts, pose, k, h, sampler=sampler)
    g1, cross1, b1 = A.fd_twist(None, verts, pose, k, h, sampler=sampler, jumps=True)
    assert np.array_equal(g0, g1) and np.array_equal(cross0, cross1)
    assert cross0[0] == 1 and abs(dxi[0] - g0[0]) > 100 * max(b0[0], 1e-9)
    assert abs(dxi[0] - g1[0]) <= b1[0]
    assert np.allclose(dxi[1:3], g1[1:3], rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------- half precision decode


def test_half_decode():
    x = np.array([1.0, -2.5, 3.140625, 65504.0, 1e-3], np.float32)
    assert np.array_equal(Q.grid_values_f64(W.to_f16_bits(x), "f16"), x.astype(np.float16).astype(np.float64))
    b = W.to_bf16_bits(np.array([1.0, -2.0, 1.00390625, 1.01171875], np.float32))
    # 1.0 -> 0x3F80; 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 ties up to 1 + 2^-6
    assert b.tolist() == [0x3F80, 0xC000, 0x3F80, 0x3F82]
    assert np.array_equal(Q.grid_values_f64(b, "bf16"), [1.0, -2.0, 1.0, 1.015625])


def test_half_error_bounded_by_corner_rounding():
    g32 = W.sample_grid(lambda p: W.field_torus(p, 0.02, 0.005), (64, 64, 64), (-0.0315,) * 3, 1e-3)
    rng = np.random.default_rng(12)
    x = rng.uniform(-0.03, 0.03, (3000, 3))
    v32 = Q.grid_values_f64(g32.values, "f32")
    p32, _, ins, cell = Q.sample(v32, g32.origin, g32.h, g32.dims, x)
    for dt in ("f16", "bf16"):
        gh = W.convert_grid(g32, dt)
        vh = Q.grid_values_f64(gh.values, dt)
        ph, _, _, _ = Q.sample(vh, gh.origin, gh.h, gh.dims, x)
        diff = np.abs(vh - v32)
        ix, iy, iz = cell[:, 0], cell[:, 1], cell[:, 2]
        cmax = np.max(np.stack([diff[iz + c, iy + b, ix + a] for a in (0, 1) for b in (0, 1) for c in (0, 1)]), 0)
        assert np.all(np.abs(ph - p32)[ins] <= cmax[ins] * (1 + 1e-12))
