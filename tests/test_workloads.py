"""Seeded input generator checks (CPU only)."""
import math

import numpy as np

from paper_2205_03532_amd import workloads as W


def test_icosphere_counts_and_radius():
    m = W.icosphere(4, 0.01)
    assert m.n == 2562 and len(m.tris) == 20 * 4**4
    assert np.allclose(np.linalg.norm(m.verts.astype(np.float64), axis=1), 0.01, rtol=1e-6)


def test_torus_workload_shape_and_seed():
    a = W.torus_workload()
    b = W.torus_workload()
    assert a.n_env == 256 and a.K == 16 and a.n_queries == 256 * 2562
    assert a.grids[0].dims == (64, 64, 64) and a.grids[0].h == np.float32(1e-3)
    assert np.array_equal(a.pose, b.pose)
    q = a.pose[:4].astype(np.float64)
    assert np.allclose(np.linalg.norm(q, axis=0), 1.0, atol=1e-6)
    assert np.all(np.abs(a.pose[4:]) <= 0.015)


def test_nut_mesh_follows_thread():
    s = W.M16_BOLT_256x256x512
    m = W.nut_mesh(s)
    assert m.n == 128 * 128 + 12
    v = m.verts.astype(np.float64)
    rho = np.hypot(v[:, 0], v[:, 1])
    bore = rho < 9e-3
    assert bore.sum() == 128 * 128
    th = np.arctan2(v[bore, 1], v[bore, 0])
    sphase = v[bore, 2] - s.P * th / (2 * math.pi)
    expect = W.thread_profile_radius(sphase, s.P, s.Rmaj) + s.clearance
    assert np.allclose(rho[bore], expect, atol=2e-8)
    assert v[:, 2].min() >= 0 and v[:, 2].max() <= np.float32(s.nut_h)


def test_thread_profile_depth_and_flank_angle():
    P, R = 2e-3, 8e-3
    s = np.linspace(0, P, 16001)
    r = W.thread_profile_radius(s, P, R)
    D = 5 / 8 * math.sqrt(3) / 2 * P
    assert math.isclose(r.max(), R) and math.isclose(r.min(), R - D, rel_tol=1e-12)
    slope = np.max(np.abs(np.diff(r) / np.diff(s)))
    assert math.isclose(math.degrees(math.atan(slope)), 60.0, abs_tol=0.01)  # 30 deg from radial


def test_bolt_field_sign_and_distance():
    P, R, L = 2e-3, 8e-3, 40e-3
    p = np.array([[0.0, 0.0, 0.02], [0.02, 0.0, 0.02], [0.0, 0.0, -0.001]])
    f = W.field_bolt(p, P, R, L)
    assert f[0] < 0 and f[1] > 0 and math.isclose(f[2], 0.001, rel_tol=1e-9)


def test_half_storage_conversion():
    w = W.torus_workload(n_env=4)
    for dt in ("f16", "bf16"):
        h = W.half_storage(w, dt)
        assert h.grids[0].values.dtype == np.uint16 and h.grids[0].dtype == dt
        assert h.grids[0].nbytes * 2 == w.grids[0].nbytes


def test_mixed_part_specs_fit_their_grids():
    for s in (W.M4_128, W.M8_192, W.M16_256):
        hi = np.asarray(s.origin) + s.h * (np.asarray(s.grid_dims) - 1)
        assert s.origin[2] < 0 and hi[2] > s.L
        assert hi[2] > s.z_range[1] + s.nut_h
        assert -s.origin[0] > s.Rmaj + s.lateral
    for s in (W.ROUND_PEG_64, W.RECT_PEG_96):
        hi = np.asarray(s.origin) + s.h * (np.asarray(s.grid_dims) - 1)
        assert np.all(hi > np.asarray(s.block_half))
