"""Pins of the mesh-to-SDF bake oracle (CPU only): the cube mesh reproduces
the exact box SDF at every node, a tetrahedron's bake equals the per-point
brute force of ``meshdist`` and is negative exactly at its interior nodes, an
icosphere's bake stays within the polyhedron's deviation from the sphere's
SDF with the sphere's sign beyond it, and planted mistakes are caught."""
import numpy as np
import pytest

from oracle import bake as OB
from oracle import meshdist as MD
from paper_2205_03532_amd import workloads as W
from test_oracle_pins import node_positions


def test_cube_bake_is_the_box_sdf():
    v, t = W.cube_mesh(0.5)
    dims, origin, h = (13, 13, 13), (-0.9, -0.9, -0.9), 0.15
    got = OB.bake(v, t, dims, origin, h)
    ref = W.field_box(node_positions(dims, origin, h), (0.5, 0.5, 0.5))
    assert np.max(np.abs(got - ref)) < 1e-12


def test_tetrahedron_bake_matches_bruteforce_and_sign():
    v, t = W.tetrahedron_mesh(0.5)
    dims, origin, h = (9, 9, 9), (-1.0, -1.0, -1.0), 0.25
    got = OB.bake(v, t, dims, origin, h)
    P = node_positions(dims, origin, h)
    assert np.max(np.abs(got - MD.MeshSDF(v, t).many(P))) < 1e-12
    # inside the tetrahedron iff on the inner side of all four face planes
    V = np.asarray(v, float)
    inside = np.ones(P.shape[:-1], dtype=bool)
    for tri in t:
        a, b, c = V[tri]
        n = np.cross(b - a, c - a)
        inside &= (P - a) @ n < 0
    assert np.array_equal(got < 0, inside)


def test_icosphere_bake_within_tessellation_of_sphere():
    r = 0.01
    m = W.icosphere(2, r)
    V = m.verts.astype(np.float64)
    T = m.tris
    # the polyhedron lies between the spheres of radius r - s and r
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    s = r - np.min(np.abs(np.sum(n * a, axis=1)))
    s += 1e-9  # the float32 vertices are within a few ulp of the sphere
    dims, origin, h = (12, 12, 12), (-0.016, -0.016, -0.016), 0.003
    got = OB.bake(V, T, dims, origin, h)
    ref = W.field_sphere(node_positions(dims, origin, h), (0, 0, 0), r)
    assert np.max(np.abs(got - ref)) <= s
    far = np.abs(ref) > s
    assert np.array_equal(np.sign(got[far]), np.sign(ref[far]))


def dented_cube(half=0.5, dent=0.3):
    """Closed cube whose top face is pushed in to a pyramid (concave edges
    and a concave apex); outward winding."""
    v, t = W.cube_mesh(half)
    v = np.vstack([v, [0.0, 0.0, half - dent]])
    apex = len(v) - 1
    top = [4, 5, 7, 6]  # z = +half corners, counter-clockwise seen from +z
    t = [tri for tri in t.tolist() if not all(v[i][2] > 0 for i in tri)]
    for i in range(4):
        t.append([top[i], top[(i + 1) % 4], apex])
    return v, np.asarray(t, dtype=np.int32)


def inside_by_ray_parity(P, v, t, d=(0.2113, 0.4387, 0.8734)):
    """Inside test independent of normals: crossings of a ray from each point
    (Moller-Trumbore), odd = inside."""
    d = np.asarray(d) / np.linalg.norm(d)
    cnt = np.zeros(len(P), dtype=np.int64)
    V = np.asarray(v, float)
    for i, j, k in t:
        a, b, c = V[i], V[j], V[k]
        e1, e2 = b - a, c - a
        pv = np.cross(d, e2)
        det = e1 @ pv
        if abs(det) < 1e-15:
            continue
        tv = P - a
        u = (tv @ pv) / det
        qv = np.cross(tv, e1)
        w = (qv @ d) / det
        s = (qv @ e2) / det
        cnt += ((u >= 0) & (w >= 0) & (u + w <= 1) & (s > 0)).astype(np.int64)
    return cnt % 2 == 1


def test_dented_cube_sign_matches_ray_parity():
    """Concave edges and a concave vertex: the pseudonormal sign rule must
    agree with ray-crossing parity at every node not on the surface."""
    v, t = dented_cube()
    dims, origin, h = (17, 17, 17), (-0.8, -0.8, -0.8), 0.1
    got = OB.bake(v, t, dims, origin, h).reshape(-1)
    P = node_positions(dims, origin, h).reshape(-1, 3) + 1e-7  # off the faces' planes
    ins = inside_by_ray_parity(P, v, t)
    clear = np.abs(got) > 1e-6
    assert np.array_equal((got < 0)[clear], ins[clear])
    assert ins.sum() > 50 and (~ins).sum() > 50


def test_closest_point_features_cover_the_regions():
    """Every feature code occurs, and the closest point is at most as far as
    any of the triangle's corners, edge midpoints and centroid."""
    rng = np.random.default_rng(4)
    a, b, c = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.2, 0.9, 0])
    P = rng.uniform(-1.0, 2.0, (4000, 3))
    q, feat = OB.closest_on_triangle(P, a, b, c)
    assert set(np.unique(feat)) == set(range(7))
    d = np.linalg.norm(P - q, axis=1)
    for s in (a, b, c, (a + b) / 2, (a + c) / 2, (b + c) / 2, (a + b + c) / 3):
        assert np.all(d <= np.linalg.norm(P - s, axis=1) + 1e-12)


@pytest.mark.parametrize("mutation", ["face_normal_flipped", "vertex_pseudonormal_unweighted",
                                      "edge_uses_one_face_normal"])
def test_planted_bake_mistake_is_caught(monkeypatch, mutation):
    orig_pn = OB.pseudonormals
    if mutation == "face_normal_flipped":
        monkeypatch.setattr(OB, "pseudonormals", lambda V, T: (lambda r: (-r[0], r[1], r[2]))(orig_pn(V, T)))
    elif mutation == "vertex_pseudonormal_unweighted":
        def unweighted(V, T):
            fn, en, vn = orig_pn(V, T)
            vn2 = np.zeros_like(vn)
            for f, tri in enumerate(np.asarray(T)):
                for i in tri:
                    vn2[i] += fn[f] * (1.0 + 5.0 * (f % 2))  # not the angle weights
            return fn, en, vn2
        monkeypatch.setattr(OB, "pseudonormals", unweighted)
    else:
        def one_face(V, T):
            fn, en, vn = orig_pn(V, T)
            return fn, np.repeat(fn[:, None, :], 3, axis=1), vn  # an edge takes this face's normal only
        monkeypatch.setattr(OB, "pseudonormals", one_face)
    caught = False
    for pin in (test_cube_bake_is_the_box_sdf, test_tetrahedron_bake_matches_bruteforce_and_sign,
                test_icosphere_bake_within_tessellation_of_sphere, test_dented_cube_sign_matches_ray_parity):
        try:
            pin()
        except AssertionError:
            caught = True
    assert caught, mutation
