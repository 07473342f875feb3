"""Seeded synthetic inputs for the vertex-vs-SDF contact path.

This module builds INPUT arrays only: voxel SDF grids sampled from closed-form
fields, vertex meshes, one pose per environment and the normal-bin direction
table.  It holds none of the query, reduction or adjoint arithmetic: the HIP
path and the CPU oracle both consume what it produces, and neither imports the
other.

Why synthetic stand-ins: the paper's assets (the NIST board parts, its OBJ
meshes and the SDFs baked from them; Section IV and the geometric
representation table of Appendix C) are not available, so the shapes here are
closed-form analogues with the same sizes: a torus, an M16-like threaded bolt
and a hex nut with a matching internal thread, round and rectangular
peg-in-hole pairs, and M4 / M8 nut-bolt pairs.

Conventions (shared with the C ABI):
  * grid values are node samples in [nz][ny][nx] order (x fastest); node
    (i, j, k) sits at origin + (i, j, k) * h; metres throughout;
  * ``origin`` and ``h`` are float32-representable (both sides read the same
    float32 numbers);
  * FP16 / BF16 grids are stored as uint16 bit patterns, rounded from the
    float32 grid to nearest-even;
  * mesh vertices are float32 (n, 3) in body A's frame;
  * poses are float32 [7][n_env]: qx, qy, qz, qw, tx, ty, tz, placing A in
    B's frame (x_B = R(q) v + t);
  * the bin table is float32 [3][K].
"""
from __future__ import annotations

import functools
import math
import os
from dataclasses import dataclass, field

import numpy as np

GEN_VERSION = 1

# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------


@dataclass
class Grid:
    values: np.ndarray  # (nz, ny, nx) float32, or uint16 bit patterns (f16 / bf16)
    dtype: str  # 'f32' | 'f16' | 'bf16'
    origin: tuple  # three float32 values, metres
    h: float  # float32 value, metres

    @property
    def dims(self):
        nz, ny, nx = self.values.shape
        return (nx, ny, nz)

    @property
    def nbytes(self):
        return int(self.values.nbytes)


@dataclass
class Mesh:
    verts: np.ndarray  # (n, 3) float32
    tris: np.ndarray | None = None  # (m, 3) int32 or None

    @property
    def n(self):
        return int(self.verts.shape[0])


@dataclass
class Workload:
    name: str
    grids: list
    meshes: list
    env_grid: np.ndarray  # int32 [n_env]
    env_mesh: np.ndarray  # int32 [n_env]
    pose: np.ndarray  # float32 [7, n_env]
    bins: np.ndarray  # float32 [3, K]
    margin: float
    meta: dict = field(default_factory=dict)

    @property
    def n_env(self):
        return int(self.env_grid.shape[0])

    @property
    def K(self):
        return int(self.bins.shape[1])

    @property
    def n_queries(self):
        return int(sum(self.meshes[m].n for m in self.env_mesh))

    def env_query_offsets(self):
        """Query index q = offset[e] + v (vertices of env e's mesh in order)."""
        n = np.array([self.meshes[m].n for m in self.env_mesh], dtype=np.int64)
        off = np.zeros(self.n_env + 1, dtype=np.int64)
        np.cumsum(n, out=off[1:])
        return off


# ----------------------------------------------------------------------------
# scalar helpers
# ----------------------------------------------------------------------------


def f32(x):
    return float(np.float32(x))


def to_f16_bits(values_f32: np.ndarray) -> np.ndarray:
    """float32 -> IEEE binary16, round to nearest even, as uint16 bits."""
    return np.ascontiguousarray(values_f32.astype(np.float32).astype(np.float16).view(np.uint16))


def to_bf16_bits(values_f32: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 (top 16 bits), round to nearest even, as uint16 bits.

    NaN stays NaN (quiet bit forced); infinities stay infinite.
    """
    u = np.ascontiguousarray(values_f32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    rounded = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    rounded = np.where(nan, ((u >> 16) | 0x40) & 0xFFFF, rounded)
    return np.ascontiguousarray(rounded.astype(np.uint16))


def convert_grid(g: Grid, dtype: str) -> Grid:
    """Re-store an FP32 grid as 'f16' or 'bf16' (RNE), same geometry."""
    if g.dtype != "f32":
        raise ValueError("convert_grid expects an f32 grid")
    if dtype == "f32":
        return g
    bits = to_f16_bits(g.values) if dtype == "f16" else to_bf16_bits(g.values)
    return Grid(values=bits, dtype=dtype, origin=g.origin, h=g.h)


def convert_workload(w: Workload, dtype: str) -> Workload:
    return Workload(
        name=f"{w.name}-{dtype}",
        grids=[convert_grid(g, dtype) for g in w.grids],
        meshes=w.meshes,
        env_grid=w.env_grid,
        env_mesh=w.env_mesh,
        pose=w.pose,
        bins=w.bins,
        margin=w.margin,
        meta=dict(w.meta, storage=dtype),
    )


# ----------------------------------------------------------------------------
# closed-form fields (FP64) that the grids sample
# ----------------------------------------------------------------------------


def field_sphere(p, c=(0.0, 0.0, 0.0), r=1.0):
    d = p - np.asarray(c, dtype=np.float64)
    return np.sqrt(np.einsum("...i,...i->...", d, d)) - r


def field_box(p, half, c=(0.0, 0.0, 0.0)):
    """Exact Euclidean signed distance of an axis-aligned box."""
    q = np.abs(p - np.asarray(c, dtype=np.float64)) - np.asarray(half, dtype=np.float64)
    outside = np.sqrt(np.sum(np.maximum(q, 0.0) ** 2, axis=-1))
    inside = np.minimum(np.max(q, axis=-1), 0.0)
    return outside + inside


def field_torus(p, R, r):
    """Torus about the z axis, centred at the origin (exact distance)."""
    rho = np.hypot(p[..., 0], p[..., 1])
    return np.hypot(rho - R, p[..., 2]) - r


def field_halfspace(p, n, z0):
    """Solid {x : n.x < z0}; value n.x - z0 (exact for unit n)."""
    return p @ np.asarray(n, dtype=np.float64) - z0


def thread_profile_radius(s, P, Rmaj):
    """Radius of a 60-degree ISO-like external thread at axial phase s.

    One period, in units of P/16: crest flat [-1, 1] at the major radius, a
    flank down over [1, 6], the root flat [6, 10] at the minor radius, a flank
    up over [10, 15].  Thread depth 5/8 H with H = sqrt(3)/2 P.
    """
    D = 5.0 / 8.0 * (math.sqrt(3.0) / 2.0) * P
    Rmin = Rmaj - D
    u = np.mod(s, P) * (16.0 / P)
    r = np.full_like(u, Rmaj)
    r = np.where((u >= 1.0) & (u < 6.0), Rmaj - D * (u - 1.0) / 5.0, r)
    r = np.where((u >= 6.0) & (u < 10.0), Rmin, r)
    r = np.where((u >= 10.0) & (u < 15.0), Rmin + D * (u - 10.0) / 5.0, r)
    return r


def _thread_polyline(P, Rmaj):
    """Profile vertices (s, rho) over periods -1..2 (covers s in [0,P) +- P)."""
    D = 5.0 / 8.0 * (math.sqrt(3.0) / 2.0) * P
    Rmin = Rmaj - D
    pts = []
    for m in (-1, 0, 1, 2):
        base = m * P
        pts += [
            (base - P / 16.0, Rmaj),
            (base + P / 16.0, Rmaj),
            (base + 6.0 * P / 16.0, Rmin),
            (base + 10.0 * P / 16.0, Rmin),
        ]
    pts.append((3 * P - P / 16.0, Rmaj))
    return np.asarray(pts, dtype=np.float64)


def field_thread_2d(rho, s, P, Rmaj):
    """Signed distance in the meridional (rho, z) plane to the periodic profile.

    Negative inside the solid rho < r(s).  s is any real; only its phase
    matters.  Exact 2-D distance: the nearest boundary point of the periodic
    profile is always within one period of s, and the polyline spans that.
    """
    sp = np.mod(s, P)
    poly = _thread_polyline(P, Rmaj)
    best = np.full(np.shape(rho), np.inf)
    for a, b in zip(poly[:-1], poly[1:]):
        ex, ey = b[0] - a[0], b[1] - a[1]
        dx, dy = sp - a[0], rho - a[1]
        t = np.clip((dx * ex + dy * ey) / (ex * ex + ey * ey), 0.0, 1.0)
        best = np.minimum(best, np.hypot(dx - t * ex, dy - t * ey))
    inside = rho < thread_profile_radius(sp, P, Rmaj)
    return np.where(inside, -best, best)


def field_bolt(p, P, Rmaj, L):
    """Threaded rod along +z, z in [0, L], right-handed helix.

    In cylindrical coordinates the thread phase is s = z - P*theta/(2 pi); the
    meridional 2-D distance is intersected with the end caps by a max.  Not an
    exact Euclidean distance (the helix lead angle tilts the true closest
    point out of the meridional plane); it is the field the grid samples.
    """
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    rho = np.hypot(x, y)
    theta = np.arctan2(y, x)
    s = z - P * theta / (2.0 * math.pi)
    f2 = field_thread_2d(rho, s, P, Rmaj)
    return np.maximum(f2, np.maximum(-z, z - L))


def field_round_hole_block(p, half, r_hole):
    """Block with a round through-hole along z (hole axis at x = y = 0)."""
    rho = np.hypot(p[..., 0], p[..., 1])
    return np.maximum(field_box(p, half), r_hole - rho)


def field_rect_hole_block(p, half, hole_half):
    """Block with a square through-hole along z."""
    q = np.abs(p[..., :2]) - np.asarray(hole_half, dtype=np.float64)
    hole2d = np.sqrt(np.sum(np.maximum(q, 0.0) ** 2, axis=-1)) + np.minimum(np.max(q, axis=-1), 0.0)
    return np.maximum(field_box(p, half), -hole2d)


def sample_grid(fn, dims, origin, h, chunk_nodes=1 << 21) -> Grid:
    """Evaluate fn at every node in FP64 and round to float32 (RNE)."""
    nx, ny, nz = (int(d) for d in dims)
    o = np.asarray([f32(v) for v in origin], dtype=np.float64)
    hh = np.float64(np.float32(h))
    xs = o[0] + hh * np.arange(nx, dtype=np.float64)
    ys = o[1] + hh * np.arange(ny, dtype=np.float64)
    zs = o[2] + hh * np.arange(nz, dtype=np.float64)
    out = np.empty((nz, ny, nx), dtype=np.float32)
    X, Y = np.meshgrid(xs, ys, indexing="xy")  # (ny, nx)
    per = max(1, chunk_nodes // (nx * ny))
    for k0 in range(0, nz, per):
        k1 = min(nz, k0 + per)
        Z = zs[k0:k1, None, None]
        p = np.empty((k1 - k0, ny, nx, 3), dtype=np.float64)
        p[..., 0] = X[None]
        p[..., 1] = Y[None]
        p[..., 2] = Z
        out[k0:k1] = fn(p).astype(np.float32)
    return Grid(values=out, dtype="f32", origin=tuple(float(v) for v in o), h=float(hh))


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------


def morton_order(verts: np.ndarray, bits: int = 10) -> np.ndarray:
    """Permutation sorting points along a 3-D Z-order curve (stable)."""
    v = np.asarray(verts, dtype=np.float64)
    lo, hi = v.min(axis=0), v.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    q = np.clip(((v - lo) / span * ((1 << bits) - 1)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(len(v), dtype=np.int64)
    for b in range(bits):
        for a in range(3):
            code |= ((q[:, a] >> b) & 1) << (3 * b + a)
    return np.argsort(code, kind="stable")


def _reorder(verts, tris, perm):
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    v = np.ascontiguousarray(verts[perm])
    t = None if tris is None else np.ascontiguousarray(inv[tris]).astype(np.int32)
    return v, t


def icosphere(level: int, radius: float) -> Mesh:
    """Subdivided icosahedron projected to a sphere: 10*4^level + 2 vertices."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0),
         (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
         (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.asarray(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = (np.asarray(verts) * radius).astype(np.float32)
    T = np.asarray(faces, dtype=np.int32)
    return Mesh(verts=V, tris=T)


def hex_nut(P, Rmaj, clearance, height, across_flats, n_theta, n_z) -> Mesh:
    """Hex nut: threaded bore surface sampled n_theta x n_z, plus the 12 hex corners.

    Local frame: bore axis = +z, z in [0, height]; the bore surface is the bolt
    profile pushed out radially by ``clearance`` with the same helix phase, so
    the nut threads onto the bolt at pose rotation 2*pi*z/P about z.
    Vertices are returned in Morton order (vertex index = array position).
    """
    th = np.arange(n_theta, dtype=np.float64) * (2.0 * math.pi / n_theta)
    zz = (np.arange(n_z, dtype=np.float64) + 0.5) * (height / n_z)
    TH, ZZ = np.meshgrid(th, zz, indexing="ij")  # (n_theta, n_z)
    s = ZZ - P * TH / (2.0 * math.pi)
    rho = thread_profile_radius(s, P, Rmaj) + clearance
    bore = np.stack([rho * np.cos(TH), rho * np.sin(TH), ZZ], axis=-1).reshape(-1, 3)
    # quads (i, j) - (i+1, j) - (i+1, j+1) - (i, j+1), wrapping in theta
    i = np.arange(n_theta)[:, None]
    j = np.arange(n_z - 1)[None, :]
    a = (i * n_z + j)
    b = (((i + 1) % n_theta) * n_z + j)
    c = b + 1
    d = a + 1
    tris = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3),
                           np.stack([a, c, d], -1).reshape(-1, 3)]).astype(np.int32)
    rc = across_flats / math.sqrt(3.0)  # hex circumradius
    ang = np.arange(6) * (math.pi / 3.0) + math.pi / 6.0
    ring = np.stack([rc * np.cos(ang), rc * np.sin(ang)], -1)
    hexv = np.concatenate([np.c_[ring, np.zeros(6)], np.c_[ring, np.full(6, height)]])
    verts = np.concatenate([bore, hexv]).astype(np.float64)
    perm = morton_order(verts)
    v, t = _reorder(verts.astype(np.float32), tris, perm)
    return Mesh(verts=v, tris=t)


def round_peg(radius, length, n_theta, n_z, n_cap_rings) -> Mesh:
    """Cylinder along +z, z in [0, length]: side n_theta x n_z plus two capped disks."""
    th = np.arange(n_theta) * (2.0 * math.pi / n_theta)
    zz = np.linspace(0.0, length, n_z)
    TH, ZZ = np.meshgrid(th, zz, indexing="ij")
    side = np.stack([radius * np.cos(TH), radius * np.sin(TH), ZZ], -1).reshape(-1, 3)
    caps = []
    for z in (0.0, length):
        caps.append([[0.0, 0.0, z]])
        for k in range(1, n_cap_rings):
            r = radius * k / n_cap_rings
            caps.append(np.stack([r * np.cos(th), r * np.sin(th), np.full(n_theta, z)], -1))
    verts = np.concatenate([side] + [np.asarray(c) for c in caps]).astype(np.float64)
    perm = morton_order(verts)
    return Mesh(verts=np.ascontiguousarray(verts[perm].astype(np.float32)))


def rect_peg(half_x, half_y, length, n_per_side) -> Mesh:
    """Square-section peg along +z, z in [0, length], surface points on a grid."""
    pts = []
    ax = np.linspace(-1.0, 1.0, n_per_side)
    az = np.linspace(0.0, length, n_per_side * 2)
    for sx in (-1.0, 1.0):  # faces x = +-half_x
        Y, Z = np.meshgrid(ax * half_y, az, indexing="ij")
        pts.append(np.stack([np.full(Y.shape, sx * half_x), Y, Z], -1).reshape(-1, 3))
    for sy in (-1.0, 1.0):
        X, Z = np.meshgrid(ax[1:-1] * half_x, az, indexing="ij")
        pts.append(np.stack([X, np.full(X.shape, sy * half_y), Z], -1).reshape(-1, 3))
    for z in (0.0, length):
        X, Y = np.meshgrid(ax[1:-1] * half_x, ax[1:-1] * half_y, indexing="ij")
        pts.append(np.stack([X, Y, np.full(X.shape, z)], -1).reshape(-1, 3))
    verts = np.concatenate(pts).astype(np.float64)
    perm = morton_order(verts)
    return Mesh(verts=np.ascontiguousarray(verts[perm].astype(np.float32)))


def bolt_mesh(P, Rmaj, L, n_theta, n_z):
    """Closed, outward-wound threaded rod along +z, z in [0, L]: the thread
    surface rho = r(z - P theta / (2 pi)) sampled n_theta x n_z (z from 0 to
    L inclusive), closed by two disk fans about the axis.
    2 n_theta (n_z - 1) + 2 n_theta triangles."""
    th = np.arange(n_theta, dtype=np.float64) * (2.0 * math.pi / n_theta)
    zz = np.linspace(0.0, L, n_z)
    TH, ZZ = np.meshgrid(th, zz, indexing="ij")  # (n_theta, n_z)
    rho = thread_profile_radius(ZZ - P * TH / (2.0 * math.pi), P, Rmaj)
    side = np.stack([rho * np.cos(TH), rho * np.sin(TH), ZZ], axis=-1).reshape(-1, 3)
    i = np.arange(n_theta)[:, None]
    j = np.arange(n_z - 1)[None, :]
    a = i * n_z + j
    b = ((i + 1) % n_theta) * n_z + j
    tris = [np.stack([a, b, b + 1], -1).reshape(-1, 3), np.stack([a, b + 1, a + 1], -1).reshape(-1, 3)]
    lo, hi = n_theta * n_z, n_theta * n_z + 1  # cap centres
    r0 = np.arange(n_theta) * n_z
    r1 = ((np.arange(n_theta) + 1) % n_theta) * n_z
    tris.append(np.stack([np.full(n_theta, lo), r1, r0], -1))  # z = 0, normal -z
    tris.append(np.stack([np.full(n_theta, hi), r0 + n_z - 1, r1 + n_z - 1], -1))  # z = L, normal +z
    verts = np.concatenate([side, [[0.0, 0.0, 0.0], [0.0, 0.0, L]]])
    return verts.astype(np.float32), np.concatenate(tris).astype(np.int32)


@dataclass(frozen=True)
class BakeSpec:
    """A mesh to bake and the grid to bake it on."""
    name: str
    P: float
    Rmaj: float
    L: float
    n_theta: int
    n_z: int
    grid_dims: tuple
    h: float
    origin: tuple


# An M4 bolt as a 47k-triangle mesh on a 144 x 144 x 256 grid (5.3 M nodes):
# the size class of the M4 bolt SDF the paper describes (Appendix, geometric
# representations); a headless threaded rod stands in for the real part.
M4_BOLT_BAKE = BakeSpec(name="m4_bolt_bake", P=0.7e-3, Rmaj=2e-3, L=12e-3, n_theta=128, n_z=184,
                        grid_dims=(144, 144, 256), h=0.06e-3,
                        origin=(-4.29e-3, -4.29e-3, -1.65e-3))


def bake_workload(spec: BakeSpec = M4_BOLT_BAKE):
    """(verts float32 (n, 3), tris int32 (m, 3), dims, origin, h) of a bake."""
    v, t = bolt_mesh(spec.P, spec.Rmaj, spec.L, spec.n_theta, spec.n_z)
    return v, t, spec.grid_dims, tuple(f32(o) for o in spec.origin), f32(spec.h)


def tetrahedron_mesh(scale=1.0):
    """Regular tetrahedron, 4 vertices, 4 outward-wound triangles."""
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64) * scale
    t = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], dtype=np.int32)
    return v, t


def cube_mesh(half=1.0):
    """Closed axis-aligned cube, 8 vertices, 12 outward-wound triangles."""
    v = np.array([[x, y, z] for z in (-1, 1) for y in (-1, 1) for x in (-1, 1)], dtype=np.float64) * half
    t = np.array([
        [0, 2, 1], [1, 2, 3],  # z = -1
        [4, 5, 6], [5, 7, 6],  # z = +1
        [0, 1, 4], [1, 5, 4],  # y = -1
        [2, 6, 3], [3, 6, 7],  # y = +1
        [0, 4, 2], [2, 4, 6],  # x = -1
        [1, 3, 5], [3, 7, 5],  # x = +1
    ], dtype=np.int32)
    return v, t


# ----------------------------------------------------------------------------
# poses and bins
# ----------------------------------------------------------------------------


def shoemake_quat(rng, n):
    """Uniform random unit quaternions (Shoemake 1992), (x, y, z, w), FP64."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    return np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                     b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=0)


def quat_about_z(theta):
    return np.stack([np.zeros_like(theta), np.zeros_like(theta), np.sin(theta / 2), np.cos(theta / 2)], axis=0)


def pack_pose(q, t):
    """q (4, n) x,y,z,w and t (3, n), FP64 -> float32 [7][n]."""
    return np.ascontiguousarray(np.concatenate([q, t], axis=0).astype(np.float32))


def fibonacci_bins(K: int) -> np.ndarray:
    """Fibonacci-lattice unit directions, float32 [3][K].

    z_k = 1 - (2k+1)/K, rho_k = sqrt(1 - z_k^2), theta_k = k * pi * (3 - sqrt 5);
    built in FP64 and rounded to float32.  Passed to both sides as data.
    """
    k = np.arange(K, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / K
    rho = np.sqrt(1.0 - z * z)
    th = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.ascontiguousarray(np.stack([rho * np.cos(th), rho * np.sin(th), z]).astype(np.float32))


# ----------------------------------------------------------------------------
# part geometry (all lengths in metres)
# ----------------------------------------------------------------------------


@dataclass(frozen=True)
class NutBoltSpec:
    name: str
    P: float  # pitch
    Rmaj: float  # bolt major radius
    L: float  # bolt length (z in [0, L])
    nut_af: float  # across flats
    nut_h: float  # nut height
    clearance: float  # radial clearance of the nut bore
    grid_dims: tuple
    h: float
    origin: tuple
    n_theta: int
    n_z: int
    z_range: tuple  # axial placement range of the nut base
    lateral: float  # +- lateral jitter
    twist_deg: float = 0.5

    @property
    def n_verts(self):
        return self.n_theta * self.n_z + 12


M16_BOLT_256x256x512 = NutBoltSpec(
    name="m16", P=2e-3, Rmaj=8e-3, L=40e-3, nut_af=24e-3, nut_h=13e-3, clearance=25e-6,
    grid_dims=(256, 256, 512), h=1e-4, origin=(-12.75e-3, -12.75e-3, -5.55e-3),
    n_theta=128, n_z=128, z_range=(0.0, 25e-3), lateral=50e-6)

# the five part types of the mixed batch (proposed sizes; see the design notes)
M4_128 = NutBoltSpec(
    name="m4", P=0.7e-3, Rmaj=2e-3, L=10e-3, nut_af=7e-3, nut_h=3.2e-3, clearance=10e-6,
    grid_dims=(128, 128, 128), h=0.1e-3, origin=(-6.35e-3, -6.35e-3, -1.35e-3),
    n_theta=100, n_z=80, z_range=(0.0, 6e-3), lateral=20e-6)
M8_192 = NutBoltSpec(
    name="m8", P=1.25e-3, Rmaj=4e-3, L=20e-3, nut_af=13e-3, nut_h=6.5e-3, clearance=15e-6,
    grid_dims=(192, 192, 192), h=0.125e-3, origin=(-11.9375e-3, -11.9375e-3, -2.0e-3),
    n_theta=160, n_z=150, z_range=(0.0, 12e-3), lateral=30e-6)
M16_256 = NutBoltSpec(
    name="m16c", P=2e-3, Rmaj=8e-3, L=40e-3, nut_af=24e-3, nut_h=13e-3, clearance=25e-6,
    grid_dims=(256, 256, 256), h=0.18e-3, origin=(-22.95e-3, -22.95e-3, -3.0e-3),
    n_theta=240, n_z=250, z_range=(0.0, 25e-3), lateral=50e-6)


@dataclass(frozen=True)
class PegSpec:
    name: str
    kind: str  # 'round' | 'rect'
    block_half: tuple
    hole: float  # hole radius (round) or hole half-width (rect)
    clearance: float
    peg_len: float
    grid_dims: tuple
    h: float
    origin: tuple


ROUND_PEG_64 = PegSpec(name="round_peg", kind="round", block_half=(10e-3, 10e-3, 10e-3), hole=4e-3,
                       clearance=50e-6, peg_len=20e-3, grid_dims=(64, 64, 64), h=0.4e-3,
                       origin=(-12.6e-3, -12.6e-3, -12.6e-3))
RECT_PEG_96 = PegSpec(name="rect_peg", kind="rect", block_half=(12e-3, 12e-3, 12e-3), hole=4e-3,
                      clearance=50e-6, peg_len=24e-3, grid_dims=(96, 96, 96), h=0.3e-3,
                      origin=(-14.25e-3, -14.25e-3, -14.25e-3))


def _cache_dir():
    d = os.environ.get("FC_WORKLOAD_CACHE")
    if d:
        os.makedirs(d, exist_ok=True)
    return d


@functools.lru_cache(maxsize=8)
def bolt_grid(spec: NutBoltSpec) -> Grid:
    d = _cache_dir()
    path = None
    if d:
        path = os.path.join(d, f"bolt_{spec.name}_{'x'.join(map(str, spec.grid_dims))}_v{GEN_VERSION}.npy")
        if os.path.exists(path):
            return Grid(values=np.load(path, allow_pickle=False), dtype="f32",
                        origin=tuple(f32(v) for v in spec.origin), h=f32(spec.h))
    g = sample_grid(lambda p: field_bolt(p, spec.P, spec.Rmaj, spec.L), spec.grid_dims, spec.origin, spec.h)
    if path:
        np.save(path, g.values)
    return g


@functools.lru_cache(maxsize=8)
def nut_mesh(spec: NutBoltSpec) -> Mesh:
    return hex_nut(spec.P, spec.Rmaj, spec.clearance, spec.nut_h, spec.nut_af, spec.n_theta, spec.n_z)


@functools.lru_cache(maxsize=4)
def peg_parts(spec: PegSpec):
    if spec.kind == "round":
        fn = lambda p: field_round_hole_block(p, spec.block_half, spec.hole)  # noqa: E731
        mesh = round_peg(spec.hole - spec.clearance, spec.peg_len, 32, 28, 3)
    else:
        fn = lambda p: field_rect_hole_block(p, spec.block_half, (spec.hole, spec.hole))  # noqa: E731
        hw = spec.hole - spec.clearance
        mesh = rect_peg(hw, hw, spec.peg_len, 16)
    return sample_grid(fn, spec.grid_dims, spec.origin, spec.h), mesh


def nut_bolt_poses(spec: NutBoltSpec, rng, n):
    z = rng.uniform(spec.z_range[0], spec.z_range[1], n)
    twist = 2.0 * math.pi * z / spec.P + np.deg2rad(rng.uniform(-spec.twist_deg, spec.twist_deg, n))
    xy = rng.uniform(-spec.lateral, spec.lateral, (2, n))
    return quat_about_z(twist), np.concatenate([xy, z[None]], axis=0)


def peg_poses(spec: PegSpec, rng, n):
    """Peg axis along -z into the hole from the top face; depth U[0, L/2]."""
    top = spec.block_half[2]
    depth = rng.uniform(0.0, 0.5 * spec.peg_len, n)
    jit = rng.uniform(-2.0 * spec.clearance, 2.0 * spec.clearance, (2, n))
    # peg local z in [0, L] points up; its bottom end goes to top - depth
    t = np.concatenate([jit, (top - depth)[None]], axis=0)
    ang = np.deg2rad(rng.uniform(-0.5, 0.5, n))
    return quat_about_z(ang), t


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------


def torus_workload(seed=1000, n_env=256, K=16, level=4) -> Workload:
    """Torus R=2 cm, r=0.5 cm on a 64^3 grid (h = 1 mm); icosphere r = 1 cm."""
    rng = np.random.default_rng(seed)
    g = sample_grid(lambda p: field_torus(p, 0.02, 0.005), (64, 64, 64), (-0.0315,) * 3, 1e-3)
    m = icosphere(level, 0.01)
    q = shoemake_quat(rng, n_env)
    t = rng.uniform(-0.015, 0.015, (3, n_env))
    return Workload(name="torus64-icosphere", grids=[g], meshes=[m],
                    env_grid=np.zeros(n_env, np.int32), env_mesh=np.zeros(n_env, np.int32),
                    pose=pack_pose(q, t), bins=fibonacci_bins(K), margin=0.0,
                    meta=dict(seed=seed, gen=GEN_VERSION))


def torus_tube_workload(seed=1005, n_env=32, K=16) -> Workload:
    """The torus grid above with a small icosphere (r = 3 mm, 642 vertices)
    inside its tube: centres on the tube's core circle (R = 2 cm) jittered by
    +-1 mm, uniform random rotations.  Every vertex penetrates, 1-3 mm deep,
    so with a narrow band of 1.5 mm many fall in bricks of the sparse grid
    that are not stored."""
    rng = np.random.default_rng(seed)
    g = sample_grid(lambda p: field_torus(p, 0.02, 0.005), (64, 64, 64), (-0.0315,) * 3, 1e-3)
    m = icosphere(3, 0.003)
    a = rng.uniform(0.0, 2.0 * math.pi, n_env)
    t = np.stack([0.02 * np.cos(a), 0.02 * np.sin(a), np.zeros(n_env)]) + rng.uniform(-1e-3, 1e-3, (3, n_env))
    q = shoemake_quat(rng, n_env)
    return Workload(name="torus64-tube-icosphere", grids=[g], meshes=[m],
                    env_grid=np.zeros(n_env, np.int32), env_mesh=np.zeros(n_env, np.int32),
                    pose=pack_pose(q, t), bins=fibonacci_bins(K), margin=0.0,
                    meta=dict(seed=seed, gen=GEN_VERSION))


def nut_bolt_workload(seed=1001, n_env=1000, K=32, spec: NutBoltSpec = M16_BOLT_256x256x512) -> Workload:
    """n_env nuts threaded onto one shared bolt grid (one SDF, one mesh)."""
    rng = np.random.default_rng(seed)
    g = bolt_grid(spec)
    m = nut_mesh(spec)
    q, t = nut_bolt_poses(spec, rng, n_env)
    return Workload(name=f"nutbolt-{spec.name}", grids=[g], meshes=[m],
                    env_grid=np.zeros(n_env, np.int32), env_mesh=np.zeros(n_env, np.int32),
                    pose=pack_pose(q, t), bins=fibonacci_bins(K), margin=0.0,
                    meta=dict(seed=seed, gen=GEN_VERSION, spec=spec.name))


MIXED_TYPES = ("round_peg", "rect_peg", "m4", "m8", "m16c")


def mixed_workload(seed=1002, n_env=4096, K=32, types=MIXED_TYPES) -> Workload:
    """Uneven batch: part type per env drawn uniformly from ``types``."""
    rng = np.random.default_rng(seed)
    specs = {"round_peg": ROUND_PEG_64, "rect_peg": RECT_PEG_96, "m4": M4_128, "m8": M8_192, "m16c": M16_256}
    grids, meshes = [], []
    for name in types:
        s = specs[name]
        if isinstance(s, PegSpec):
            g, m = peg_parts(s)
        else:
            g, m = bolt_grid(s), nut_mesh(s)
        grids.append(g)
        meshes.append(m)
    typ = rng.integers(0, len(types), n_env).astype(np.int32)
    q = np.zeros((4, n_env))
    t = np.zeros((3, n_env))
    for ti, name in enumerate(types):
        sel = np.nonzero(typ == ti)[0]
        s = specs[name]
        if isinstance(s, PegSpec):
            qq, tt = peg_poses(s, rng, len(sel))
        else:
            qq, tt = nut_bolt_poses(s, rng, len(sel))
        q[:, sel], t[:, sel] = qq, tt
    return Workload(name="mixed5", grids=grids, meshes=meshes, env_grid=typ.copy(), env_mesh=typ.copy(),
                    pose=pack_pose(q, t), bins=fibonacci_bins(K), margin=0.0,
                    meta=dict(seed=seed, gen=GEN_VERSION, types=list(types)))


def subset(w: Workload, envs) -> Workload:
    """The same workload restricted to the listed envs (order kept)."""
    envs = np.asarray(envs, dtype=np.int64)
    return Workload(name=f"{w.name}[{len(envs)}]", grids=w.grids, meshes=w.meshes,
                    env_grid=np.ascontiguousarray(w.env_grid[envs]), env_mesh=np.ascontiguousarray(w.env_mesh[envs]),
                    pose=np.ascontiguousarray(w.pose[:, envs]), bins=w.bins, margin=w.margin, meta=dict(w.meta))


def half_storage(w: Workload, dtype: str) -> Workload:
    """The same workload with every grid stored in 'f16' or 'bf16'."""
    return convert_workload(w, dtype)
