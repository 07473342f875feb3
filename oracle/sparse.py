"""FP64 reference of the narrow-band sparse grid (test infrastructure only).

Section VII names sparse SDF representations as the way to cut an SDF's
memory footprint; the paper gives no scheme.  Readings (listed with the
others in the design notes):
  * the grid is cut into bricks of 3 x 3 x 3 cells (4 x 4 x 4 nodes, brick b
    covering cells 3b .. 3b + 2 on each axis, neighbours sharing face nodes);
  * a brick is stored iff one of its nodes has |value| <= band, its nodes
    have both signs (value < 0 and value >= 0), or it reaches past the grid's
    last node on some axis (3b + 3 > n - 1);
  * a point whose cell lies in a stored brick takes the dense trilinear
    interpolant (value and gradient) of the grid;
  * a point whose cell lies in a brick that is not stored takes the trilinear
    interpolant of that brick's 8 corner nodes, the coarse grid of spacing 3h
    through nodes 3b: local coordinates (u - 3b) / 3, gradient per metre
    with 3h as the spacing.
"""
from __future__ import annotations

import numpy as np

from . import query as Q


def brick_counts(dims):
    """Bricks per axis (bx, by, bz) of a grid with dims (nx, ny, nz)."""
    return tuple(-(-(int(n) - 1) // 3) for n in dims)


def brick_stored(vals64, band, bricks):
    """Stored flag of each brick (rows of bricks: (bx, by, bz) indices);
    vals64 is the decoded grid [nz][ny][nx], band the narrow band (the same
    number the library compares with)."""
    nz, ny, nx = vals64.shape
    b = np.asarray(bricks, dtype=np.int64).reshape(-1, 3)
    n = np.array([nx, ny, nz])
    partial = np.any(3 * b + 3 > n - 1, axis=1)
    k = np.arange(4)
    x = np.minimum(3 * b[:, 0, None] + k, nx - 1)  # (m, 4); clamped nodes only matter for partial bricks
    y = np.minimum(3 * b[:, 1, None] + k, ny - 1)
    z = np.minimum(3 * b[:, 2, None] + k, nz - 1)
    block = vals64[z[:, :, None, None], y[:, None, :, None], x[:, None, None, :]]  # (m, 4, 4, 4)
    flat = block.reshape(len(b), -1)
    near = np.min(np.abs(flat), axis=1) <= np.float64(band)
    mixed = np.any(flat < 0.0, axis=1) & np.any(flat >= 0.0, axis=1)
    return partial | near | mixed


def coarse_interpolant(vals64, cell, t, h):
    """Value and gradient (per metre) of the trilinear interpolant of the
    8 corner nodes of the brick holding each cell: the coarse grid of
    nodes 3i (spacing 3h), local coordinates (u - 3b) / 3.  Meaningful for
    full bricks (the only ones that can be left unstored)."""
    b = cell // 3
    coarse = vals64[::3, ::3, ::3]
    coarse = np.pad(coarse, [(0, max(0, 2 - n)) for n in coarse.shape], mode="edge")  # tiny grids: unused
    cz, cy, cx = coarse.shape
    bc = np.minimum(b, np.array([cx - 2, cy - 2, cz - 2]))  # partial bricks: any valid cell, unused
    tc = ((cell + t) - 3.0 * bc) / 3.0
    return Q.trilinear_value_grad(coarse, bc, tc, 3.0 * np.float64(h))


def sample_sparse(vals64, origin, h, dims, x, band):
    """phi, grad (per metre), inside, stored-brick flag at B-frame points
    (NaN phi outside the grid), under the readings above."""
    inside, cell, t = Q.locate(x, origin, h, dims)
    b = cell // 3
    stored = brick_stored(vals64, band, b.reshape(-1, 3)).reshape(b.shape[:-1])
    phi, grad = Q.trilinear_value_grad(vals64, cell, t, h)
    pc, gc = coarse_interpolant(vals64, cell, t, h)
    phi = np.where(stored, phi, pc)
    grad = np.where(stored[..., None], grad, gc)
    phi = np.where(inside, phi, np.nan)
    grad = np.where(inside[..., None], grad, 0.0)
    return phi, grad, inside, stored


def sparse_sampler(vals64, origin, h, dims, band):
    """x -> (phi, grad, inside, cell) of the sparse field above (the fine cell
    is returned as the cell), for the penalty adjoint and its differences."""

    def f(x):
        phi, grad, inside, _ = sample_sparse(vals64, origin, h, dims, x, band)
        _, cell, _ = Q.locate(x, origin, h, dims)
        return phi, grad, inside, cell

    return f
