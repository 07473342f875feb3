"""The pins have teeth: each plausible mistake planted in the oracle (on the
CPU, by monkeypatching) makes at least one pin fail."""
import numpy as np
import pytest

import test_oracle_pins as P
from oracle import adjoint as OA
from oracle import query as OQ
from oracle import reduce as ORD

PINS = [
    P.test_rotation_matches_scipy,
    P.test_rotation_quarter_turn_about_z,
    P.test_transform_identity_and_translation_exact,
    lambda: P.test_trilinear_reproduces_q1_fields(0),
    P.test_node_reproduction_and_far_boundary,
    P.test_outside_points_are_not_inside,
    P.test_upper_cell_on_shared_face,
    P.test_sphere_within_interpolation_bound,
    P.test_box_exact_in_face_regions,
    P.test_halfspace_contacts_closed_form,
    P.test_bin_tie_goes_to_lowest_k_and_zero_normal_to_bin0,
    lambda: P.test_reduce_matches_bruteforce_and_is_order_free(0),
    P.test_reduce_signed_zero_and_empty,
    P.test_penalty_halfspace_closed_form,
    P.test_penalty_gradient_matches_finite_differences,
]


def some_pin_fails():
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            return True
        except Exception:  # a crash also counts as caught
            return True
    return False


def test_unmutated_oracle_passes_every_pin():
    assert not some_pin_fails()


_orig_tri = OQ.trilinear_value_grad
_orig_rot = OQ.rotation_from_quaternion
_orig_locate = OQ.locate


def tri_swap_xy(vals, cell, t, h):
    t2 = t.copy()
    t2[..., [0, 1]] = t2[..., [1, 0]]
    return _orig_tri(vals, cell, t2, h)


def tri_drop_corner(vals, cell, t, h):
    phi, g = _orig_tri(vals, cell, t, h)
    ix, iy, iz = cell[..., 0], cell[..., 1], cell[..., 2]
    w = t[..., 0] * t[..., 1] * t[..., 2]
    return phi - w * vals[iz + 1, iy + 1, ix + 1], g


def tri_grad_sign(vals, cell, t, h):
    phi, g = _orig_tri(vals, cell, t, h)
    return phi, -g


def tri_grad_unscaled(vals, cell, t, h):
    phi, g = _orig_tri(vals, cell, t, h)
    return phi, g * h


def rot_transposed(q):
    return _orig_rot(q).T


def locate_no_clamp(x, origin, h, dims):
    inside, cell, t = _orig_locate(x, origin, h, dims)
    u = (np.asarray(x, dtype=np.float64) - np.asarray(origin)) / h
    us = np.where(inside[..., None], u, 0.0)
    cell2 = np.minimum(np.floor(us), np.asarray(dims) - 1.0)  # forgets the n-2 clamp
    return inside, cell2.astype(np.int64), us - cell2


def locate_lower_cell(x, origin, h, dims):
    inside, cell, t = _orig_locate(x, origin, h, dims)
    on_face = (t == 0.0) & (cell > 0)
    cell = np.where(on_face, cell - 1, cell)
    t = np.where(on_face, 1.0, t)
    return inside, cell, t


_orig_reduce = ORD.reduce_contacts


def reduce_highest_index(env, vidx, depth32, bins, cand, n_env, K):
    return _orig_reduce(env, -np.asarray(vidx), depth32, bins, cand, n_env, K)


_orig_pen = OA.penalty_env


def penalty_cross_sign(grid, verts, pose, k, vals64=None, sampler=None):
    L, dxi, dv = _orig_pen(grid, verts, pose, k, vals64, sampler)
    dxi = dxi.copy()
    dxi[3:] = -dxi[3:]
    return L, dxi, dv


_orig_nb = OQ.normals_and_bins


def bins_highest_on_tie(grad, bins):
    n, b, dots = _orig_nb(grad, bins)
    K = dots.shape[-1]
    return n, (K - 1 - np.argmax(dots[..., ::-1], axis=-1)).astype(np.int64), dots


MUTATIONS = [
    (OQ, "trilinear_value_grad", tri_swap_xy),
    (OQ, "trilinear_value_grad", tri_drop_corner),
    (OQ, "trilinear_value_grad", tri_grad_sign),
    (OQ, "trilinear_value_grad", tri_grad_unscaled),
    (OQ, "rotation_from_quaternion", rot_transposed),
    (OQ, "locate", locate_no_clamp),
    (OQ, "locate", locate_lower_cell),
    (ORD, "reduce_contacts", reduce_highest_index),
    (OA, "penalty_env", penalty_cross_sign),
    (OQ, "normals_and_bins", bins_highest_on_tie),
]


@pytest.mark.parametrize("mod,name,fn", MUTATIONS, ids=[m[2].__name__ for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, mod, name, fn):
    monkeypatch.setattr(mod, name, fn)
    assert some_pin_fails(), f"no pin catches {fn.__name__}"
