"""Shared helpers of the adjoint parity tests: FP32 error bounds of the
penalty adjoint per env, the element-wise check against the FP64 oracle
(each env with its own grid and mesh), the split of a shared vertex
gradient into its per-mesh blocks, and the check against FP64 central
finite differences."""
import math

import numpy as np

import itertools

from _gpu_common import FACE_BAND, ULP32, gradient_sensitivity, oracle_rows, position_error_voxels, to_np, torch_gpu
from oracle import adjoint as OA
from oracle import query as OQ
from paper_2205_03532_amd import fc

KP = 1e4


def face_slack(w, o, k, sampler_of=None):
    """Per-row allowances for points within the FP32 position error of a cell
    face: the kernel may take the cell on either side, where the trilinear
    field's gradient jumps (and a sparse field's value may jump too).  The
    point is nudged across every near face (all sign combinations of the
    near axes) and the whole difference of its loss term, w = k phi grad and
    moment x_B x w between the sides is allowed.  ``sampler_of(e)`` gives
    env e's field (default: the dense interpolant of its grid)."""
    n = len(o["phi"])
    out = {key: np.zeros(n) for key in ("loss", "w", "mom")}
    du = np.max(position_error_voxels(o), axis=1)
    band = np.maximum(FACE_BAND, 2.0 * du)[:, None]
    t = o["u"] - np.floor(o["u"])
    near = ((t < band) | (t > 1.0 - band)) & o["inside"][:, None]
    idx = np.nonzero(near.any(axis=1))[0]
    if not len(idx):
        return out

    def terms(phi, grad):
        act = np.isfinite(phi) & (np.nan_to_num(phi, nan=1.0) < 0)
        p = np.where(act, phi, 0.0)
        return 0.5 * k * p ** 2, k * p[:, None] * np.where(act[:, None], grad, 0.0)

    t0, w0 = terms(o["phi"][idx], o["grad"][idx])
    x0 = o["x_b"][idx]
    h = o["h"][idx][:, None]
    env = o["env"][idx]
    samplers, dense = {}, {}
    for e in np.unique(env):
        if sampler_of is not None:
            samplers[e] = sampler_of(int(e))
        else:
            gi = int(w.env_grid[e])
            if gi not in dense:
                dense[gi] = OA.dense_sampler(w.grids[gi])
            samplers[e] = dense[gi]
    for sgn in itertools.product((-1.0, 0.0, 1.0), repeat=3):
        step = np.asarray(sgn)[None, :] * near[idx] * (2.0 * band[idx] * h)
        if not step.any():
            continue
        phi = np.full(len(idx), np.nan)
        grad = np.zeros((len(idx), 3))
        for e in np.unique(env):
            sel = env == e
            phi[sel], grad[sel], _, _ = samplers[e](x0[sel] + step[sel])
        t1, w1 = terms(phi, grad)
        dw = np.linalg.norm(w1 - w0, axis=1)
        out["loss"][idx] = np.maximum(out["loss"][idx], np.abs(t1 - t0))
        out["w"][idx] = np.maximum(out["w"][idx], dw)
        out["mom"][idx] = np.maximum(out["mom"][idx], np.linalg.norm(x0, axis=1) * dw)
    return out


def adjoint_bounds(w, envs, k, o=None, S=None, cmax=None, extra_ulps=0.0, row_slack=None, sampler_of=None):
    """FP32 error bounds of the adjoint per env, from the oracle's per-vertex data.

    Per vertex: dx <= position rounding (m); dphi <= |g| dx + 4 ulp(cmax) (lerp
    rounding); dgrad <= (sqrt(3) S du + 8 ulp cmax) / h; for a penetrating
    vertex dw <= k (dphi |g| + |phi| dgrad) + 3 ulp |w|.  A vertex with
    |phi| <= dphi may be penetrating on one side only: its whole term,
    k (|phi| + dphi)(|g| + dgrad), is allowed.

    ``o`` overrides the oracle rows (another field's phi and grad), ``S`` and
    ``cmax`` the cell data of gradient_sensitivity (e.g. corners the kernel
    synthesises), ``extra_ulps`` adds that many ulps of cmax to the corner
    rounding (for corners that are themselves computed in FP32).
    ``row_slack`` adds per-row allowances {"loss", "w", "mom"}; the rows near a
    cell face always get face_slack's (with ``sampler_of`` as the field).
    """
    o = oracle_rows(w, envs) if o is None else o
    du = np.max(position_error_voxels(o), axis=1)
    dx = du * o["h"]
    if S is None:
        S, cmax = gradient_sensitivity(w, o)
    g = np.linalg.norm(o["grad"], axis=1)
    phi_all = np.nan_to_num(o["phi"], nan=1.0)
    act = o["inside"] & (phi_all < 0)
    dphi = g * dx + (4 + extra_ulps) * ULP32 * cmax
    near0 = o["inside"] & (np.abs(phi_all) <= dphi)
    phi = np.where(act | near0, phi_all, 0.0)
    dgrad = (math.sqrt(3) * S * du + (8 + 2 * extra_ulps) * ULP32 * cmax) / o["h"]
    wabs = k * np.abs(phi) * g
    dw = np.where(act, k * (dphi * g + np.abs(phi) * dgrad) + 3 * ULP32 * wabs, 0.0)
    dw = np.where(near0, k * (np.abs(phi) + dphi) * (g + dgrad), dw)
    xb = np.linalg.norm(o["x_b"], axis=1)
    dloss = np.where(act, k * np.abs(phi) * dphi + 2 * ULP32 * 0.5 * k * phi ** 2, 0.0)
    dloss = np.where(near0, 0.5 * k * (np.abs(phi) + dphi) ** 2, dloss)
    dmom = np.where(act | near0, xb * dw + wabs * dx + 3 * ULP32 * xb * wabs, 0.0)
    fs = face_slack(w, o, k, sampler_of)
    dloss, dw, dmom = dloss + fs["loss"], dw + fs["w"], dmom + fs["mom"]
    if row_slack is not None:
        dloss = dloss + row_slack["loss"]
        dw = dw + row_slack["w"]
        dmom = dmom + row_slack["mom"]
    out = {}
    for e in envs:
        sel = o["env"] == e
        out[e] = dict(loss=dloss[sel].sum(), rho=dw[sel].sum(), omega=dmom[sel].sum(), verts=dw[sel],
                      abs_terms=(0.5 * k * phi[sel] ** 2).sum() + wabs[sel].sum() * (1 + xb[sel].max()))
    return out


def run_backward(batch, pose, per_env, upstream=None):
    torch = torch_gpu()
    g = batch.new_grads(per_env=per_env)
    fc.fc_sdf_query_backward(batch, pose, KP, g, upstream=upstream)
    torch.cuda.synchronize()
    return to_np({k: v for k, v in g.items() if k != "per_env"})


def check_vs_oracle(w, res, envs, per_env, penalty=None, bounds=None):
    """Per env (its own grid and mesh): loss, twist and (per-env mode) vertex
    gradients within the FP32 bounds of the FP64 oracle.  Returns, per mesh,
    the oracle's sum of the checked envs' vertex gradients and its bound, and
    the largest twist error over its bound.  ``penalty(e)`` overrides the
    oracle call (e.g. another field sampler), ``bounds`` the error bounds."""
    bounds = adjoint_bounds(w, envs, KP) if bounds is None else bounds
    off = w.env_query_offsets()
    vals = {}
    meshes = sorted({int(w.env_mesh[e]) for e in envs})
    shared = {m: np.zeros((w.meshes[m].n, 3)) for m in meshes}
    shared_tol = {m: np.zeros(w.meshes[m].n) for m in meshes}
    worst = 0.0
    for e in envs:
        gi, mi = int(w.env_grid[e]), int(w.env_mesh[e])
        g = w.grids[gi]
        if penalty is not None:
            L, dxi, dv = penalty(e)
        else:
            if gi not in vals:
                vals[gi] = OQ.grid_values_f64(g.values, g.dtype)
            L, dxi, dv = OA.penalty_env(g, w.meshes[mi].verts, w.pose[:, e], KP, vals[gi])
        b = bounds[e]
        slack = 1e-6 * b["abs_terms"] + 1e-12
        assert abs(res["loss"][e] - L) <= 2 * b["loss"] + slack, (e, res["loss"][e], L, b["loss"])
        for i in range(3):
            assert abs(res["d_pose"][i, e] - dxi[i]) <= 2 * b["rho"] + slack, (e, i)
            assert abs(res["d_pose"][3 + i, e] - dxi[3 + i]) <= 2 * b["omega"] + slack, (e, 3 + i)
        worst = max(worst, np.max(np.abs(res["d_pose"][:, e] - dxi)) / (2 * max(b["rho"], b["omega"]) + slack))
        if per_env:
            gv = res["d_verts"].reshape(3, -1)[:, off[e]:off[e + 1]].T
            err = np.abs(gv - dv)
            tolv = 2 * b["verts"][:, None] + 1e-9
            if not np.all(err <= tolv):
                r = int(np.argmax(np.max(err / tolv, axis=1)))
                raise AssertionError(f"env {e} vertex {r}: gpu {gv[r]} oracle {dv[r]} bound {tolv[r, 0]:.3e}")
        shared[mi] += dv
        shared_tol[mi] += 2 * b["verts"]
    return shared, shared_tol, worst


def shared_blocks(w, d_verts):
    """Split a shared-mode d_verts into its per-mesh [n_verts][3] blocks
    (blocks in mesh order, each [3][n_verts])."""
    out, o = [], 0
    for m in w.meshes:
        out.append(d_verts[o:o + 3 * m.n].reshape(3, m.n).T)
        o += 3 * m.n
    assert o == len(d_verts)
    return out


def check_fd(w, res, envs, bounds=None, sampler_of=None, h=1e-6, jumps=False):
    """Twist and vertex gradients (per-env mode results) against FP64 central
    differences of the loss, each env on its own grid and mesh: kink-free
    components within 1e-3 relative plus the FP32 bound, components with a
    cell or sign crossing within their computed jump bound besides.
    ``sampler_of(e)`` gives another field's sampler, ``jumps`` says that
    field may jump in value across cell faces.  Returns the counts of
    smooth and kinked twist components."""
    bounds = adjoint_bounds(w, envs, KP) if bounds is None else bounds
    n_kinked = n_smooth = 0
    off = w.env_query_offsets()
    vals = {}
    for e in envs:
        gi, mi = int(w.env_grid[e]), int(w.env_mesh[e])
        g, verts = w.grids[gi], w.meshes[mi].verts
        if sampler_of is not None:
            smp = sampler_of(e)
        else:
            if gi not in vals:
                vals[gi] = OQ.grid_values_f64(g.values, g.dtype)
            smp = OA.dense_sampler(g, vals[gi])
        gfd, cross, kb = OA.fd_twist(g, verts, w.pose[:, e], KP, h, sampler=smp, jumps=jumps)
        ref = np.max(np.abs(gfd))
        for i in range(6):
            fp32 = 2 * (bounds[e]["rho"] if i < 3 else bounds[e]["omega"])
            tol = 1e-3 * max(abs(gfd[i]), 1e-3 * ref) + kb[i] + fp32 + 1e-9
            assert abs(res["d_pose"][i, e] - gfd[i]) <= tol, (e, i, res["d_pose"][i, e], gfd[i], cross[i], kb[i])
            n_kinked += int(cross[i] > 0)
            n_smooth += int(cross[i] == 0)
        # vertex gradients: smooth coordinates only (each vertex's own term)
        gv, crossed = OA.fd_verts(g, verts, w.pose[:, e], KP, h, sampler=smp)
        dv = res["d_verts"].reshape(3, -1)[:, off[e]:off[e + 1]].T
        ok = ~crossed
        tolv = 1e-3 * np.abs(gv) + 2 * bounds[e]["verts"][:, None] + 1e-7
        assert np.all(np.abs(dv - gv)[ok] <= tolv[ok]), e
    return n_smooth, n_kinked
