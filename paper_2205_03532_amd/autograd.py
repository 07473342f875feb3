"""torch.autograd.Function around the hand-written adjoint kernel.

``SdfPenalty.apply(batch, pose, xi, k, *mesh_vertices)`` returns the per-env
penetration penalty L_e = sum over vertices with phi < 0 of 0.5 k phi^2
(forward: ``fc_sdf_query_backward`` with only the loss requested).  Its
backward calls the same kernel with the upstream gradient and returns:

  * for ``xi`` (n_env, 6): dL/dxi at xi = 0 for the left twist
    T <- exp(xi^) T, xi = (rho, omega) -- the twist is a probe that receives
    the pose gradient; its value must be zero (checked);
  * for each mesh vertex tensor (3, n_m): the vertex gradient summed over
    the envs that use that mesh, in a fixed order.

``mesh_vertices`` must be the batch's own device vertex tensors
(``batch.mesh_tensors``): the kernels read them in place.
"""
from __future__ import annotations

import torch

from . import fc


class SdfPenalty(torch.autograd.Function):
    @staticmethod
    def forward(ctx, batch, pose, xi, k, *mesh_vertices):
        if len(mesh_vertices) != len(batch.mesh_tensors):
            raise ValueError("pass every mesh vertex tensor of the batch")
        for a, b in zip(mesh_vertices, batch.mesh_tensors):
            if a.data_ptr() != b.data_ptr():
                raise ValueError("mesh_vertices must be the batch's own vertex tensors")
        if xi.shape != (batch.n_env, 6):
            raise ValueError("xi must be (n_env, 6)")
        if torch.count_nonzero(xi).item() != 0:
            raise ValueError("xi must be zero: it only receives dL/dxi at xi = 0")
        g = batch.new_grads(loss=True, d_pose=False, d_verts=False)
        fc.fc_sdf_query_backward(batch, pose, k, g)
        ctx.batch, ctx.k = batch, float(k)
        ctx.save_for_backward(pose)
        return g["loss"]

    @staticmethod
    def backward(ctx, g_loss):
        (pose,) = ctx.saved_tensors
        batch = ctx.batch
        g = batch.new_grads(per_env=False, loss=False, d_pose=True, d_verts=True)
        up = g_loss.detach().to(torch.float32).contiguous()
        fc.fc_sdf_query_backward(batch, pose, ctx.k, g, upstream=up)
        d_xi = g["d_pose"].t().contiguous()
        outs = []
        off = 0
        for n in batch.mesh_sizes:
            outs.append(g["d_verts"][off:off + 3 * n].view(3, n))
            off += 3 * n
        return (None, None, d_xi, None, *outs)


def penalty(batch, pose, k, xi=None):
    """Per-env penalty with autograd to ``xi`` and the batch's vertex tensors."""
    if xi is None:
        xi = torch.zeros(batch.n_env, 6, device=batch.device, requires_grad=True)
    return SdfPenalty.apply(batch, pose, xi, k, *batch.mesh_tensors), xi
