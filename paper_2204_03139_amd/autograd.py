"""torch.autograd.Function over the C ABI: sampling (Eq. 3) + Chamfer (Eq. 1/2) forward, and the
backward through the saved neighbours and Eq. 4 to the mesh vertices.

The forward saves the face choice, barycentric weights, sampled points and the neighbour index
arrays (only a -> b for the unidirectional loss, which needs nothing else); the backward never
recomputes them.
"""
from __future__ import annotations

import torch

from . import _lib


class DiffCloudChamfer(torch.autograd.Function):
    """loss[t] for a mesh trajectory verts [T,V,3] against an observed cloud [T,Nb,3].

    apply(verts, faces, observed, n_sim, seed, precision, reduction, frame_w, uniforms, face_mask)
    returns the per-frame loss [T] (float64).  Gradients flow to verts (and to observed when it
    requires grad).  face_mask (uint8 [F] or [T,F]) samples only a subset of the faces."""

    @staticmethod
    def forward(ctx, verts, faces, observed, n_sim, seed=0, precision=_lib.DC_PREC_FP32,
                reduction=_lib.DC_RED_BIDIR_MEAN, frame_w=None, uniforms=None, face_mask=None):
        v = verts.detach().contiguous()
        obs = observed.detach().contiguous()
        points, face_idx, bary = _lib.sample_surface(v, faces, n_sim, seed=seed, uniforms=uniforms,
                                                     face_mask=face_mask)
        # the unidirectional loss (Eq. 2) needs only the a -> b search
        b_side = reduction != _lib.DC_RED_SIM2REAL_SUM
        out = _lib.chamfer_fwd(points, obs, precision=precision, reduction=reduction,
                               frame_w=frame_w, b_side=b_side)
        idx_b = out["idx_b"] if b_side else torch.empty(0, dtype=torch.int32)
        ctx.save_for_backward(faces, obs, points, face_idx, bary, out["idx_a"], idx_b,
                              frame_w if frame_w is not None else torch.empty(0))
        ctx.b_side = b_side
        ctx.V = v.shape[1]
        ctx.reduction = reduction
        ctx.has_w = frame_w is not None
        ctx.mark_non_differentiable(out["idx_a"])
        return out["loss"]

    @staticmethod
    def backward(ctx, grad_loss):
        faces, obs, points, face_idx, bary, idx_a, idx_b, fw = ctx.saved_tensors
        fw = fw if ctx.has_w else None
        want_b = ctx.needs_input_grad[2]
        ga, gb = _lib.chamfer_bwd(grad_loss.detach().to(torch.float64).contiguous(), points, obs,
                                  idx_a, idx_b if ctx.b_side else None, reduction=ctx.reduction,
                                  frame_w=fw, want_b=want_b)
        gv = _lib.sample_surface_bwd(ga, faces, face_idx, bary, ctx.V)
        return gv, None, gb, None, None, None, None, None, None, None


def diffcloud_loss(verts, faces, observed, n_sim, seed=0, precision=_lib.DC_PREC_FP32,
                   reduction=_lib.DC_RED_BIDIR_MEAN, frame_w=None, uniforms=None, face_mask=None):
    """Sum over frames of the per-frame loss (a scalar, float64)."""
    return DiffCloudChamfer.apply(verts, faces, observed, n_sim, seed, precision, reduction,
                                  frame_w, uniforms, face_mask).sum()


class RigidPose(torch.autograd.Function):
    """verts [T,V,3] of rigid meshes from poses q [T,B,6] (Sec. III-C): apply(q, p0, body_start,
    base) with base [T,V,3] supplying the vertices owned by no body (or None).  The backward is
    the chain rule J^T g per body; base receives the gradient of the vertices it supplies."""

    @staticmethod
    def forward(ctx, q, p0, body_start, base=None):
        out = base.detach().clone().contiguous() if base is not None else None
        verts = _lib.rigid_pose(q.detach().contiguous(), p0, body_start, out=out)
        ctx.save_for_backward(q.detach(), p0, body_start)
        ctx.has_base = base is not None
        return verts

    @staticmethod
    def backward(ctx, grad_verts):
        q, p0, body_start = ctx.saved_tensors
        g = grad_verts.detach().to(torch.float32).contiguous()
        gq = _lib.rigid_pose_bwd(q, p0, body_start, g)
        gbase = None
        if ctx.has_base:
            owned = torch.zeros(g.shape[1], dtype=torch.bool, device=g.device)
            for s, e in zip(body_start[:-1].tolist(), body_start[1:].tolist()):
                owned[s:e] = True
            gbase = g.masked_fill(owned[None, :, None], 0.0)
        return gq.to(q.dtype), None, None, gbase
