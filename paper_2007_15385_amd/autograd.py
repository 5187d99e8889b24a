"""Differentiable collision cost (forward and hand-written backward run in
the library's HIP kernels; this module only marshals tensors)."""
from __future__ import annotations

import torch

from .api import _check, _dev, _lib, _stream, context


def _footprint(F):
    if F.dtype != torch.float32 or F.dim() != 2 or F.shape[1] != 2:
        raise ValueError("footprint must be a float32 tensor of shape [n, 2]")
    return F.contiguous()


def _poses(poses):
    if poses.dtype != torch.float32 or poses.shape[-1] != 3:
        raise ValueError("poses must be a float32 tensor of shape [..., 3]")
    return poses.reshape(-1, 3).contiguous()


def _points(Q):
    if Q.dtype != torch.float32 or Q.dim() != 2 or Q.shape[1] != 2:
        raise ValueError("points must be a float32 tensor of shape [m, 2]")
    return Q.contiguous()


def cost_workspace_bytes(n: int, K: int, m: int) -> int:
    return int(_lib().pip_cost_workspace_bytes(int(n), int(K), int(m)))


def pip_cost_fwd(footprint, poses, points, workspace=None):
    """Cost per pose ([K] float32 for poses of shape [K, 3])."""
    F, P, Q = _footprint(footprint), _poses(poses), _points(points)
    d = _dev(F)
    n, K, m = F.shape[0], P.shape[0], Q.shape[0]
    need = cost_workspace_bytes(n, K, m)
    if need == 0:
        raise ValueError(f"unsupported footprint size n = {n}")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=F.device)
    cost = torch.empty(max(K, 1), dtype=torch.float32, device=F.device)
    ctx = context(d)
    s = _lib().pip_cost_fwd(ctx, F.data_ptr(), n, P.data_ptr() if K else None, K,
                            Q.data_ptr() if m else None, m, cost.data_ptr(), workspace.data_ptr(),
                            workspace.numel(), _stream(d))
    _check(s, "pip_cost_fwd", ctx)
    return cost[:K]


def pip_cost_bwd(footprint, poses, points, grad_cost, workspace=None):
    """(grad_pose [K, 3], grad_footprint [n, 2], residual [2])."""
    F, P, Q = _footprint(footprint), _poses(poses), _points(points)
    d = _dev(F)
    n, K, m = F.shape[0], P.shape[0], Q.shape[0]
    g = grad_cost.reshape(-1).to(torch.float32).contiguous()
    if g.numel() != K:
        raise ValueError("grad_cost must have one entry per pose")
    need = cost_workspace_bytes(n, K, m)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=F.device)
    gp = torch.empty((max(K, 1), 3), dtype=torch.float32, device=F.device)
    gF = torch.empty((n, 2), dtype=torch.float32, device=F.device)
    res = torch.empty(2, dtype=torch.float32, device=F.device)
    ctx = context(d)
    s = _lib().pip_cost_bwd(ctx, F.data_ptr(), n, P.data_ptr() if K else None, K,
                            Q.data_ptr() if m else None, m, g.data_ptr() if K else None,
                            gp.data_ptr(), gF.data_ptr(), res.data_ptr(), workspace.data_ptr(),
                            workspace.numel(), _stream(d))
    _check(s, "pip_cost_bwd", ctx)
    return gp[:K], gF, res


class CollisionCost(torch.autograd.Function):
    """cost[...] = sum over points of relu(min over edges of the normalized
    Voronoi margin) for each pose in poses[..., 3]; differentiable with
    respect to the poses and the footprint vertices."""

    @staticmethod
    def forward(ctx, poses, footprint, points):
        cost = pip_cost_fwd(footprint, poses, points)
        ctx.save_for_backward(poses, footprint, points)
        ctx.pose_shape = poses.shape
        return cost.reshape(poses.shape[:-1])

    @staticmethod
    def backward(ctx, grad_cost):
        poses, footprint, points = ctx.saved_tensors
        gp, gF, _ = pip_cost_bwd(footprint, poses, points, grad_cost)
        gpose = gp.reshape(ctx.pose_shape) if ctx.needs_input_grad[0] else None
        gfoot = gF if ctx.needs_input_grad[1] else None
        return gpose, gfoot, None


def collision_cost(poses, footprint, points):
    return CollisionCost.apply(poses, footprint, points)
