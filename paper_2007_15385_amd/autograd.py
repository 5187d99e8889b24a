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


class CostPlan:
    """pip_cost_fwd (backward=False) or pip_cost_bwd (backward=True) bound to
    fixed buffers: autotune() times the cost with and without the
    bounding-disk cull, checks that both give the same outputs word for word
    and captures the faster in a hipGraph; launch() replays it.  The
    outputs are the attributes cost, or grad_pose, grad_footprint, residual.

    The plan binds the caller's footprint, poses, points and grad_cost
    tensors themselves (no copies): each launch reads their current values,
    so in-place updates between launches are seen.  They must therefore be
    contiguous float32 tensors (grad_cost with one entry per pose); without
    grad_cost the plan owns a tensor of ones, exposed as ``grad_cost``."""

    def __init__(self, footprint, poses, points, backward: bool = False, grad_cost=None):
        import ctypes
        for t, name in ((footprint, "footprint"), (poses, "poses"), (points, "points")):
            if not t.is_contiguous():
                raise ValueError(f"CostPlan binds the caller's {name}: pass a contiguous tensor")
        if backward and grad_cost is not None and (grad_cost.dtype != torch.float32 or
                                                   not grad_cost.is_contiguous()):
            raise ValueError("CostPlan binds the caller's grad_cost: pass a contiguous float32 tensor")
        self.F, self.P, self.Q = _footprint(footprint), _poses(poses), _points(points)
        self.device = _dev(self.F)
        n, K, m = self.F.shape[0], self.P.shape[0], self.Q.shape[0]
        dev = self.F.device
        self.backward = bool(backward)
        self.cost = None if backward else torch.zeros(max(K, 1), dtype=torch.float32, device=dev)
        self.grad_cost = None
        if backward:
            g = grad_cost if grad_cost is not None else torch.ones(K, dtype=torch.float32, device=dev)
            self.grad_cost = g.reshape(-1)  # a view of a contiguous tensor: the caller's storage
            if self.grad_cost.numel() != K:
                raise ValueError("grad_cost must have one entry per pose")
        self.grad_pose = torch.zeros((max(K, 1), 3), dtype=torch.float32, device=dev) if backward else None
        self.grad_footprint = torch.zeros((n, 2), dtype=torch.float32, device=dev) if backward else None
        self.residual = torch.zeros(2, dtype=torch.float32, device=dev) if backward else None
        self.ctx = context(self.device)
        ptr = lambda t: t.data_ptr() if t is not None else None
        h = ctypes.c_void_p()
        s = _lib().pip_plan_create_cost(self.ctx, 1 if backward else 0, self.F.data_ptr(), n,
                                        self.P.data_ptr(), K, ptr(self.Q) if m else None, m,
                                        ptr(self.cost), ptr(self.grad_cost), ptr(self.grad_pose),
                                        ptr(self.grad_footprint), ptr(self.residual),
                                        ctypes.byref(h))
        _check(s, "pip_plan_create_cost", self.ctx)
        self.handle = h.value

    def autotune(self, reps: int = 3):
        s = _lib().pip_plan_autotune(self.handle, int(reps), _stream(self.device))
        _check(s, "pip_plan_autotune", self.ctx)
        return self.config()

    def launch(self):
        s = _lib().pip_plan_launch(self.handle, _stream(self.device))
        _check(s, "pip_plan_launch", self.ctx)

    def config(self):
        import ctypes
        from ._lib import VariantConfig
        cfg = VariantConfig()
        ms = ctypes.c_float()
        s = _lib().pip_plan_variant(self.handle, ctypes.byref(cfg), ctypes.byref(ms))
        _check(s, "pip_plan_variant", self.ctx)
        return (cfg.cull, cfg.pair), float(ms.value)

    def set_config(self, cull: int, pair: int):
        import ctypes
        from ._lib import VariantConfig
        s = _lib().pip_plan_set_variant(self.handle, ctypes.byref(VariantConfig(int(cull), int(pair))))
        _check(s, "pip_plan_set_variant", self.ctx)

    def close(self):
        if getattr(self, "handle", None):
            _lib().pip_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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
