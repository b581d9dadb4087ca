"""Huber-robust reprojection cost as a torch.autograd.Function.

forward(cams [m,9], pts [n,3]) -> F = 1/2 sum rho(|e|^2)   (FP64 scalar)
backward(dF)                     -> dF * sum rho' J_c^T e, dF * sum rho' J_p^T e
                                    (dF read on the device: no host synchronisation)

Both directions run in libba's HIP kernels through the device-pointer calls
(ba_cost_fwd_device / ba_cost_bwd_device): the backward kernels recompute the
Jacobians and reduce them per camera and per point.  torch supplies device
memory and the stream only.  The observation graph (which camera sees which
point, the pixels and the Huber threshold) is the one the Problem was
created with; cams and pts are in the caller's order.
"""
from __future__ import annotations

import torch

from .native import Problem

_DTYPES = {torch.float64: 0, torch.float32: 1}


def _stream():
    return torch.cuda.current_stream().cuda_stream


class HuberReprojCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cams, pts, problem: Problem):
        if not (cams.is_cuda and pts.is_cuda):
            raise ValueError("cams and pts must be device tensors")
        if cams.dtype != pts.dtype or cams.dtype not in _DTYPES:
            raise ValueError("cams and pts must both be float32 or float64")
        if tuple(cams.shape) != (problem.m, 9) or tuple(pts.shape) != (problem.n, 3):
            raise ValueError("parameter shapes do not match the problem")
        cams = cams.contiguous()
        pts = pts.contiguous()
        out = torch.zeros((), dtype=torch.float64, device=cams.device)
        problem.cost_fwd_device(_DTYPES[cams.dtype], cams.data_ptr(), pts.data_ptr(), out.data_ptr(),
                                _stream())
        ctx.save_for_backward(cams, pts)
        ctx.problem = problem
        return out

    @staticmethod
    def backward(ctx, gout):
        cams, pts = ctx.saved_tensors
        problem = ctx.problem
        gc = torch.empty_like(cams) if ctx.needs_input_grad[0] else None
        gp = torch.empty_like(pts) if ctx.needs_input_grad[1] else None
        # the upstream gradient stays on the device: the kernels read it on the
        # stream, so backward never waits for the GPU (a temporary copy is
        # reused by torch's allocator only in the order of that stream)
        g = gout.to(device=cams.device, dtype=torch.float64).contiguous()
        problem.cost_bwd_device(_DTYPES[cams.dtype], cams.data_ptr(), pts.data_ptr(), 1.0,
                                None if gc is None else gc.data_ptr(),
                                None if gp is None else gp.data_ptr(), _stream(), gout_ptr=g.data_ptr())
        return gc, gp, None


def huber_reprojection_cost(cams, pts, problem: Problem):
    return HuberReprojCost.apply(cams, pts, problem)
