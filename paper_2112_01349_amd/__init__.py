"""MI355X bundle adjustment: the per-iteration Levenberg-Marquardt step of
MegBA (arXiv 2112.01349) in HIP kernels behind the C ABI of include/ba.h.

    from paper_2112_01349_amd import Problem
    prob = Problem(cameras, points, obs_camera, obs_point, obs_uv, huber_delta=1.0)
    report = prob.lm_solve(max_lm_iters=20)

`HuberReprojCost` (in .autograd) exposes the robust reprojection cost and its
gradient as a torch.autograd.Function.
"""
from .native import (BAError, DAMP_IDENTITY, DAMP_MARQUARDT, FP32_MIXED, FP64, Problem,  # noqa: F401
                     lib)

__all__ = ["Problem", "BAError", "FP64", "FP32_MIXED", "DAMP_MARQUARDT", "DAMP_IDENTITY", "lib"]
