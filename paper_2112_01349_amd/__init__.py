"""MI355X bundle adjustment: the per-iteration Levenberg-Marquardt step of
MegBA (arXiv 2112.01349) in HIP kernels behind the C ABI of include/ba.h.

    from paper_2112_01349_amd import Problem
    prob = Problem(cameras, points, obs_camera, obs_point, obs_uv, huber_delta=1.0)
    report = prob.lm_solve(max_lm_iters=20)

Options (keyword arguments of Problem and lm_solve, the fields of ba_options):
precision, damping, huber_delta, max_lm_iters, max_pcg_iters, pcg_rtol,
pcg_fixed_iters, pcg_schedule, lambda_init, min_relative_decrease,
time_kernels, jacobian (0 analytic, 1 forward-mode autodiff), solver
(SOLVER_PCG, or SOLVER_DENSE: the reduced system written out and factored, at
most DENSE_MAX_CAMERAS cameras, fixed when the Problem is made) and
preconditioner (PRECOND_CAMERA_BLOCKS of Alg. 2, or PRECOND_SCHUR_JACOBI).

`HuberReprojCost` (in .autograd) exposes the robust reprojection cost and its
gradient as a torch.autograd.Function.
"""
from .native import (BAError, DAMP_IDENTITY, DAMP_MARQUARDT, DENSE_MAX_CAMERAS, FP32_MIXED, FP64,  # noqa: F401
                     PRECOND_CAMERA_BLOCKS, PRECOND_SCHUR_JACOBI, SOLVER_DENSE, SOLVER_PCG, Problem, lib)

__all__ = ["Problem", "BAError", "FP64", "FP32_MIXED", "DAMP_MARQUARDT", "DAMP_IDENTITY", "SOLVER_PCG",
           "SOLVER_DENSE", "DENSE_MAX_CAMERAS", "PRECOND_CAMERA_BLOCKS", "PRECOND_SCHUR_JACOBI", "lib"]
