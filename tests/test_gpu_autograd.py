"""HuberReprojCost (torch.autograd.Function over the HIP cost kernels) on the
differentiation workload: 1,000 cameras, 200k points, 1M observations,
Huber delta = 1 px with 5% outliers.

Checks, for FP64 and FP32 parameters: the cost against the oracle's FP64 cost,
the full gradient against the oracle's gradient, and 1,000 seeded gradient
entries against central finite differences (h = 1e-6 max(1, |x|), FP64) of
the oracle's local cost (the observations touching that parameter).
Tolerances: FP64 1e-6 relative for the FD check (its truncation/round-off
level) and 1e-10 against the oracle's gradient; FP32 1e-3 relative.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2112_01349_amd import Problem, synth
from paper_2112_01349_amd.autograd import HuberReprojCost

pytestmark = pytest.mark.gpu
DELTA = 1.0


@pytest.fixture(scope="module")
def diff():
    prob = synth.generate("diff", seed=0)
    args = (prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv)
    gpu = Problem(*args, huber_delta=DELTA)
    F, gc, gp = orc.gradient(*args, DELTA)
    cam_csr = orc.csr(prob.obs_camera, prob.num_cameras)
    pt_csr = orc.csr(prob.obs_point, prob.num_points)
    yield dict(prob=prob, args=args, gpu=gpu, F=F, gc=gc, gp=gp, cam_csr=cam_csr, pt_csr=pt_csr)
    gpu.close()


def fd_entries(d, rng, count):
    """Central differences of the oracle's local cost for `count` seeded
    (block, component) parameters; returns [(is_camera, index, comp, fd)]."""
    prob = d["prob"]
    cams, pts, oc, op, uv = d["args"]
    out = []
    for _ in range(count):
        if rng.random() < 0.5:
            j, a = int(rng.integers(prob.num_cameras)), int(rng.integers(9))
            off, order = d["cam_csr"]
            local = order[off[j]:off[j + 1]]
            base = cams[j, a]
            h = 1e-6 * max(1.0, abs(base))
            cp, cm = cams.copy(), cams.copy()
            cp[j, a] += h
            cm[j, a] -= h
            fd = (orc.cost_subset(local, cp, pts, oc, op, uv, DELTA)
                  - orc.cost_subset(local, cm, pts, oc, op, uv, DELTA)) / (2 * h)
            out.append((True, j, a, fd))
        else:
            i, a = int(rng.integers(prob.num_points)), int(rng.integers(3))
            off, order = d["pt_csr"]
            local = order[off[i]:off[i + 1]]
            base = pts[i, a]
            h = 1e-6 * max(1.0, abs(base))
            pp, pm = pts[[i]].copy(), pts[[i]].copy()
            pp[0, a] += h
            pm[0, a] -= h
            # local cost with only point i changed: evaluate on a one-point array
            sub_op = np.zeros(len(local), np.int32)
            fd = (orc.cost_subset(np.arange(len(local)), cams, pp, oc[local], sub_op, uv[local], DELTA)
                  - orc.cost_subset(np.arange(len(local)), cams, pm, oc[local], sub_op, uv[local], DELTA)) / (2 * h)
            out.append((False, i, a, fd))
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_autograd_cost_and_gradient(diff, dtype):
    prob = diff["prob"]
    cams = torch.tensor(prob.cameras0, dtype=dtype, device="cuda", requires_grad=True)
    pts = torch.tensor(prob.points0, dtype=dtype, device="cuda", requires_grad=True)
    F = HuberReprojCost.apply(cams, pts, diff["gpu"])
    assert F.dtype == torch.float64
    (2.5 * F).backward()
    torch.cuda.synchronize()
    gc = cams.grad.double().cpu().numpy() / 2.5
    gp = pts.grad.double().cpu().numpy() / 2.5
    if dtype == torch.float64:
        assert abs(F.item() - diff["F"]) <= 1e-12 * diff["F"]
        tol_oracle, tol_fd = 1e-10, 1e-6
    else:
        # FP32 parameters: the oracle evaluates at the same FP32-rounded values
        c32 = prob.cameras0.astype(np.float32).astype(np.float64)
        p32 = prob.points0.astype(np.float32).astype(np.float64)
        F32, _, _ = orc.gradient(c32, p32, prob.obs_camera, prob.obs_point, prob.obs_uv, DELTA)
        assert abs(F.item() - F32) <= 1e-5 * F32
        tol_oracle, tol_fd = 1e-3, 1e-3
    for g, ref in ((gc, diff["gc"]), (gp, diff["gp"])):
        assert np.max(np.abs(g - ref)) <= tol_oracle * np.max(np.abs(ref))
    rng = np.random.default_rng(2024)
    scale_c, scale_p = np.max(np.abs(diff["gc"]), axis=0), np.max(np.abs(diff["gp"]), axis=0)
    for is_cam, idx, comp, fd in fd_entries(diff, rng, 1000):
        g = gc[idx, comp] if is_cam else gp[idx, comp]
        ref_scale = (scale_c if is_cam else scale_p)[comp]
        assert abs(g - fd) <= tol_fd * max(abs(fd), 1e-3 * ref_scale), (is_cam, idx, comp, g, fd)


def test_autograd_matches_host_gradient_call(diff):
    """The device-pointer path and ba_eval_cost_grad agree (FP64)."""
    prob = diff["prob"]
    F, gc, gp = diff["gpu"].eval_cost_grad()
    cams = torch.tensor(prob.cameras0, device="cuda", requires_grad=True)
    pts = torch.tensor(prob.points0, device="cuda", requires_grad=True)
    Fd = HuberReprojCost.apply(cams, pts, diff["gpu"])
    Fd.backward()
    assert abs(Fd.item() - F) <= 1e-13 * F
    np.testing.assert_allclose(cams.grad.cpu().numpy(), gc, rtol=0, atol=1e-12 * np.abs(gc).max())
    np.testing.assert_allclose(pts.grad.cpu().numpy(), gp, rtol=0, atol=1e-12 * np.abs(gp).max())
