"""The entry point that allocates nothing (ba_cost_device_noalloc) against
ba_cost_fwd_device on the same problems, through the C ABI: two calls in a
row, the second on a smaller problem, in both dtypes; and the oracle's cost.
Its only scratch is a fixed device array of partial sums shared by every
call on the device, so the second, smaller call must not see the first's
leftovers."""
import numpy as np
import pytest

from helpers import small_zipf
from oracle import oracle as orc
from paper_2112_01349_amd import Problem, synth
from paper_2112_01349_amd.native import BAError, cost_device_noalloc

pytestmark = pytest.mark.gpu


def device_arrays(torch, prob, dt):
    cams = torch.tensor(prob.cameras0, dtype=dt, device="cuda")
    pts = torch.tensor(prob.points0, dtype=dt, device="cuda")
    oc = torch.tensor(prob.obs_camera, dtype=torch.int32, device="cuda")
    op = torch.tensor(prob.obs_point, dtype=torch.int32, device="cuda")
    uv = torch.tensor(prob.obs_uv, dtype=torch.float64, device="cuda")
    return cams, pts, oc, op, uv


def noalloc_cost(torch, prob, dtype, delta):
    dt = torch.float64 if dtype == 0 else torch.float32
    cams, pts, oc, op, uv = device_arrays(torch, prob, dt)
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    cost_device_noalloc(prob.num_cameras, prob.num_points, prob.num_obs, dtype, cams.data_ptr(), pts.data_ptr(),
                        oc.data_ptr(), op.data_ptr(), uv.data_ptr(), delta, out.data_ptr(), stream)
    torch.cuda.synchronize()
    return float(out.item())


def handle_cost(torch, prob, dtype, delta):
    dt = torch.float64 if dtype == 0 else torch.float32
    gpu = Problem(prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv, huber_delta=delta)
    cams = torch.tensor(prob.cameras0, dtype=dt, device="cuda")
    pts = torch.tensor(prob.points0, dtype=dt, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    gpu.cost_fwd_device(dtype, cams.data_ptr(), pts.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    gpu.close()
    return float(out.item())


@pytest.mark.parametrize("dtype", [0, 1])
def test_noalloc_cost_matches_handle_cost_on_two_calls(dtype):
    import torch

    torch.cuda.set_device(0)
    big = synth.generate("diff", seed=0)        # 1M observations: every partial-sum slot in use
    small = small_zipf(seed=31)                  # 700 observations: three slots
    for prob in (big, small):
        F = noalloc_cost(torch, prob, dtype, 1.0)
        Fh = handle_cost(torch, prob, dtype, 1.0)
        assert abs(F - Fh) <= 1e-12 * abs(Fh), (prob.num_obs, F, Fh)
        if dtype == 0:
            Fo = orc.cost(prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv, 1.0)
            assert abs(F - Fo) <= 1e-12 * Fo, (prob.num_obs, F, Fo)


def test_noalloc_cost_edge_cases():
    import torch

    torch.cuda.set_device(0)
    prob = small_zipf(seed=32)
    # squared loss, and no observation at all
    F = noalloc_cost(torch, prob, 0, 0.0)
    Fo = orc.cost(prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv, 0.0)
    assert abs(F - Fo) <= 1e-12 * Fo
    cams, pts, oc, op, uv = device_arrays(torch, prob, torch.float64)
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    cost_device_noalloc(prob.num_cameras, prob.num_points, 0, 0, cams.data_ptr(), pts.data_ptr(), oc.data_ptr(),
                        op.data_ptr(), uv.data_ptr(), 1.0, out.data_ptr(), None)
    torch.cuda.synchronize()
    assert out.item() == 0.0
    # an observation index out of range makes the cost NaN (the kernel checks every index)
    bad = op.clone()
    bad[5] = prob.num_points
    cost_device_noalloc(prob.num_cameras, prob.num_points, prob.num_obs, 0, cams.data_ptr(), pts.data_ptr(),
                        oc.data_ptr(), bad.data_ptr(), uv.data_ptr(), 1.0, out.data_ptr(), None)
    torch.cuda.synchronize()
    assert np.isnan(out.item())
    # host-side validation
    with pytest.raises(BAError):
        cost_device_noalloc(0, prob.num_points, prob.num_obs, 0, cams.data_ptr(), pts.data_ptr(), oc.data_ptr(),
                            op.data_ptr(), uv.data_ptr(), 1.0, out.data_ptr(), None)
    with pytest.raises(BAError):
        cost_device_noalloc(prob.num_cameras, prob.num_points, prob.num_obs, 2, cams.data_ptr(), pts.data_ptr(),
                            oc.data_ptr(), op.data_ptr(), uv.data_ptr(), 1.0, out.data_ptr(), None)
