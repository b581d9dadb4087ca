"""Shared input builders for the tests (inputs only; no arithmetic of the method)."""
import numpy as np

from paper_2112_01349_amd import synth


def small_zipf(seed=1, m=12, n=150, N=700, vmax=8, outliers=0.05):
    """A small problem with the Zipf/outlier structure of the large workloads."""
    cfg = dict(m=m, n=n, N=N, vmax=vmax, half=50.0, ring=150.0, outliers=outliers)
    synth.CONFIGS["_small"] = cfg
    try:
        return synth.generate("_small", seed=seed)
    finally:
        del synth.CONFIGS["_small"]


def with_edge_cases(prob, seed=3, long_point_views=300):
    """Adds the degenerate structures the method must accept: a camera with no
    observation, a point with none, a point with a single observation, a
    duplicated (camera, point) pair, and a point seen by more cameras than one
    workgroup tile holds (its views spread over every camera, repeating)."""
    rng = np.random.default_rng(seed)
    cams0 = np.concatenate([prob.cameras0, prob.cameras0[:1] * 1.001])       # camera m: unseen
    m = len(cams0)
    pts0 = np.concatenate([prob.points0, rng.uniform(-1, 1, size=(3, 3))])
    n0 = len(prob.points0)
    unseen, single, longp = n0, n0 + 1, n0 + 2
    oc = [prob.obs_camera, [0], [prob.obs_camera[0]]]
    op = [prob.obs_point, [single], [prob.obs_point[0]]]
    uv = [prob.obs_uv, [[3.0, -2.0]], [prob.obs_uv[0] + 0.5]]
    cams_for_long = np.arange(long_point_views) % (m - 1)
    oc.append(cams_for_long)
    op.append(np.full(long_point_views, longp))
    uv.append(rng.normal(0, 20, size=(long_point_views, 2)))
    oc = np.concatenate([np.asarray(a, np.int32) for a in oc])
    op = np.concatenate([np.asarray(a, np.int32) for a in op])
    uv = np.concatenate([np.asarray(a, np.float64).reshape(-1, 2) for a in uv])
    return cams0, pts0, oc, op, uv, dict(unseen_camera=m - 1, unseen_point=unseen)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
