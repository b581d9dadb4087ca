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


def order_spread(name):
    """How far rounding alone moves the oracle's LM trace on workload `name`:
    per iteration, the largest relative difference of the trial cost and of
    the accepted cost between the oracle's stored run
    (tests/golden/lm_trace_<name>.json) and its runs on the same problem with
    the observations in seeded random orders, replaying the same PCG counts
    (tests/golden/order_spread_<name>_seed*.json).  Both runs are FP64 and
    differ only in summation order, as the GPU's run does.  None when the
    files are missing."""
    import glob
    import json
    import os

    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    ref_path = os.path.join(here, f"lm_trace_{name}.json")
    paths = sorted(glob.glob(os.path.join(here, f"order_spread_{name}_seed*.json")))
    if not os.path.exists(ref_path) or not paths:
        return None
    ref = json.load(open(ref_path))
    trial = np.zeros(ref["iters_run"])
    cost = np.zeros(ref["iters_run"])
    for p in paths:
        g = json.load(open(p))
        assert g["digest"] == ref["digest"] and g["pcg_iters"] == ref["pcg_iters"], p
        t0, t1 = np.asarray(ref["trial_cost"]), np.asarray(g["trial_cost"])
        c0, c1 = np.asarray(ref["cost"]), np.asarray(g["cost"])
        trial = np.maximum(trial, np.abs(t1 - t0) / t0)
        cost = np.maximum(cost, np.abs(c1 - c0) / c0)
    return dict(trial=trial, cost=cost, runs=len(paths), trace=ref)


def oracle_spread(arrays, trace, seeds=(1, 2, 3), **oracle_kw):
    """order_spread for a small problem, measured on the spot: the oracle's
    LM run on `arrays` with the observations in seeded random orders,
    replaying trace's PCG counts (oracle_kw: the solver options of the run
    that produced `trace`, as orc.lm_solve takes them).  Compared while the
    accept/reject decisions agree."""
    from oracle import oracle as orc

    cams, pts, oc, op, uv = arrays[:5]
    oc, op, uv = np.asarray(oc), np.asarray(op), np.asarray(uv)
    kw = {k: v for k, v in oracle_kw.items() if k not in ("max_pcg_iters", "pcg_rtol", "pcg_schedule")}
    n_it = trace["iters_run"]
    trial, cost = np.zeros(n_it), np.zeros(n_it)
    for sd in seeds:
        perm = np.random.default_rng(sd).permutation(len(oc))
        _, _, t2, _ = orc.lm_solve(cams, pts, oc[perm], op[perm], uv[perm], max_lm_iters=n_it,
                                   pcg_schedule=trace["pcg_iters"], **kw)
        for k in range(min(n_it, t2["iters_run"])):
            trial[k] = max(trial[k], abs(t2["trial_cost"][k] - trace["trial_cost"][k]) / trace["trial_cost"][k])
            cost[k] = max(cost[k], abs(t2["cost"][k] - trace["cost"][k]) / trace["cost"][k])
            if t2["accepted"][k] != trace["accepted"][k]:
                break
    return dict(trial=trial, cost=cost, runs=len(seeds))


def rel_err_rows(a, b):
    """Largest error of a row (one camera's block) relative to that row's
    own largest entry: a small row is held to its own scale, not to the
    largest row's."""
    a = np.asarray(a, dtype=np.float64).reshape(len(b), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    scale = np.maximum(np.max(np.abs(b), axis=1), 1e-300)
    return float(np.max(np.max(np.abs(a - b), axis=1) / scale))
