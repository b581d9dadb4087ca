"""Writes the oracle's LM traces for the medium and large synthetic workloads.

Calls only the FP64 CPU oracle (oracle/) and the seeded input generator.
Usage: python tests/golden/make_golden.py {medium|large|synth_small} [iters] [--permuted SEED]

Output: tests/golden/lm_trace_<name>.json with the generator digest, the
solver options, the per-iteration trace (trial cost, cost, lambda,
predicted decrease, PCG iterations, how each PCG solve ended, accepted)
and the oracle's wall time,
and tests/golden/lm_params_<name>.npz with the final parameters: every
camera, and a seeded sample of 10,000 points (indices and values).

With --permuted SEED the oracle runs on the same problem with its
observations in a seeded random order, replaying the stored trace's PCG
counts, and writes tests/golden/order_spread_<name>_seed<SEED>.json: the
per-iteration trace of that run.  Two FP64 runs that differ only in summation order
measure how far rounding alone moves each iteration's costs; the parity
tolerances for the GPU are set from this spread.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2112_01349_amd import synth  # noqa: E402

SETTINGS = {
    "medium": dict(huber_delta=0.0, max_pcg_iters=100, pcg_rtol=1e-6),
    "large": dict(huber_delta=1.0, max_pcg_iters=100, pcg_rtol=1e-6),
    # the synthesised recipe at oracle size, as its GPU parity test runs it
    "synth_small": dict(huber_delta=0.0, max_pcg_iters=30, pcg_rtol=1e-8),
}
DEFAULT_ITERS = {"synth_small": 4}
POINT_SAMPLE = 10_000


def trace_fields(tr):
    return {"initial_cost": tr["initial_cost"], "final_cost": tr["final_cost"], "iters_run": tr["iters_run"],
            "trial_cost": tr["trial_cost"].tolist(), "cost": tr["cost"].tolist(), "lambda": tr["lambda"].tolist(),
            "pred": tr["pred"].tolist(), "pcg_iters": tr["pcg_iters"].tolist(),
            "accepted": tr["accepted"].tolist(), "pcg_stop": tr["pcg_stop"].tolist()}


def point_sample(n):
    return np.sort(np.random.default_rng(10).choice(n, min(n, POINT_SAMPLE), replace=False)).astype(np.int64)


def main():
    args = [a for a in sys.argv[1:]]
    permuted = None
    if "--permuted" in args:
        k = args.index("--permuted")
        permuted = int(args[k + 1])
        del args[k:k + 2]
    name = args[0]
    iters = int(args[1]) if len(args) > 1 else DEFAULT_ITERS.get(name, 20)
    opts = SETTINGS[name]
    t0 = time.time()
    prob = synth.generate(name, seed=0)
    t_gen = time.time() - t0
    print(f"[golden] {name}: generated {prob.num_obs} observations in {t_gen:.1f}s digest {prob.digest()}",
          flush=True)
    oc, op, uv = prob.obs_camera, prob.obs_point, prob.obs_uv
    kw = dict(max_lm_iters=iters, **opts)
    if permuted is not None:
        ref = json.load(open(os.path.join(HERE, f"lm_trace_{name}.json")))
        assert ref["digest"] == prob.digest()
        perm = np.random.default_rng(permuted).permutation(prob.num_obs)
        oc, op, uv = oc[perm], op[perm], uv[perm]
        kw["pcg_schedule"] = ref["pcg_iters"]
    t0 = time.time()
    cams, pts, tr, rc = orc.lm_solve(prob.cameras0, prob.points0, oc, op, uv, **kw)
    wall = time.time() - t0
    out = {
        "description": "FP64 CPU oracle LM trace (single thread) on the seeded synthetic workload; "
                       "written by tests/golden/make_golden.py",
        "workload": name, "seed": 0, "digest": prob.digest(),
        "shape": [prob.num_cameras, prob.num_points, prob.num_obs],
        "options": dict(opts, max_lm_iters=iters, lambda_init=1e-4, min_relative_decrease=1e-3, damping=0),
        "status": rc, "oracle_seconds": wall, **trace_fields(tr),
    }
    if permuted is not None:
        out["description"] = ("FP64 CPU oracle LM trace with the observations in a seeded random order "
                              "(numpy default_rng(%d).permutation), replaying the PCG counts of "
                              "lm_trace_%s.json; written by tests/golden/make_golden.py" % (permuted, name))
        out["permutation_seed"] = permuted
        path = os.path.join(HERE, f"order_spread_{name}_seed{permuted}.json")
    else:
        path = os.path.join(HERE, f"lm_trace_{name}.json")
        idx = point_sample(prob.num_points)
        np.savez(os.path.join(HERE, f"lm_params_{name}.npz"), cameras=cams, point_index=idx, points=pts[idx])
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[golden] {name}: {tr['iters_run']} iterations in {wall:.0f}s, final cost {tr['final_cost']:.10g} "
          f"-> {path}", flush=True)


if __name__ == "__main__":
    main()
