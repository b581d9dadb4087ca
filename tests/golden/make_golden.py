"""Writes the oracle's LM traces for the medium and large synthetic workloads.

Calls only the FP64 CPU oracle (oracle/) and the seeded input generator.
Usage: python tests/golden/make_golden.py {medium|large} [iters]
Output: tests/golden/lm_trace_<name>.json with the generator digest, the
solver options, the per-iteration trace (trial cost, cost, lambda,
predicted decrease, PCG iterations, accepted) and the oracle's wall time.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2112_01349_amd import synth  # noqa: E402

SETTINGS = {
    "medium": dict(huber_delta=0.0, max_pcg_iters=100, pcg_rtol=1e-6),
    "large": dict(huber_delta=1.0, max_pcg_iters=100, pcg_rtol=1e-6),
}


def main():
    name = sys.argv[1]
    iters = int(sys.argv[2]) if len(sys.argv) > 2 else 20
    opts = SETTINGS[name]
    t0 = time.time()
    prob = synth.generate(name, seed=0)
    t_gen = time.time() - t0
    print(f"[golden] {name}: generated {prob.num_obs} observations in {t_gen:.1f}s digest {prob.digest()}",
          flush=True)
    t0 = time.time()
    _, _, tr, rc = orc.lm_solve(prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv,
                                max_lm_iters=iters, **opts)
    wall = time.time() - t0
    out = {
        "description": "FP64 CPU oracle LM trace (single thread) on the seeded synthetic workload; "
                       "written by tests/golden/make_golden.py",
        "workload": name, "seed": 0, "digest": prob.digest(),
        "shape": [prob.num_cameras, prob.num_points, prob.num_obs],
        "options": dict(opts, max_lm_iters=iters, lambda_init=1e-4, min_relative_decrease=1e-3, damping=0),
        "status": rc, "oracle_seconds": wall,
        "initial_cost": tr["initial_cost"], "final_cost": tr["final_cost"], "iters_run": tr["iters_run"],
        "trial_cost": tr["trial_cost"].tolist(), "cost": tr["cost"].tolist(), "lambda": tr["lambda"].tolist(),
        "pred": tr["pred"].tolist(), "pcg_iters": tr["pcg_iters"].tolist(), "accepted": tr["accepted"].tolist(),
    }
    path = os.path.join(HERE, f"lm_trace_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[golden] {name}: {tr['iters_run']} iterations in {wall:.0f}s, final cost {tr['final_cost']:.10g} "
          f"-> {path}", flush=True)


if __name__ == "__main__":
    main()
