"""The basis of the parity tolerances: how far the oracle's own LM trace moves
when only its summation order changes (the observations permuted, the same
PCG counts replayed).  The GPU differs from the oracle in exactly that way,
so these spreads, not observed GPU differences, set the bounds the GPU tests
use (1e-9 relative, or 4 times the spread where that is larger)."""
import json
import os

import numpy as np
import pytest

from helpers import order_spread, small_zipf, with_edge_cases
from oracle import oracle as orc
from paper_2112_01349_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def permuted_spread(arrays, delta, iters, max_pcg, rtol, seeds=(1, 2, 3)):
    cams, pts, oc, op, uv = arrays[:5]
    _, _, tr, rc = orc.lm_solve(cams, pts, oc, op, uv, huber_delta=delta, max_lm_iters=iters,
                                max_pcg_iters=max_pcg, pcg_rtol=rtol)
    assert rc == 0
    worst = 0.0
    for sd in seeds:
        perm = np.random.default_rng(sd).permutation(len(oc))
        _, _, t2, _ = orc.lm_solve(cams, pts, oc[perm], op[perm], uv[perm], huber_delta=delta, max_lm_iters=iters,
                                   pcg_schedule=tr["pcg_iters"])
        # compare while both runs are on the same path; a decision may differ
        # only where the cost change is itself round-off (a converged solve)
        prev = tr["initial_cost"]
        for k in range(iters):
            worst = max(worst, abs(t2["trial_cost"][k] - tr["trial_cost"][k]) / tr["trial_cost"][k])
            if t2["accepted"][k] != tr["accepted"][k]:
                assert abs(prev - tr["trial_cost"][k]) <= 1e-10 * prev, (sd, k)
                break
            prev = tr["cost"][k]
    return worst


@pytest.mark.parametrize("case", ["tiny", "huber_edge", "hot_cold"])
def test_small_problems_spread_far_below_the_floor(case):
    """The small LM-trace problems of the GPU tests (their exact settings):
    the oracle's order spread stays below 1e-11, so the 1e-9 floor leaves a
    margin of 100 and more."""
    if case == "tiny":
        p = synth.generate("tiny", seed=0)
        arrays, delta, iters, max_pcg = (p.cameras0, p.points0, p.obs_camera, p.obs_point, p.obs_uv), 0.0, 10, 50
    elif case == "huber_edge":
        arrays, delta, iters, max_pcg = with_edge_cases(small_zipf(seed=11, m=20, n=400, N=2400)), 1.0, 8, 60
    else:
        arrays, delta, iters, max_pcg = with_edge_cases(small_zipf(seed=13, m=14, n=300, N=1500)), 1.0, 5, 40
    assert permuted_spread(arrays, delta, iters, max_pcg, 1e-8) < 1e-11


def test_stored_spread_is_the_scripts_output():
    """The stored permuted run of the synthesised recipe is what the oracle
    gives today with that permutation (the file is written by
    tests/golden/make_golden.py from the oracle alone), and its spread is
    the one the GPU test of that recipe is held to."""
    sp = order_spread("synth_small")
    assert sp is not None and sp["runs"] >= 3
    g = json.load(open(os.path.join(GOLDEN, "order_spread_synth_small_seed1.json")))
    prob = synth.generate("synth_small", seed=0)
    assert prob.digest() == g["digest"]
    perm = np.random.default_rng(g["permutation_seed"]).permutation(prob.num_obs)
    o = g["options"]
    _, _, tr, rc = orc.lm_solve(prob.cameras0, prob.points0, prob.obs_camera[perm], prob.obs_point[perm],
                                prob.obs_uv[perm], huber_delta=o["huber_delta"], max_lm_iters=o["max_lm_iters"],
                                pcg_schedule=sp["trace"]["pcg_iters"])
    assert rc == 0
    np.testing.assert_array_equal(tr["trial_cost"], g["trial_cost"])
    # near the zero-cost optimum the spread grows far above the floor
    assert sp["trial"].max() > 1e-8
