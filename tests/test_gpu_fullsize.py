"""Full-size parity: the 29M-observation workload (13,700 cameras, 4.5M points,
Huber delta = 1 px, 5% outliers) in the launch configuration bench.py times.

At this size the oracle computes sampled outputs one by one: the FP64 cost
over all observations, the gradient of sampled cameras (including the most
observed one) and points from their own observation lists, and rows of the
reduced camera system S x for sampled cameras from scratch.  The LM traces
are compared with the oracle's stored traces (tests/golden/lm_trace_*.json,
written by tests/golden/make_golden.py), replaying the oracle's PCG counts.
"""
import json
import os

import numpy as np
import pytest

from helpers import order_spread
from oracle import oracle as orc
from paper_2112_01349_amd import FP32_MIXED, FP64, Problem, synth
from test_gpu_parity import SPREAD_FACTOR

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DELTA = 1.0


@pytest.fixture(scope="module")
def large():
    prob = synth.generate("large", seed=0)
    args = (prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv)
    cam_csr = orc.csr(prob.obs_camera, prob.num_cameras)
    pt_csr = orc.csr(prob.obs_point, prob.num_points)
    return dict(prob=prob, args=args, cam_csr=cam_csr, pt_csr=pt_csr)


def sampled_cameras(d):
    """The two most observed cameras; hot cameras of rank 20 and 100 (in the
    LDS hot-camera table, and among the 256 whose records the recomputing
    product reads from LDS) and 1000 (in the table, record read from
    memory); the camera of rank 3000 and three random ones of rank 2261 and
    beyond, cold in every product (the recomputing product's table holds the
    1,862 most observed cameras in FP32, 1,464 in FP64; the stored-block
    product's 2,261)."""
    counts = np.diff(d["cam_csr"][0])
    order = np.argsort(-counts, kind="stable")
    rng = np.random.default_rng(5)
    return [int(order[r]) for r in (0, 1, 20, 100, 1000, 3000)] + [int(x) for x in
                                                                 rng.choice(order[2261:], 3, replace=False)]


def test_large_cost_gradient_fp64(large):
    prob = large["prob"]
    gpu = Problem(*large["args"], huber_delta=DELTA)
    F, gc, gp = gpu.eval_cost_grad()
    gpu.close()
    Fo = orc.cost(*large["args"], DELTA)
    assert abs(F - Fo) <= 1e-12 * Fo
    off, order = large["cam_csr"]
    for j in sampled_cameras(large):
        s = orc.subset_sums(order[off[j]:off[j + 1]], *large["args"], DELTA)
        ref = -s["v"]
        assert np.max(np.abs(gc[j] - ref)) <= 1e-10 * np.max(np.abs(ref)), j
    poff, porder = large["pt_csr"]
    rng = np.random.default_rng(6)
    for i in rng.choice(prob.num_points, 200, replace=False):
        s = orc.subset_sums(porder[poff[i]:poff[i + 1]], *large["args"], DELTA)
        ref = -s["w"]
        assert np.max(np.abs(gp[i] - ref)) <= 1e-10 * np.max(np.abs(ref)) + 1e-300, i


@pytest.fixture(scope="module")
def large_rows(large):
    """The oracle's rows of the damped reduced system at lambda 1e-3 for the
    sampled cameras (rank 20 and below), computed once from scratch."""
    prob = large["prob"]
    x = np.random.default_rng(7).normal(size=(prob.num_cameras, 9))
    rows = sampled_cameras(large)[2:]
    ref = orc.schur_rows(rows, *large["args"][:2], *large["args"][2:], x, 1e-3, DELTA,
                         cam_csr=large["cam_csr"], pt_csr=large["pt_csr"])
    return dict(x=x, rows=rows, ref=ref, lam=1e-3)


@pytest.mark.parametrize("stored", [0, 1])
@pytest.mark.parametrize("precision", [FP64, FP32_MIXED])
def test_large_schur_rows(large, large_rows, precision, stored, monkeypatch):
    """Sampled rows of the reduced-system product at full size, from the
    recomputing product and from the stored-block one, against the oracle's
    rows computed from scratch: three hot cameras (their camera side goes
    through the workgroups' LDS tables and the fold; two of them with their
    records read from LDS) and four cold ones (the camera-major cold pass).  Each row is compared relative to its own
    largest entry."""
    monkeypatch.setenv("BA_SCHUR_STORED", str(stored))
    gpu = Problem(*large["args"], precision=precision, huber_delta=DELTA)
    q = gpu.schur_matvec(large_rows["x"], large_rows["lam"])
    gpu.close()
    counts = np.diff(large["cam_csr"][0])
    order = np.argsort(-counts, kind="stable")
    assert large_rows["rows"][:3] == [int(order[r]) for r in (20, 100, 1000)]   # hot (rank < 1464)
    # FP32-mixed: float rounding through a row's thousands of points gives
    # 2e-7 .. 3e-6; the bound is ten times that and more
    tol = 1e-9 if precision == FP64 else 5e-5
    errs = [np.max(np.abs(q[j] - large_rows["ref"][t])) / np.max(np.abs(large_rows["ref"][t]))
            for t, j in enumerate(large_rows["rows"])]
    print(f"precision {precision} stored {stored}: row errors " + " ".join(f"{e:.1e}" for e in errs))
    for t, j in enumerate(large_rows["rows"]):
        assert errs[t] <= tol, (j, q[j], large_rows["ref"][t])


def load_golden(name):
    path = os.path.join(GOLDEN, f"lm_trace_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet")
    return json.load(open(path))


def replay(name, precision=FP64, schedule=True):
    g = load_golden(name)
    prob = synth.generate(name, seed=0)
    assert prob.digest() == g["digest"], "generator output differs from the one the trace was taken on"
    o = g["options"]
    gpu = Problem(prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv,
                  precision=precision, huber_delta=o["huber_delta"])
    kw = dict(max_lm_iters=o["max_lm_iters"], max_pcg_iters=o["max_pcg_iters"], pcg_rtol=o["pcg_rtol"])
    if schedule:
        kw["pcg_schedule"] = g["pcg_iters"]
    rep = gpu.lm_solve(**kw)
    gpu.close()
    return g, rep


@pytest.mark.parametrize("name", ["medium", "large"])
def test_lm_trace_fp64_matches_oracle(name):
    """Per-iteration parity on the trial and accepted costs, replaying the
    oracle's PCG counts: relative 1e-9, or 4 times the oracle's own spread at
    that iteration where that is larger.  The spread is how far the oracle's
    trace moves when only its summation order changes (its stored runs on
    the same problem with the observations permuted): after a PCG solve that
    stopped at its cap unconverged, or at a trial point far outside the
    step's linear model (the first steps at lambda_0 = 1e-4 raise the cost to
    3.4e19 against 1.3e8 by putting observations near a camera's principal
    plane), the step carries that rounding into the cost.  Where the trial
    cost rises more than tenfold both sides must reject."""
    spread = order_spread(name)
    if spread is None:
        pytest.skip(f"tests/golden/order_spread_{name}_seed*.json not written yet")
    # where the spread, not the 1e-9 floor, sets a bound, one permuted run is
    # too small a sample of it: the largest of several is taken
    if spread["runs"] < 3 and np.any(SPREAD_FACTOR * spread["trial"] > 1e-9):
        pytest.skip(f"{spread['runs']} stored permuted run(s) of {name}; the spread bound needs three")
    g, rep = replay(name)
    assert rep["status"] == 0 and rep["iters_run"] == g["iters_run"]
    assert abs(rep["initial_cost"] - g["initial_cost"]) <= 1e-12 * g["initial_cost"]
    prev = g["initial_cost"]
    same_path = True
    for k in range(g["iters_run"]):
        ft = g["trial_cost"][k]
        rel = max(1e-9, SPREAD_FACTOR * spread["trial"][k])
        crel = max(1e-9, SPREAD_FACTOR * spread["cost"][k])
        err = abs(rep["trial_cost"][k] - ft)
        print(f"iter {k}: trial rel diff {err / ft:.2e} (tol {rel:.1e}, oracle spread {spread['trial'][k]:.1e}), "
              f"pcg {g['pcg_iters'][k]}")
        assert err <= rel * ft, k
        assert abs(rep["cost"][k] - g["cost"][k]) <= max(rel * ft, crel * g["cost"][k]), k
        if ft > 10 * prev:
            assert not rep["accepted"][k] and not g["accepted"][k], k
        if same_path and abs(prev - ft) > max(1e-10, 2 * rel) * prev:
            assert rep["accepted"][k] == g["accepted"][k], k
        else:
            same_path = False
        prev = g["cost"][k]


# How far above the oracle's 20-iteration cost the FP32-mixed solve may end
# after the same 20 iterations: over repeated runs it ended between -4.8e-4
# and +5.1e-4 of it (8 of 9 at or below +1e-4), so twice the worst excess.
MIXED_20_MARGIN = 1e-3


def test_lm_mixed_meets_oracle_final_cost():
    """The FP32-mixed solve of the 29M workload (PCG rtol 1e-6, no replayed
    schedule) against the oracle's 20-iteration FP64 cost.  After exactly 20
    iterations its cost is at most MIXED_20_MARGIN above the oracle's: the
    problem is still descending ~2e-4 per iteration, late PCG solves stop
    at their cap or break down on the FP32 products' rounding, and a
    rejected step costs an iteration, so the 20-iteration cost varies by a
    few 1e-4 either side from run to run.  Within 30 iterations it reaches
    the oracle's cost within 1e-4, with non-increasing accepted costs."""
    g = load_golden("large")
    prob = synth.generate("large", seed=0)
    gpu = Problem(prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv,
                  precision=FP32_MIXED, huber_delta=g["options"]["huber_delta"])
    rep = gpu.lm_solve(max_lm_iters=30, max_pcg_iters=g["options"]["max_pcg_iters"],
                       pcg_rtol=g["options"]["pcg_rtol"])
    gpu.close()
    assert rep["status"] == 0, (rep["error"], rep["lambda"].tolist(), rep["cost"].tolist())
    costs = np.concatenate([[rep["initial_cost"]], rep["cost"]])
    assert np.all(np.diff(costs) <= 0)
    F20 = rep["cost"][19] / g["final_cost"] - 1
    reached = np.nonzero(rep["cost"] <= g["final_cost"] * (1 + 1e-4))[0]
    print(f"mixed cost after 20 iterations: {F20:+.2e} relative to the oracle; within 1e-4 from iteration "
          f"{reached[0] + 1 if len(reached) else None}; PCG stops {rep['pcg_stop'].tolist()}")
    assert F20 <= MIXED_20_MARGIN
    assert len(reached) > 0, (rep["final_cost"], g["final_cost"])


def test_stress_cost_gradient_and_schur_rows():
    """The 60M-observation stress workload (20,000 cameras, 10M points, Huber,
    5% outliers) in the FP32-mixed form: FP64 cost and sampled gradients
    against the oracle, sampled reduced-system rows against the oracle's rows
    computed from scratch, and two LM iterations with non-increasing cost."""
    prob = synth.generate("stress", seed=0)
    args = (prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv)
    gpu = Problem(*args, precision=FP32_MIXED, huber_delta=DELTA)
    F, gc, gp = gpu.eval_cost_grad()
    Fo = orc.cost(*args, DELTA)
    assert abs(F - Fo) <= 1e-12 * Fo
    cam_csr = orc.csr(prob.obs_camera, prob.num_cameras)
    pt_csr = orc.csr(prob.obs_point, prob.num_points)
    counts = np.diff(cam_csr[0])
    order = np.argsort(-counts, kind="stable")
    rows = [int(order[5000]), int(order[-1]), int(order[12000])]
    off, obs = cam_csr
    for j in rows:
        ref = -orc.subset_sums(obs[off[j]:off[j + 1]], *args, DELTA)["v"]
        assert np.max(np.abs(gc[j] - ref)) <= 1e-10 * np.max(np.abs(ref)), j
    x = np.random.default_rng(8).normal(size=(prob.num_cameras, 9))
    q = gpu.schur_matvec(x, 1e-3)
    ref = orc.schur_rows(rows, *args[:2], *args[2:], x, 1e-3, DELTA, cam_csr=cam_csr, pt_csr=pt_csr)
    errs = [np.max(np.abs(q[j] - ref[t])) / np.max(np.abs(ref[t])) for t, j in enumerate(rows)]
    print("60M FP32-mixed row errors " + " ".join(f"{e:.1e}" for e in errs))
    for t, j in enumerate(rows):
        assert errs[t] <= 5e-5, j  # float rounding: 2e-7 .. 2.4e-6 measured
    rep = gpu.lm_solve(max_lm_iters=2, max_pcg_iters=200, pcg_rtol=1e-6)
    gpu.close()
    assert rep["status"] == 0
    costs = np.concatenate([[rep["initial_cost"]], rep["cost"]])
    assert np.all(np.diff(costs) <= 0)


def test_synthesised_20000_cost_gradient_and_schur_rows():
    """The paper's synthesised problem at full size (20,000 cameras, 80,000
    points seen 1,000 times each, 80M observations), in both precisions:
    FP64 cost and sampled camera and point gradients against the oracle,
    sampled rows of the reduced system against the oracle's rows computed
    from scratch, and two LM iterations with non-increasing cost."""
    prob = synth.generate("synth20000", seed=0)
    args = (prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv)
    Fo = orc.cost(*args, 0.0)
    cam_csr = orc.csr(prob.obs_camera, prob.num_cameras)
    pt_csr = orc.csr(prob.obs_point, prob.num_points)
    rng = np.random.default_rng(9)
    cams = [int(j) for j in rng.choice(prob.num_cameras, 3, replace=False)]
    pts = [int(i) for i in rng.choice(prob.num_points, 20, replace=False)]
    x = rng.normal(size=(prob.num_cameras, 9))
    ref_rows = orc.schur_rows(cams, *args[:2], *args[2:], x, 1e-3, 0.0, cam_csr=cam_csr, pt_csr=pt_csr)
    for precision in (FP64, FP32_MIXED):
        gpu = Problem(*args, precision=precision)
        F, gc, gp = gpu.eval_cost_grad()
        assert abs(F - Fo) <= 1e-12 * Fo, precision
        gtol = 1e-10 if precision == FP64 else 1e-3
        off, order = cam_csr
        for j in cams:
            ref = -orc.subset_sums(order[off[j]:off[j + 1]], *args, 0.0)["v"]
            assert np.max(np.abs(gc[j] - ref)) <= gtol * np.max(np.abs(ref)), (precision, j)
        off, order = pt_csr
        for i in pts:
            ref = -orc.subset_sums(order[off[i]:off[i + 1]], *args, 0.0)["w"]
            assert np.max(np.abs(gp[i] - ref)) <= gtol * np.max(np.abs(ref)), (precision, i)
        q = gpu.schur_matvec(x, 1e-3)
        qtol = 1e-9 if precision == FP64 else 5e-5  # FP32-mixed: 1e-9 .. 7e-8 measured
        errs = [np.max(np.abs(q[j] - ref_rows[t])) / np.max(np.abs(ref_rows[t])) for t, j in enumerate(cams)]
        print(f"80M precision {precision}: row errors " + " ".join(f"{e:.1e}" for e in errs))
        for t, j in enumerate(cams):
            assert errs[t] <= qtol, (precision, j)
        rep = gpu.lm_solve(max_lm_iters=2, max_pcg_iters=100, pcg_rtol=1e-6)
        gpu.close()
        assert rep["status"] == 0
        costs = np.concatenate([[rep["initial_cost"]], rep["cost"]])
        assert np.all(np.diff(costs) <= 0) and costs[-1] < costs[0], precision


def test_chunk_of_eight_lm_matches_oracle():
    """One GPU's share of the 29M workload split over eight GPUs (all 13,700
    cameras, the first 1/8 of the observations at point boundaries): three
    FP64 LM iterations (lambda_0 = 1e-2, so the steps are accepted, and a
    fixed PCG count of 12) match the oracle's costs to 1e-9."""
    full = synth.generate("large", seed=0)
    prob = synth.point_chunk(full, 0, 8)
    del full
    assert abs(prob.num_obs - 29_000_000 / 8) < 100
    args = (prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv)
    kw = dict(huber_delta=DELTA, max_lm_iters=3, pcg_schedule=[12, 12, 12], lambda_init=1e-2)
    _, _, tr, rc = orc.lm_solve(*args, **kw)
    assert rc == 0 and list(tr["accepted"]) == [1, 1, 1]
    gpu = Problem(*args, huber_delta=DELTA)
    rep = gpu.lm_solve(max_lm_iters=3, pcg_schedule=[12, 12, 12], lambda_init=1e-2)
    gpu.close()
    assert rep["status"] == 0
    assert abs(rep["initial_cost"] - tr["initial_cost"]) <= 1e-12 * tr["initial_cost"]
    for k in range(3):
        assert abs(rep["trial_cost"][k] - tr["trial_cost"][k]) <= 1e-9 * tr["trial_cost"][k], k
        assert rep["accepted"][k] == 1, k
