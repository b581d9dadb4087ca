"""HIP path vs the FP64 CPU oracle, element by element, through the C ABI.

Tolerances: the FP64 path matches the oracle's per-iteration cost to relative
1e-9 with the PCG iteration counts matched (the oracle runs first with its
rtol and the GPU replays its counts); cost, gradient and Schur products agree
to near round-off (1e-12 .. 1e-10 relative, the spread of summation order over
a few thousand terms).  The FP32-mixed path must reach a final cost within
relative 1e-4 of the oracle's.
"""
import numpy as np
import pytest

from helpers import oracle_spread, order_spread, rel_err, rel_err_rows, small_zipf, with_edge_cases
from oracle import oracle as orc
from paper_2112_01349_amd import FP32_MIXED, FP64, Problem, synth
from paper_2112_01349_amd.native import PRECOND_SCHUR_JACOBI, SOLVER_DENSE

pytestmark = pytest.mark.gpu

# The FP32-mixed reduced-system product against the FP64 oracle, per camera
# row relative to the row's largest entry.  Float rounding (unit 6e-8) of the
# Jacobian and of the per-point sums, carried through C~^-1 and the sum over
# a camera's points, gives 1e-7 .. 5e-6 on these problems; the bound is about
# 800 float units, ten times the largest seen.
FP32_PRODUCT_TOL = 5e-5


def make(prob_or_arrays, precision=FP64, **opts):
    if isinstance(prob_or_arrays, tuple):
        cams, pts, oc, op, uv = prob_or_arrays[:5]
    else:
        p = prob_or_arrays
        cams, pts, oc, op, uv = p.cameras0, p.points0, p.obs_camera, p.obs_point, p.obs_uv
    return Problem(cams, pts, oc, op, uv, precision=precision, **opts), (cams, pts, oc, op, uv)


@pytest.fixture(scope="module")
def tiny():
    return synth.generate("tiny", seed=0)


@pytest.mark.parametrize("delta", [0.0, 1.0])
def test_cost_and_gradient(tiny, delta):
    src = tiny if delta == 0.0 else small_zipf()
    prob, (cams, pts, oc, op, uv) = make(src, huber_delta=delta)
    F, gc, gp = prob.eval_cost_grad()
    Fo, gco, gpo = orc.gradient(cams, pts, oc, op, uv, delta)
    assert abs(F - Fo) <= 1e-13 * abs(Fo)
    assert rel_err_rows(gc, gco) <= 1e-10
    assert rel_err_rows(gp, gpo) <= 1e-10
    c2, p2 = prob.get_params()
    np.testing.assert_array_equal(c2, cams)
    np.testing.assert_array_equal(p2, pts)


@pytest.mark.parametrize("stored", [0, 1])
@pytest.mark.parametrize("damping", [0, 1])
def test_schur_matvec(tiny, damping, stored, monkeypatch):
    monkeypatch.setenv("BA_SCHUR_STORED", str(stored))
    prob, (cams, pts, oc, op, uv) = make(tiny)
    lam = 1e-3
    A = orc.assemble(cams, pts, oc, op, uv)
    Bd, Cd, Dc, Dp = orc.damp(A["B"], A["C"], lam, damping)
    Ci = orc.invert_points(Cd)
    x = np.random.default_rng(4).normal(size=(len(cams), 9))
    ref = orc.schur_matvec(oc, op, Bd, A["E"], Ci, x)
    q = prob.schur_matvec(x, lam, damping)
    assert rel_err_rows(q, ref) <= 1e-11


@pytest.mark.parametrize("hot", [12, 3, 0])
def test_camera_rows_at_row_and_chunk_boundaries(hot, monkeypatch):
    """The camera-side build cuts the camera-sorted stream into rows of at
    most 64 observations of one camera and gives each wavefront 32 rows, a
    camera's terms leaving in one partial sum per chunk it touches.  Cameras
    seen 4097, 2049, 2048, 2047, 130 ... 127, 65, 64, 63 and 1 times end
    before, at and after row and chunk boundaries (and the cold stream, the
    tail of that order, starts inside a chunk when only 3 cameras are hot):
    B_j through the Schur product and v_j through the gradient match the
    oracle's, in both precisions."""
    monkeypatch.setenv("BA_HOT_CAMERAS", str(hot))
    base = small_zipf(seed=21, m=12, n=4200, N=9000, vmax=8)
    counts = [4097, 2049, 2048, 2047, 130, 129, 128, 127, 65, 64, 63, 1]
    rng = np.random.default_rng(8)
    n = len(base.points0)
    oc = np.concatenate([np.full(c, j, np.int32) for j, c in enumerate(counts)])
    op = np.concatenate([rng.choice(n, size=c, replace=False) for c in counts]).astype(np.int32)
    uv = rng.normal(0, 20, size=(len(oc), 2))
    arrays = (base.cameras0, base.points0, oc, op, uv)
    Fo, gco, gpo = orc.gradient(*arrays, 0.0)
    lam = 1e-3
    A = orc.assemble(*arrays)
    Bd, Cd, Dc, Dp = orc.damp(A["B"], A["C"], lam, 0)
    Ci = orc.invert_points(Cd)
    x = np.random.default_rng(9).normal(size=(len(counts), 9))
    ref = orc.schur_matvec(oc, op, Bd, A["E"], Ci, x)
    for precision in (FP64, FP32_MIXED):
        prob, _ = make(arrays, precision=precision)
        if precision == FP64:
            F, gc, gp = prob.eval_cost_grad()
            assert abs(F - Fo) <= 1e-13 * abs(Fo)
            assert rel_err_rows(gc, gco) <= 1e-10 and rel_err_rows(gp, gpo) <= 1e-10
        err = rel_err_rows(prob.schur_matvec(x, lam), ref)
        print(f"hot {hot} precision {precision}: product error {err:.2e} of each row")
        assert err <= (1e-10 if precision == FP64 else FP32_PRODUCT_TOL), precision
        prob.close()


def test_edge_cases_cost_gradient_matvec():
    arrays = with_edge_cases(small_zipf(seed=7))
    cams, pts, oc, op, uv, info = arrays
    prob, _ = make(arrays, huber_delta=1.0)
    F, gc, gp = prob.eval_cost_grad()
    Fo, gco, gpo = orc.gradient(cams, pts, oc, op, uv, 1.0)
    assert abs(F - Fo) <= 1e-13 * abs(Fo)
    assert rel_err_rows(gc, gco) <= 1e-10 and rel_err_rows(gp, gpo) <= 1e-10
    assert np.all(gc[info["unseen_camera"]] == 0.0) and np.all(gp[info["unseen_point"]] == 0.0)
    lam = 1e-2
    A = orc.assemble(cams, pts, oc, op, uv, 1.0)
    Bd, Cd, Dc, Dp = orc.damp(A["B"], A["C"], lam, 0)
    Ci = orc.invert_points(Cd)
    x = np.random.default_rng(5).normal(size=(len(cams), 9))
    ref = orc.schur_matvec(oc, op, Bd, A["E"], Ci, x)
    assert rel_err_rows(prob.schur_matvec(x, lam), ref) <= 1e-10


def lm_pair(src, delta=0.0, iters=10, max_pcg=50, rtol=1e-8, spread=True):
    arrays = src if isinstance(src, tuple) else None
    if arrays is None:
        arrays = (src.cameras0, src.points0, src.obs_camera, src.obs_point, src.obs_uv)
    cams, pts, oc, op, uv = arrays[:5]
    oc_, op_, tr, rc = orc.lm_solve(cams, pts, oc, op, uv, huber_delta=delta, max_lm_iters=iters,
                                    max_pcg_iters=max_pcg, pcg_rtol=rtol)
    assert rc == 0
    if spread:
        tr["spread"] = oracle_spread(arrays, tr, huber_delta=delta)
    prob, _ = make(arrays[:5], huber_delta=delta)
    gpu = prob.lm_solve(max_lm_iters=iters, pcg_schedule=tr["pcg_iters"], max_pcg_iters=max_pcg,
                        pcg_rtol=rtol)
    if len(arrays) > 5 and "unseen_point" in arrays[5]:
        # a point with no observation never moves (its step is zero in the
        # oracle, and the device must not leave it to whatever memory held)
        u = arrays[5]["unseen_point"]
        np.testing.assert_array_equal(prob.get_params()[1][u], pts[u])
    return tr, gpu, prob, (oc_, op_)


# How far the GPU's trace may sit from the oracle's beyond the 1e-9 floor:
# SPREAD_FACTOR times the oracle's own spread under a permuted observation
# order (the GPU differs from the oracle only in summation order, and a
# handful of permuted runs bounds that spread from below).
SPREAD_FACTOR = 4.0


def assert_traces_match(tr, gpu, tol=1e-9, decisive=1e-10, spread=None):
    """Per-iteration trial and accepted costs agree to relative `tol`, or to
    SPREAD_FACTOR times the oracle's own per-iteration spread under permuted
    observation orders where that is given and larger.  Accept/reject
    decisions (and so lambda) must agree while the oracle's cost change is
    above round-off (|F - F_trial| > decisive * F, or above the spread
    bound); once the solve has converged the gain ratio is a ratio of
    rounding errors and either decision is correct.  A trial point whose
    cost rises more than tenfold must be rejected by both sides."""
    if spread is None:
        spread = tr.get("spread")
    assert gpu["status"] == 0
    assert gpu["iters_run"] == tr["iters_run"]
    assert abs(gpu["initial_cost"] - tr["initial_cost"]) <= 1e-13 * tr["initial_cost"]
    np.testing.assert_array_equal(gpu["pcg_iters"], tr["pcg_iters"])
    # the oracle ran to its rtol (converged or cap) and the GPU replayed its counts
    replayed = np.where(np.isin(tr["pcg_stop"], (orc.PCG_BREAKDOWN, orc.PCG_DIRECT)), tr["pcg_stop"], orc.PCG_FIXED)
    np.testing.assert_array_equal(gpu["pcg_stop"], replayed)
    prev = tr["initial_cost"]
    same_path = True
    for k in range(tr["iters_run"]):
        ft = tr["trial_cost"][k]
        rel = tol if spread is None else max(tol, SPREAD_FACTOR * spread["trial"][k])
        crel = tol if spread is None else max(tol, SPREAD_FACTOR * spread["cost"][k])
        wild = ft > 10 * prev
        assert abs(gpu["trial_cost"][k] - ft) <= rel * ft, (k, gpu["trial_cost"][k], ft, rel)
        assert abs(gpu["cost"][k] - tr["cost"][k]) <= max(rel * ft, crel * tr["cost"][k]), k
        if wild:
            assert not gpu["accepted"][k] and not tr["accepted"][k], k
        if abs(prev - ft) > max(decisive, 2 * rel) * prev and same_path:
            assert gpu["accepted"][k] == tr["accepted"][k], k
            assert abs(gpu["lambda"][k] - tr["lambda"][k]) <= 1e-6 * tr["lambda"][k], k
        else:
            same_path = False
        prev = tr["cost"][k]


def test_lm_trace_fp64_tiny(tiny):
    tr, gpu, prob, (co, po) = lm_pair(tiny)
    assert_traces_match(tr, gpu)
    c, p = prob.get_params()
    assert rel_err(c, co) <= 1e-6 and rel_err(p, po) <= 1e-6


def test_lm_trace_fp64_huber_edge_cases():
    arrays = with_edge_cases(small_zipf(seed=11, m=20, n=400, N=2400))
    tr, gpu, prob, _ = lm_pair(arrays, delta=1.0, iters=8, max_pcg=60, rtol=1e-8)
    assert_traces_match(tr, gpu)


def test_lm_rtol_mode_agrees(tiny):
    cams, pts, oc, op, uv = tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv
    _, _, tr, rc = orc.lm_solve(cams, pts, oc, op, uv, max_lm_iters=10, max_pcg_iters=50, pcg_rtol=1e-8)
    prob, _ = make(tiny)
    gpu = prob.lm_solve(max_lm_iters=10, max_pcg_iters=50, pcg_rtol=1e-8)
    # decisions above round-off agree; PCG counts differ by at most one
    prev = tr["initial_cost"]
    for k in range(10):
        if abs(prev - tr["trial_cost"][k]) <= 1e-10 * prev:
            break
        assert gpu["accepted"][k] == tr["accepted"][k], k
        assert abs(int(gpu["pcg_iters"][k]) - int(tr["pcg_iters"][k])) <= 1, k
        # a solve that stops short of the cap has met the residual test
        stop = orc.PCG_CAP if gpu["pcg_iters"][k] >= 50 else orc.PCG_CONVERGED
        assert gpu["pcg_stop"][k] == stop, k
        prev = tr["cost"][k]
    assert abs(gpu["final_cost"] - tr["final_cost"]) <= 1e-9 * tr["final_cost"]


def test_mixed_precision_reaches_oracle_cost(tiny):
    cams, pts, oc, op, uv = tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv
    _, _, tr, rc = orc.lm_solve(cams, pts, oc, op, uv, max_lm_iters=10, max_pcg_iters=50, pcg_rtol=1e-8)
    prob, _ = make(tiny, precision=FP32_MIXED)
    gpu = prob.lm_solve(max_lm_iters=10, max_pcg_iters=50, pcg_rtol=1e-8)
    assert gpu["status"] == 0
    assert np.all(np.diff(np.concatenate([[gpu["initial_cost"]], gpu["cost"]])) <= 0)
    assert gpu["final_cost"] <= tr["final_cost"] * (1 + 1e-4)


def test_lm_monotone_and_state_consistent(tiny):
    prob, _ = make(tiny)
    gpu = prob.lm_solve(max_lm_iters=6, max_pcg_iters=50, pcg_rtol=1e-8)
    costs = np.concatenate([[gpu["initial_cost"]], gpu["cost"]])
    assert np.all(np.diff(costs) <= 0)
    assert abs(prob.cost() - gpu["final_cost"]) <= 1e-13 * gpu["final_cost"]
    c, p = prob.get_params()
    assert abs(orc.cost(c, p, tiny.obs_camera, tiny.obs_point, tiny.obs_uv) - gpu["final_cost"]) \
        <= 1e-12 * gpu["final_cost"]


@pytest.mark.parametrize("stored", [0, 1])
@pytest.mark.parametrize("hot,cached", [(0, 0), (3, 5), (7, 2), (0, 15), (7, 15)])
def test_hot_cold_split_matches_oracle(hot, cached, stored, monkeypatch):
    """The Schur product splits cameras into an LDS-held hot set and a
    camera-major cold stream, and the recomputing product reads the camera
    records of its first `cached` cameras from an LDS copy and the others
    from memory; every split gives the oracle's product and LM trace (with a
    point longer than one tile in the problem), both for the product that
    recomputes E from the Jacobian and for the one that reads the stored
    blocks (which keeps no camera records)."""
    monkeypatch.setenv("BA_HOT_CAMERAS", str(hot))
    monkeypatch.setenv("BA_CACHE_CAMERAS", str(cached))
    monkeypatch.setenv("BA_SCHUR_STORED", str(stored))
    arrays = with_edge_cases(small_zipf(seed=13, m=14, n=300, N=1500))
    cams, pts, oc, op, uv, _ = arrays
    for precision in (FP64, FP32_MIXED):
        prob, _ = make(arrays, precision=precision, huber_delta=1.0)
        lam = 1e-3
        A = orc.assemble(cams, pts, oc, op, uv, 1.0)
        Bd, Cd, Dc, Dp = orc.damp(A["B"], A["C"], lam, 0)
        Ci = orc.invert_points(Cd)
        x = np.random.default_rng(hot).normal(size=(len(cams), 9))
        ref = orc.schur_matvec(oc, op, Bd, A["E"], Ci, x)
        tol = 1e-10 if precision == FP64 else FP32_PRODUCT_TOL
        err = rel_err_rows(prob.schur_matvec(x, lam), ref)
        print(f"hot {hot} cached {cached} stored {stored} precision {precision}: product error {err:.2e} of each row")
        assert err <= tol, precision
        prob.close()
    tr, gpu, prob, _ = lm_pair(arrays, delta=1.0, iters=5, max_pcg=40, rtol=1e-8)
    assert_traces_match(tr, gpu)


@pytest.mark.parametrize("precision", [FP64, FP32_MIXED])
def test_without_hot_table_runs_are_bitwise_repeatable(precision, monkeypatch):
    """With no LDS hot table (BA_HOT_CAMERAS=0) every sum of the solve runs in
    a fixed order (segmented scans, fixed slots, ordered last-block and slot
    reductions), so two solves from the same state give the same bits: the
    deterministic mode.  The table's LDS atomics are the only order the
    hardware chooses."""
    monkeypatch.setenv("BA_HOT_CAMERAS", "0")
    arrays = with_edge_cases(small_zipf(seed=17, m=16, n=400, N=2500))
    runs = []
    for _ in range(2):
        prob, _ = make(arrays[:5], precision=precision, huber_delta=1.0)
        rep = prob.lm_solve(max_lm_iters=5, max_pcg_iters=40, pcg_rtol=1e-8)
        assert rep["status"] == 0
        runs.append((rep, prob.get_params()))
        prob.close()
    (r0, p0), (r1, p1) = runs
    for key in ("cost", "trial_cost", "lambda", "pcg_iters", "accepted"):
        np.testing.assert_array_equal(r0[key], r1[key], err_msg=key)
    np.testing.assert_array_equal(p0[0], p1[0])
    np.testing.assert_array_equal(p0[1], p1[1])


def zero_rotation_variant(arrays):
    """The same problem with camera 0's angle-axis set to exactly zero (the
    first-order branch of the rotation)."""
    cams = np.array(arrays[0], copy=True)
    cams[0, :3] = 0.0
    return (cams,) + tuple(arrays[1:5])


@pytest.mark.parametrize("edge", [False, True])
def test_autodiff_jacobian_cost_gradient_matvec(tiny, edge):
    """Forward-mode autodiff Jacobians (the paper's "-a" form): cost, gradient
    and the reduced-system product match the oracle as tightly as the analytic
    form does, including a camera at exactly zero rotation."""
    src = (tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv)
    arrays = zero_rotation_variant(with_edge_cases(small_zipf(seed=7))[:5] if edge else src)
    cams, pts, oc, op, uv = arrays
    prob = Problem(cams, pts, oc, op, uv, huber_delta=1.0, jacobian=1)
    F, gc, gp = prob.eval_cost_grad()
    Fo, gco, gpo = orc.gradient(cams, pts, oc, op, uv, 1.0)
    assert abs(F - Fo) <= 1e-13 * abs(Fo)
    assert rel_err_rows(gc, gco) <= 1e-10 and rel_err_rows(gp, gpo) <= 1e-10
    lam = 1e-2
    A = orc.assemble(cams, pts, oc, op, uv, 1.0)
    Bd, Cd, Dc, Dp = orc.damp(A["B"], A["C"], lam, 0)
    Ci = orc.invert_points(Cd)
    x = np.random.default_rng(5).normal(size=(len(cams), 9))
    ref = orc.schur_matvec(oc, op, Bd, A["E"], Ci, x)
    assert rel_err_rows(prob.schur_matvec(x, lam), ref) <= 1e-10
    prob.close()
    mixed = Problem(cams, pts, oc, op, uv, precision=FP32_MIXED, huber_delta=1.0, jacobian=1)
    err = rel_err_rows(mixed.schur_matvec(x, lam), ref)
    print(f"autodiff edge={edge}: FP32-mixed product error {err:.2e} of each row")
    assert err <= FP32_PRODUCT_TOL
    mixed.close()


def test_autodiff_lm_trace_matches_oracle(tiny):
    """An FP64 LM solve with autodiff Jacobians replays the oracle's trace."""
    arrays = zero_rotation_variant((tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv))
    cams, pts, oc, op, uv = arrays
    _, _, tr, rc = orc.lm_solve(cams, pts, oc, op, uv, huber_delta=1.0, max_lm_iters=8, max_pcg_iters=50,
                                pcg_rtol=1e-8)
    assert rc == 0
    tr["spread"] = oracle_spread(arrays, tr, huber_delta=1.0)
    prob = Problem(cams, pts, oc, op, uv, huber_delta=1.0)
    gpu = prob.lm_solve(max_lm_iters=8, pcg_schedule=tr["pcg_iters"], max_pcg_iters=50, pcg_rtol=1e-8, jacobian=1)
    prob.close()
    assert_traces_match(tr, gpu)


def narrow_baseline(seed=0, m=3, n=400, base=0.01, depth=100.0):
    """Cameras 0.01 apart on a line, facing points about 100 away; every point
    is seen by two neighbouring cameras, so its rays meet at ~1e-4 rad and its
    block C_i, scaled to unit diagonal, has a smallest eigenvalue of 1e-8 ..
    3e-6.  Rounding each float product of the Jacobian to float would move
    those eigenvalues by up to ~6e-8 and leave about a sixth of the blocks
    indefinite (checked by emulating float products on the oracle's
    Jacobians)."""
    rng = np.random.default_rng(seed)
    cams = np.zeros((m, 9))
    cams[:, :3] = rng.normal(scale=1e-3, size=(m, 3))
    cams[:, 3] = base * np.arange(m)
    cams[:, 6] = 500.0
    cams[:, 7], cams[:, 8] = -1e-7, 1e-13
    pts = np.column_stack([rng.uniform(-30, 30, n), rng.uniform(-30, 30, n), -depth + rng.uniform(-10, 10, n)])
    j = np.arange(n) % (m - 1)
    oc = np.column_stack([j, j + 1]).ravel().astype(np.int32)
    op = np.repeat(np.arange(n), 2).astype(np.int32)
    uv = np.array([orc.project(cams[a], pts[b]) for a, b in zip(oc, op)])
    uv += rng.normal(scale=0.5, size=uv.shape)
    return cams, pts, oc, op, uv


def test_mixed_blocks_factor_at_narrow_baselines():
    """The FP32-mixed form forms every product of its Gram blocks B_j and C_i
    in FP64 from the float Jacobian, so the blocks stay positive semidefinite
    and their damped forms factor wherever the FP64 form's do, down to
    lambda = 0, on two-view points whose rays nearly coincide.  The FP64
    product matches the oracle's at lambda 1e-6."""
    arrays = narrow_baseline()
    cams, pts, oc, op, uv = arrays
    x = np.random.default_rng(3).normal(size=(len(cams), 9))
    A = orc.assemble(cams, pts, oc, op, uv, 0.0)
    Bd, Cd, _, _ = orc.damp(A["B"], A["C"], 1e-6, 0)
    ref = orc.schur_matvec(oc, op, Bd, A["E"], orc.invert_points(Cd), x)
    for precision in (FP64, FP32_MIXED):
        prob, _ = make(arrays, precision=precision)
        for lam in (1e-6, 1e-12, 0.0):
            q = prob.schur_matvec(x, lam)
            assert np.all(np.isfinite(q)), (precision, lam)
            if precision == FP64 and lam == 1e-6:
                assert rel_err(q, ref) <= 1e-7
        prob.close()


@pytest.mark.parametrize("hot", [None, 400])
def test_synthesised_recipe_matches_oracle(hot, monkeypatch):
    """The synthesised recipe at oracle size (400 cameras, 1,600 points seen
    300 times each: every point spans five or six tiles), with the library's
    own choice of hot set and with all 400 cameras forced hot (every long
    point walked twice).  Both give the oracle's product and FP64 LM trace.
    The problem has a zero-cost optimum: four iterations take the cost from
    1.8e5 to 0.64, so the late trial costs are small next to the rounding
    carried in the step, and the oracle's own trace moves by up to 5e-8
    relative when only its summation order changes (stored permuted runs);
    the trace is compared to that spread."""
    if hot is not None:
        monkeypatch.setenv("BA_HOT_CAMERAS", str(hot))
    prob = synth.generate("synth_small", seed=0)
    arrays = (prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv)
    cams, pts, oc, op, uv = arrays
    lam = 1e-3
    A = orc.assemble(cams, pts, oc, op, uv, 0.0)
    Bd, Cd, _, _ = orc.damp(A["B"], A["C"], lam, 0)
    x = np.random.default_rng(11).normal(size=(len(cams), 9))
    ref = orc.schur_matvec(oc, op, Bd, A["E"], orc.invert_points(Cd), x)
    for precision in (FP64, FP32_MIXED):
        gpu, _ = make(arrays, precision=precision)
        tol = 1e-10 if precision == FP64 else FP32_PRODUCT_TOL
        err = rel_err_rows(gpu.schur_matvec(x, lam), ref)
        print(f"synthesised recipe, hot {hot}, precision {precision}: product error {err:.2e} of each row")
        assert err <= tol, precision
        gpu.close()
    tr, rep, _, _ = lm_pair(arrays, iters=4, max_pcg=30, rtol=1e-8, spread=False)
    spread = order_spread("synth_small")
    assert spread is not None, "tests/golden/order_spread_synth_small_seed*.json missing"
    np.testing.assert_array_equal(tr["trial_cost"], spread["trace"]["trial_cost"])  # the same oracle run
    assert_traces_match(tr, rep, spread=spread)


def test_mixed_point_at_camera_centre(monkeypatch):
    """A point within FP32 resolution of a camera's centre (LM can drift there
    when a point's other views are outliers: every projection is available
    from the centre) has a depth made of rounding in FP32.  The FP32-mixed
    form forms that observation's geometry in FP64 from the FP64 camera
    constants and point (and stores it in FP32), so the blocks, the product
    and the LM step stay finite; the FP64 form needs no such step.  With no
    hot cameras the observation goes through the camera-major cold pass,
    which finds the point through its record: its mixed product matches the
    point-major pass's.  (Against the FP64 product the mixed rows of the two
    cameras that see this point differ by ~1e-2: their terms reach 1e7 times
    the others' and cancel, so float rounding of the geometry shows there.)"""
    from scipy.spatial.transform import Rotation

    prob = synth.generate("tiny", seed=0)
    cams, pts = prob.cameras0.copy(), prob.points0.copy()
    R = Rotation.from_rotvec(cams[0, :3]).as_matrix()
    centre = -R.T @ cams[0, 3:6]
    X = centre - 1e-7 * R[2]  # just in front of camera 0, on its optical axis
    pts = np.vstack([pts, X])
    i = len(pts) - 1
    oc = np.concatenate([prob.obs_camera, [0, 1]]).astype(np.int32)
    op = np.concatenate([prob.obs_point, [i, i]]).astype(np.int32)
    uv = np.vstack([prob.obs_uv, [[12.0, -7.0], orc.project(cams[1], X) + 0.3]])
    x = np.random.default_rng(2).normal(size=(len(cams), 9))
    q = {}
    for precision, hot in ((FP64, None), (FP32_MIXED, None), (FP32_MIXED, 0)):
        if hot is not None:
            monkeypatch.setenv("BA_HOT_CAMERAS", str(hot))
        gpu, _ = make((cams, pts, oc, op, uv), precision=precision, huber_delta=1.0)
        F, gc, gp = gpu.eval_cost_grad()
        assert np.isfinite(F) and np.all(np.isfinite(gc)) and np.all(np.isfinite(gp)), precision
        q[precision, hot] = gpu.schur_matvec(x, 1e-3)
        assert np.all(np.isfinite(q[precision, hot])), precision
        rep = gpu.lm_solve(max_lm_iters=3, max_pcg_iters=30, pcg_rtol=1e-6)
        assert rep["status"] == 0, (precision, rep["error"])
        assert np.all(np.diff(np.concatenate([[rep["initial_cost"]], rep["cost"]])) <= 0)
        gpu.close()
    err = rel_err_rows(q[FP32_MIXED, 0], q[FP32_MIXED, None])
    far = rel_err_rows(q[FP32_MIXED, None], q[FP64, None])
    print(f"cold pass against point-major pass (mixed): {err:.2e} of each row; mixed against FP64 {far:.1e}")
    assert err <= FP32_PRODUCT_TOL


def dense_pair(arrays, delta=0.0, iters=6, precision=FP64):
    """The oracle's LM trace with the reduced camera system written out and
    factored, beside the library's direct option on the same problem."""
    cams, pts, oc, op, uv = arrays[:5]
    _, _, tr, rc = orc.lm_solve(cams, pts, oc, op, uv, huber_delta=delta, max_lm_iters=iters, solver=1)
    assert rc == 0
    tr["spread"] = oracle_spread(arrays, tr, huber_delta=delta, solver=1)
    prob, _ = make(arrays[:5], precision=precision, huber_delta=delta, solver=SOLVER_DENSE)
    gpu = prob.lm_solve(max_lm_iters=iters)
    return tr, gpu, prob


def test_dense_solver_trace_tiny(tiny):
    """Direct option on the tiny problem: 9m = 144 rows, two full tiles of
    the factorisation and a ragged one."""
    arrays = (tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv)
    tr, gpu, prob = dense_pair(arrays, iters=10)
    assert np.all(gpu["pcg_iters"] == 0)
    assert_traces_match(tr, gpu)
    co, po = orc.lm_solve(*arrays, max_lm_iters=10, solver=1)[:2]
    c, p = prob.get_params()
    assert rel_err(c, co) <= 1e-6 and rel_err(p, po) <= 1e-6


@pytest.mark.parametrize("stored", [0, 1])
def test_dense_solver_trace_edge_cases(stored, monkeypatch):
    """Huber loss, an unseen camera, single-view points, a duplicated pair
    and a point of 300 views (whose Schur terms span 5 x 5 row pairs), for
    either right-hand-side product."""
    monkeypatch.setenv("BA_SCHUR_STORED", str(stored))
    arrays = with_edge_cases(small_zipf(seed=13, m=14, n=300, N=1500))
    tr, gpu, _ = dense_pair(arrays, delta=1.0, iters=6)
    assert_traces_match(tr, gpu)


def test_dense_solver_trace_many_tiles():
    """150 cameras: 9m = 1350 rows, 21 full 64-row tiles and a ragged one,
    so every step of the tiled factorisation runs many times."""
    arrays = small_zipf(seed=5, m=150, n=2500, N=15000)
    arrays = (arrays.cameras0, arrays.points0, arrays.obs_camera, arrays.obs_point, arrays.obs_uv)
    tr, gpu, _ = dense_pair(arrays, delta=1.0, iters=4)
    assert_traces_match(tr, gpu)


def test_dense_solver_mixed_reaches_oracle_cost(tiny):
    arrays = (tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv)
    tr, gpu, _ = dense_pair(arrays, iters=10, precision=FP32_MIXED)
    assert gpu["status"] == 0, gpu["error"]
    assert np.all(np.diff(np.concatenate([[gpu["initial_cost"]], gpu["cost"]])) <= 0)
    assert gpu["final_cost"] <= tr["final_cost"] * (1 + 1e-4)


def test_dense_solver_matches_converged_pcg(tiny):
    """The direct step is the limit of PCG: with a tight tolerance and
    enough iterations the two options follow the same LM path."""
    arrays = (tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv)
    dense, _ = make(arrays, solver=SOLVER_DENSE)
    pcg, _ = make(arrays)
    a = dense.lm_solve(max_lm_iters=5)
    b = pcg.lm_solve(max_lm_iters=5, max_pcg_iters=500, pcg_rtol=1e-14)
    assert a["status"] == 0 and b["status"] == 0
    np.testing.assert_array_equal(a["accepted"], b["accepted"])
    np.testing.assert_allclose(a["cost"], b["cost"], rtol=1e-8)
    with pytest.raises(Exception, match="solver differs"):
        dense.lm_solve(max_lm_iters=1, solver=0)


def schur_jacobi_pair(arrays, delta=0.0, iters=8, max_pcg=60, rtol=1e-8, precision=FP64, **opts):
    """Oracle and library LM traces with the Schur-Jacobi preconditioner; the
    library replays the oracle's PCG counts."""
    cams, pts, oc, op, uv = arrays[:5]
    _, _, tr, rc = orc.lm_solve(cams, pts, oc, op, uv, huber_delta=delta, max_lm_iters=iters,
                                max_pcg_iters=max_pcg, pcg_rtol=rtol, preconditioner=1)
    assert rc == 0
    tr["spread"] = oracle_spread(arrays, tr, huber_delta=delta, preconditioner=1)
    prob, _ = make(arrays[:5], precision=precision, huber_delta=delta, preconditioner=PRECOND_SCHUR_JACOBI,
                   **opts)
    gpu = prob.lm_solve(max_lm_iters=iters, pcg_schedule=tr["pcg_iters"], max_pcg_iters=max_pcg, pcg_rtol=rtol)
    return tr, gpu, prob


def test_schur_jacobi_trace_tiny(tiny):
    arrays = (tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv)
    tr, gpu, _ = schur_jacobi_pair(arrays, iters=10, max_pcg=50)
    assert_traces_match(tr, gpu)


@pytest.mark.parametrize("jacobian", [0, 1])
def test_schur_jacobi_trace_edge_cases(jacobian):
    """Huber loss, an unseen camera (no Schur term: M_j = B~_j), a repeated
    pair (no cross term) and a point of 300 views; analytic and
    forward-mode Jacobians."""
    arrays = with_edge_cases(small_zipf(seed=13, m=14, n=300, N=1500))
    tr, gpu, _ = schur_jacobi_pair(arrays, delta=1.0, iters=6, jacobian=jacobian)
    assert_traces_match(tr, gpu)


def test_schur_jacobi_changes_the_preconditioner(tiny):
    """The option reaches the solver: in tolerance mode the PCG counts follow
    the oracle's with Schur-Jacobi blocks, not with the camera blocks."""
    arrays = (tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv)
    cams, pts, oc, op, uv = arrays
    sj = orc.lm_solve(cams, pts, oc, op, uv, max_lm_iters=1, max_pcg_iters=200, pcg_rtol=1e-8, preconditioner=1)[2]
    cb = orc.lm_solve(cams, pts, oc, op, uv, max_lm_iters=1, max_pcg_iters=200, pcg_rtol=1e-8)[2]
    prob, _ = make(arrays)
    a = prob.lm_solve(max_lm_iters=1, max_pcg_iters=200, pcg_rtol=1e-8, preconditioner=PRECOND_SCHUR_JACOBI)
    prob.close()
    prob, _ = make(arrays)
    b = prob.lm_solve(max_lm_iters=1, max_pcg_iters=200, pcg_rtol=1e-8)
    assert abs(int(a["pcg_iters"][0]) - int(sj["pcg_iters"][0])) <= 1
    assert abs(int(b["pcg_iters"][0]) - int(cb["pcg_iters"][0])) <= 1


def test_schur_jacobi_mixed_reaches_oracle_cost(tiny):
    arrays = (tiny.cameras0, tiny.points0, tiny.obs_camera, tiny.obs_point, tiny.obs_uv)
    cams, pts, oc, op, uv = arrays
    _, _, tr, rc = orc.lm_solve(cams, pts, oc, op, uv, max_lm_iters=10, max_pcg_iters=50, pcg_rtol=1e-8,
                                preconditioner=1)
    prob, _ = make(arrays, precision=FP32_MIXED, preconditioner=PRECOND_SCHUR_JACOBI)
    gpu = prob.lm_solve(max_lm_iters=10, max_pcg_iters=50, pcg_rtol=1e-8)
    assert gpu["status"] == 0, gpu["error"]
    assert np.all(np.diff(np.concatenate([[gpu["initial_cost"]], gpu["cost"]])) <= 0)
    assert gpu["final_cost"] <= tr["final_cost"] * (1 + 1e-4)
