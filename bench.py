"""Benchmark: LM iterations/s and Schur-PCG iterations/s of the bundle-
adjustment LM step on one MI355X, FP32-mixed and FP64.

A step is one LM iteration (residual/Jacobian, Schur block assembly, damping,
reduced right-hand side, block-Jacobi PCG with implicit Schur matvecs,
back-substitution, trial cost and the accept/reject decision) over the whole
synthetic problem, whose inputs are resident in device memory before timing.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]

Prints one JSON line.  `value` is the FP32-mixed LM iterations per second;
the FP64 figures and the PCG rates ride along in the same line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PCG_STOP_NAMES = ("converged", "cap", "breakdown", "fixed", "direct")  # ba_pcg_stop (include/ba.h)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed instructions (this build compiles with packed
# FP32 off): 256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2.4 GHz; the
# published 157.3 TFLOP/s counts the packed (two-wide) FMA
FP32_UNPACKED_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# wavefront VALU instructions the chip can issue per second: 256 CUs x 4 SIMDs,
# one wave64 instruction per SIMD every 4 cycles at 2.4 GHz
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
# L1 (TCP) cache-line lookups per second: about one per CU per cycle
L1_LOOKUPS_PER_S = 256 * 2.4e9
WORKLOADS = {  # name -> synth config and solver settings
    "large": dict(config="large", huber_delta=1.0, max_pcg_iters=100, pcg_rtol=1e-6),
    "medium": dict(config="medium", huber_delta=0.0, max_pcg_iters=100, pcg_rtol=1e-6),
    "stress": dict(config="stress", huber_delta=1.0, max_pcg_iters=200, pcg_rtol=1e-6),
    # one GPU's share of the 29M workload split over 8 GPUs (point-aligned edge partition)
    "large_chunk8": dict(config="large", chunk=(0, 8), huber_delta=1.0, max_pcg_iters=100, pcg_rtol=1e-6),
    "tiny": dict(config="tiny", huber_delta=0.0, max_pcg_iters=50, pcg_rtol=1e-8),
    # the paper's synthesised problem: 20,000 cameras, 80,000 points seen 1,000 times each
    "synth20000": dict(config="synth20000", huber_delta=0.0, max_pcg_iters=100, pcg_rtol=1e-6),
    "synth_small": dict(config="synth_small", huber_delta=0.0, max_pcg_iters=100, pcg_rtol=1e-6),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def matvec_algorithmic_bytes(m, n, N, w):
    """One-pass minimum bytes of one implicit Schur matvec: every coupling
    block (27 words) and its camera index once, every damped point inverse
    (6 words) and point offset once, camera vectors in and out and the
    damped camera blocks (45 words)."""
    return N * (27 * w + 4) + n * (6 * w + 4) + m * (9 * w * 2 + 45 * w)


def hot_pass_algorithmic_bytes(n, N, w):
    """The share of the one-pass minimum that the point-major pass (the
    dominant kernel) must move: the observation and point terms."""
    return N * (27 * w + 4) + n * (6 * w + 4)


def free_pass_algorithmic_flops(n, N):
    """Arithmetic of the point-major pass when E is formed from the Jacobian
    (an FMA counts 2): per observation the geometry (de/dP, projection, lever
    arm: 57), E_k^T x in factored form (57), the camera side E_k b (51), the
    point sum (3) and the camera sum (9); per point b_i = C~_i^-1 a_i (15)."""
    return N * (57 + 57 + 51 + 3 + 9) + n * 15


def schur_product_kind():
    """The point-major kernel the library runs: it forms E from the Jacobian
    unless BA_SCHUR_STORED=1 selects the stored blocks (read at creation)."""
    return "stored" if os.environ.get("BA_SCHUR_STORED", "0") not in ("", "0") else "recompute"


COUNTER_FILES = {"k_schur_hot<float>": "schur_hot_stored_29M_hbm_counters.md",
                 "k_schur_free<float>": "schur_free_29M_counters.md"}
# the sources the point-major product kernels are built from (their hash
# dates a counter summary)
COUNTER_SOURCES = ("matvec.hip", "ba_internal.h", "camera_model.h", "camera_cache.h", "wave_ops.h")


def counted(kernel):
    """Per-launch figures of `kernel` from its committed rocprofv3 counter
    summary (HBM bytes from FETCH_SIZE and WRITE_SIZE scaled by a plain copy's
    reading; VALU instructions where taken), or {} when the kernel sources have
    changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", COUNTER_FILES[kernel])
    if not os.path.exists(path):
        return {}
    fields = {}
    for line in open(path):
        key, sep, val = line.strip().partition(": ")
        if sep:
            fields[key] = val
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
        path = os.path.join(ROOT, "paper_2112_01349_amd", "csrc", f)
        if not os.path.exists(path):
            return {}
        h.update(open(path, "rb").read())
    if fields.get("kernel") != kernel or fields.get("source_sha256") != h.hexdigest()[:16]:
        return {}
    return {k: float(v) for k, v in fields.items() if k.endswith("_per_launch")}


def roofline(s32, m, n, N, counters_apply, s64=None):
    """Roofline entry of the dominant kernel, the FP32 point-major pass of the
    implicit Schur product.  `achieved` is the algorithmic bytes of one launch
    (the one-pass minimum of the product's point-major half: every coupling
    block and camera index once, every damped point inverse and offset once)
    over its mean duration, against the HBM peak.  The default kernel forms E
    from the Jacobian instead of reading it, so it moves far fewer bytes than
    that (`traffic`, counted); its own limit is VALU issue (`valu_issue_frac`)."""
    ms = s32["hot_kernel_ms"]
    alg = hot_pass_algorithmic_bytes(n, N, 4)
    gbs = alg / (ms * 1e-3) / 1e9
    stored = schur_product_kind() == "stored"
    kernel = "k_schur_hot<float>" if stored else "k_schur_free<float>"
    c = counted(kernel) if counters_apply else {}
    traffic = c.get("traffic_bytes_per_launch")
    mv_alg = matvec_algorithmic_bytes(m, n, N, 4)
    out = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "traffic": traffic,
           "kernel": kernel + (" (point-major pass of the implicit Schur product, stored E)" if stored else
                               " (point-major pass of the implicit Schur product, E formed from the Jacobian)"),
           "bytes_per_launch": alg, "avg_ms": ms,
           # (i) counted HBM traffic over the same duration
           "counted_gbs": traffic / (ms * 1e-3) / 1e9 if traffic else None,
           "counted_frac": traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
           # (ii) the whole product (every kernel of one matvec) against its one-pass minimum
           "matvec_bytes": mv_alg, "matvec_ms": s32["matvec_ms"],
           "matvec_frac": mv_alg / (s32["matvec_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if not stored:
        flops = free_pass_algorithmic_flops(n, N)
        tflops = flops / (ms * 1e-3) / 1e12
        insts = c.get("valu_insts_per_launch")
        lookups = c.get("l1_lookups_per_launch")
        out.update(alu_flops_per_launch=flops, alu_tflops=tflops, alu_peak_tflops=FP32_UNPACKED_PEAK_TFLOPS,
                   alu_frac=tflops / FP32_UNPACKED_PEAK_TFLOPS,
                   valu_issue_frac=(insts / VALU_ISSUE_PER_S) / (ms * 1e-3) if insts else None,
                   # L1 line lookups against one per CU per cycle (the limit of per-lane gathers)
                   l1_lookup_frac=(lookups / L1_LOOKUPS_PER_S) / (ms * 1e-3) if lookups else None,
                   note="E is formed again from the Jacobian, so the algorithmic bytes bound a design that "
                        "stores E, not this kernel (frac can pass 1); its limits are VALU issue and L1 line "
                        "lookups of the per-lane camera gathers")
    if s64 is not None:
        alg64 = hot_pass_algorithmic_bytes(n, N, 8)
        mv64 = matvec_algorithmic_bytes(m, n, N, 8)
        out["fp64"] = {"avg_ms": s64["hot_kernel_ms"], "bytes_per_launch": alg64,
                       "frac": alg64 / (s64["hot_kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "matvec_ms": s64["matvec_ms"], "matvec_bytes": mv64,
                       "matvec_frac": mv64 / (s64["matvec_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def load_golden(name):
    """The oracle's stored LM trace and final parameters for a workload, or None."""
    path = os.path.join(ROOT, "tests", "golden", f"lm_trace_{name}.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    ppath = os.path.join(ROOT, "tests", "golden", f"lm_params_{name}.npz")
    if os.path.exists(ppath):
        with np.load(ppath) as z:
            g["params"] = {k: z[k] for k in z.files}
    return g


def oracle_errors(rep, params, golden, steps):
    """Final cost and parameters of a timed solve against the oracle's run of
    the same number of LM iterations (relative errors; parameters as
    relative 2-norms over all cameras and over the stored point sample)."""
    if golden is None or steps > golden["iters_run"]:
        return None
    F_orc = golden["cost"][steps - 1]
    out = {"oracle_iterations": steps, "oracle_cost": F_orc, "final_cost_rel_err": rep["final_cost"] / F_orc - 1.0}
    gp = golden.get("params")
    if gp is not None and steps == golden["iters_run"] and params is not None:
        cams, pts = params
        sel = gp["point_index"]
        out["cameras_rel_err"] = float(np.linalg.norm(cams - gp["cameras"]) / np.linalg.norm(gp["cameras"]))
        out["points_rel_err"] = float(np.linalg.norm(pts[sel] - gp["points"]) / np.linalg.norm(gp["points"]))
        out["points_sampled"] = int(len(sel))
        # per point and per camera: a few weakly constrained points (depth
        # along a narrow baseline) can dominate the 2-norm above
        for name, a, b in (("cameras", cams, gp["cameras"]), ("points", pts[sel], gp["points"])):
            e = np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)
            out[f"{name}_rel_err_median"] = float(np.median(e))
            out[f"{name}_rel_err_p99"] = float(np.quantile(e, 0.99))
            out[f"{name}_rel_err_max"] = float(e.max())
    return out


def run_precision(prob_data, precision, wl, steps, warmup, jacobian=0, solver=0, preconditioner=0):
    import torch

    from paper_2112_01349_amd import Problem

    cams, pts, oc, op, uv = prob_data
    t0 = time.perf_counter()
    prob = Problem(cams, pts, oc, op, uv, precision=precision, huber_delta=wl["huber_delta"],
                   max_pcg_iters=wl["max_pcg_iters"], pcg_rtol=wl["pcg_rtol"], jacobian=jacobian, solver=solver,
                   preconditioner=preconditioner)
    device_bytes = prob.memory_bytes()
    log(f"[bench] precision={precision} create {time.perf_counter() - t0:.1f}s "
        f"device bytes {device_bytes / 1e9:.2f} GB")
    if warmup > 0:
        prob.lm_solve(max_lm_iters=warmup)
        prob.set_params(cams, pts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = prob.lm_solve(max_lm_iters=steps, time_kernels=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] precision={precision} {steps} LM iters in {wall:.3f}s; pcg {rep['pcg_iters'].tolist()} "
        f"stops {[PCG_STOP_NAMES[k] for k in rep['pcg_stop']]} "
        f"accepted {rep['accepted'].tolist()} cost {rep['initial_cost']:.6g} -> {rep['final_cost']:.6g}")
    rep["params"] = prob.get_params()   # after the timed region
    prob.close()
    rep["device_bytes"] = device_bytes
    return rep, wall


def time_to_cost(rep, target):
    """Wall time (ms) of the LM iterations until the accepted cost first
    reaches `target`, or None."""
    t = 0.0
    for c, ms in zip(rep["cost"], rep["ms"]):
        t += ms
        if c <= target:
            return t
    return None


def iterations_to_cost(rep, target):
    """LM iterations until the accepted cost first reaches `target`, or None."""
    hit = np.nonzero(np.asarray(rep["cost"]) <= target)[0]
    return int(hit[0]) + 1 if len(hit) else None


def equal_cost_speedup(rep32, rep64, oracle_final=None):
    """FP64 time / FP32-mixed time to reach the target cost: the oracle's
    final cost x (1 + 1e-4) when given, else the FP64 run's.  The speedup is
    split into the product's speed (FP64 / FP32 ms per matvec) and the PCG
    work each form spent on the way (matvecs until the target)."""
    target = (oracle_final if oracle_final is not None else rep64["final_cost"]) * (1 + 1e-4)
    t64, t32 = time_to_cost(rep64, target), time_to_cost(rep32, target)
    if t64 is None or t32 is None:
        return None
    k64, k32 = iterations_to_cost(rep64, target), iterations_to_cost(rep32, target)
    out = dict(target_cost=target, target_from="oracle" if oracle_final is not None else "fp64 run",
               fp64_ms=t64, fp32_mixed_ms=t32, speedup=t64 / t32, fp64_lm_iters=k64, fp32_mixed_lm_iters=k32)
    if "matvec_ms" in rep64 and rep64.get("matvec_launches") and rep32.get("matvec_launches"):
        mv64 = rep64["matvec_ms"] / rep64["matvec_launches"]
        mv32 = rep32["matvec_ms"] / rep32["matvec_launches"]
        n64 = int(np.sum(rep64["pcg_iters"][:k64]))
        n32 = int(np.sum(rep32["pcg_iters"][:k32]))
        out.update(matvec_speed_ratio=mv64 / mv32, fp64_matvecs=n64, fp32_mixed_matvecs=n32,
                   matvec_count_ratio=n64 / max(1, n32))
    return out


def autograd_throughput(reps=5):
    """Forward + backward of HuberReprojCost on the differentiation workload
    (1,000 cameras, 200k points, 1M observations), observations per second."""
    import torch

    from paper_2112_01349_amd import Problem, synth
    from paper_2112_01349_amd.autograd import HuberReprojCost

    prob = synth.generate("diff", seed=0)
    gpu = Problem(prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv, huber_delta=1.0)
    out = {"workload": "diff: 1000 cameras, 200000 points, 1000000 observations, Huber delta=1"}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        cams = torch.tensor(prob.cameras0, dtype=dt, device="cuda", requires_grad=True)
        pts = torch.tensor(prob.points0, dtype=dt, device="cuda", requires_grad=True)
        HuberReprojCost.apply(cams, pts, gpu).backward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            cams.grad = None
            pts.grad = None
            HuberReprojCost.apply(cams, pts, gpu).backward()
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / reps
        out[f"{name}_fwd_bwd_ms"] = 1e3 * dt_s
        out[f"{name}_obs_per_s"] = prob.num_obs / dt_s
    gpu.close()
    return out


def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(prob, wl, n_pcg):
    """The FP64 oracle on a bounded sample: the observations of the first
    points (about a quarter of the problem) with every camera, one LM iteration
    with the PCG count the GPU averaged; scaled by the observation ratio."""
    from oracle import oracle as orc

    frac = 1.0 / 4.0
    n_sub = max(1, int(prob.num_points * frac))
    sel = prob.obs_point < n_sub
    oc, op, uv = prob.obs_camera[sel], prob.obs_point[sel], prob.obs_uv[sel]
    t0 = time.perf_counter()
    _, _, tr, rc = orc.lm_solve(prob.cameras0, prob.points0[:n_sub], oc, op, uv, huber_delta=wl["huber_delta"],
                                max_lm_iters=1, pcg_schedule=[max(1, int(round(n_pcg)))])
    dt = time.perf_counter() - t0
    scale = prob.num_obs / max(1, int(sel.sum()))
    model, nproc = host_cpu()
    return dict(value=1.0 / (dt * scale), unit="LM iter/s", cores=1, kind="oracle", host_cpu=model, nproc=nproc,
                sample=f"1 LM iteration (assembly + {int(round(n_pcg))} Schur matvecs + trial cost) over "
                       f"{int(sel.sum())} of {prob.num_obs} observations (first {n_sub} points, all cameras), "
                       f"{dt:.1f}s, scaled x{scale:.1f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64", type=int, default=1, help="also time the FP64 form")
    ap.add_argument("--autograd", type=int, default=1, help="also time the autograd Function (1M observations)")
    ap.add_argument("--jacobian", default="analytic", choices=["analytic", "autodiff"],
                    help="analytic Jacobians (the paper's -m) or forward-mode autodiff (-a)")
    ap.add_argument("--solver", default="pcg", choices=["pcg", "dense"],
                    help="PCG on implicit Schur products, or the reduced system written out and factored "
                         "(at most 2048 cameras)")
    ap.add_argument("--preconditioner", default="camera-blocks", choices=["camera-blocks", "schur-jacobi"],
                    help="PCG preconditioner: damped camera blocks (Alg. 2) or the Schur-Jacobi blocks")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (scale reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2112_01349_amd import FP32_MIXED, FP64, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = WORKLOADS[args.workload]
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 copies of 1 GiB done")
        del src, dst
    t0 = time.perf_counter()
    prob = synth.generate(wl["config"], seed=0)
    if "chunk" in wl:
        prob = synth.point_chunk(prob, *wl["chunk"])
    log(f"[bench] generated {args.workload}: m={prob.num_cameras} n={prob.num_points} N={prob.num_obs} "
        f"in {time.perf_counter() - t0:.1f}s")
    data = (prob.cameras0, prob.points0, prob.obs_camera, prob.obs_point, prob.obs_uv)
    m, n, N = prob.num_cameras, prob.num_points, prob.num_obs

    jac = 1 if args.jacobian == "autodiff" else 0
    variant = dict(solver=1 if args.solver == "dense" else 0,
                   preconditioner=1 if args.preconditioner == "schur-jacobi" else 0)
    rep32, wall32 = run_precision(data, FP32_MIXED, wl, args.steps, args.warmup, jac, **variant)
    res = {}
    for name, rep, wall, w in [("fp32_mixed", rep32, wall32, 4)]:
        res[name] = rep, wall, w
    if args.fp64:
        rep64, wall64 = run_precision(data, FP64, wl, args.steps, args.warmup, jac, **variant)
        res["fp64"] = rep64, wall64, 8

    def summary(rep, wall, w):
        launches = max(1, rep["matvec_launches"])
        mv_ms = rep["matvec_ms"] / launches
        hot_ms = rep["schur_hot_ms"] / launches
        out = dict(lm_iter_per_s=args.steps / wall, ms_per_lm_iter=1e3 * wall / args.steps,
                   pcg_iter_per_s=rep["pcg_iters_total"] / max(1e-9, rep["pcg_ms"] * 1e-3),
                   pcg_iters=int(rep["pcg_iters_total"]), matvec_ms=mv_ms, hot_kernel_ms=hot_ms)
        if schur_product_kind() == "stored":
            # HBM rates of the stored-block kernels (the bytes they must move)
            gbs = matvec_algorithmic_bytes(m, n, N, w) / (mv_ms * 1e-3) / 1e9
            hot_bytes = hot_pass_algorithmic_bytes(n, N, w)
            hot_gbs = hot_bytes / (hot_ms * 1e-3) / 1e9
            out.update(matvec_gbs=gbs, matvec_frac=gbs / HBM_PEAK_GBS, hot_kernel_bytes=hot_bytes,
                       hot_kernel_gbs=hot_gbs, hot_kernel_frac=hot_gbs / HBM_PEAK_GBS)
        else:
            # arithmetic rate of the recomputing pass; the bytes the stored design moves are not moved
            flops = free_pass_algorithmic_flops(n, N)
            out.update(hot_kernel_flops=flops,
                       hot_kernel_tflops=flops / (hot_ms * 1e-3) / 1e12 if hot_ms > 0 else None)
        out.update(initial_cost=rep["initial_cost"], final_cost=rep["final_cost"],
                   device_bytes=int(rep["device_bytes"]),
                   pcg_per_lm=rep["pcg_iters"].tolist(), pcg_stop=[PCG_STOP_NAMES[k] for k in rep["pcg_stop"]],
                   accepted=rep["accepted"].tolist(),
                   vs_oracle=oracle_errors(rep, rep.get("params"), golden, args.steps))
        return out

    golden = load_golden(args.workload) if args.solver == "pcg" and "chunk" not in wl else None
    if golden is not None and golden["shape"] != [m, n, N]:
        golden = None
    s32 = summary(*res["fp32_mixed"])
    out = {
        "metric": "LM iter/s + Schur-PCG iter/s (29M obs), FP32-mixed vs FP64, % HBM peak",
        "value": s32["lm_iter_per_s"],
        "unit": "LM iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": s32["ms_per_lm_iter"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64 (mixed)", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {m} cameras, {n} points, {N} observations, "
                               + (f"point-aligned chunk {wl['chunk'][0]} of {wl['chunk'][1]} of '{wl['config']}', "
                                  if "chunk" in wl else "")
                               + ("uniform visibility, " if wl["config"] in synth.CIRCLE_CONFIGS else "Zipf visibility, ")
                               + f"Huber delta={wl['huber_delta']}, {args.jacobian} Jacobians, "
                               + ("dense reduced system, Cholesky" if args.solver == "dense" else
                                  f"PCG ({args.preconditioner}) max {wl['max_pcg_iters']} rtol {wl['pcg_rtol']}"),
                   "cameras": m, "points": n, "observations": N},
        "pcg_iter_per_s": s32["pcg_iter_per_s"],
        # the roofline entry describes the PCG path's dominant kernel
        "roofline": None,
        "fp32_mixed": s32,
    }
    s64 = None
    if "fp64" in res:
        s64 = summary(*res["fp64"])
        out["fp64"] = s64
        out["mixed_speedup_lm"] = s32["lm_iter_per_s"] / s64["lm_iter_per_s"]
        oracle_final = golden["cost"][args.steps - 1] if golden and args.steps <= golden["iters_run"] else None
        out["mixed_speedup_equal_cost"] = equal_cost_speedup(res["fp32_mixed"][0], res["fp64"][0], oracle_final)
    if args.solver == "pcg":
        out["roofline"] = roofline(s32, m, n, N, args.workload == "large", s64)
    if args.autograd:
        out["autograd"] = autograd_throughput()
    if not args.no_cpu_baseline and args.solver == "pcg":
        out["cpu_baseline"] = cpu_baseline(prob, wl, s32["pcg_iters"] / max(1, args.steps))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
