"""Host-side checks of bench.py's measurement arithmetic (no GPU): the
algorithmic byte and flop counts the roofline divides by, the time-to-cost
comparison, the counter-summary parser and the one-GPU guard."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_counts_at_29m():
    n, N, m = 4_500_000, 29_000_000, 13_700
    # stored design: 27 words of E and a camera index per observation, 6 words and an offset per point
    assert bench.hot_pass_algorithmic_bytes(n, N, 4) == N * (27 * 4 + 4) + n * (6 * 4 + 4)
    assert abs(bench.hot_pass_algorithmic_bytes(n, N, 4) / 1e9 - 3.374) < 1e-3
    # the whole matvec adds the camera vectors in and out and the damped camera blocks
    assert bench.matvec_algorithmic_bytes(m, n, N, 8) - bench.hot_pass_algorithmic_bytes(n, N, 8) == \
        m * (9 * 8 * 2 + 45 * 8)
    # recomputing pass: 177 flops per observation and 15 per point
    assert bench.free_pass_algorithmic_flops(n, N) == 177 * N + 15 * n
    assert abs(bench.VALU_ISSUE_PER_S - 614.4e9) < 1.0


def test_time_to_cost_and_equal_cost_speedup():
    rep64 = dict(cost=np.array([10.0, 5.0, 2.0, 1.0]), ms=np.array([4.0, 4.0, 4.0, 4.0]), final_cost=1.0)
    rep32 = dict(cost=np.array([9.0, 4.0, 1.00005, 0.9]), ms=np.array([2.0, 2.0, 2.0, 2.0]), final_cost=0.9)
    assert bench.time_to_cost(rep64, 2.0) == 12.0
    assert bench.time_to_cost(rep64, 0.5) is None
    sp = bench.equal_cost_speedup(rep32, rep64)
    # target 1.0001: FP64 reaches it after 4 iterations (16 ms), FP32-mixed after 3 (6 ms)
    assert sp["fp64_ms"] == 16.0 and sp["fp32_mixed_ms"] == 6.0 and sp["speedup"] == pytest.approx(16.0 / 6.0)


def test_counter_summary_is_read_only_for_matching_sources(tmp_path, monkeypatch):
    kernel = "k_schur_free<float>"
    summary = os.path.join(ROOT, "profiles", bench.COUNTER_FILES[kernel])
    fake = tmp_path / "repo"
    (fake / "profiles").mkdir(parents=True)
    csrc = fake / "paper_2112_01349_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.COUNTER_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2112_01349_amd", "csrc", f), csrc / f)
    shutil.copy(summary, fake / "profiles" / os.path.basename(summary))
    monkeypatch.setattr(bench, "ROOT", str(fake))
    got = bench.counted(kernel)
    fields = dict(line.strip().partition(": ")[::2] for line in open(summary) if ": " in line)
    if got:  # the committed summary was taken from these sources
        assert got["traffic_bytes_per_launch"] == float(fields["traffic_bytes_per_launch"])
    # any change to a kernel source makes the figures stale
    with open(csrc / "matvec.hip", "a") as fh:
        fh.write("\n// edited\n")
    assert bench.counted(kernel) == {}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_equal_cost_speedup_uses_the_oracle_target_and_splits_the_ratio():
    rep64 = dict(cost=np.array([10.0, 5.0, 2.0, 1.0]), ms=np.array([4.0, 4.0, 4.0, 4.0]), final_cost=1.0,
                 pcg_iters=np.array([10, 20, 30, 40]), matvec_ms=300.0, matvec_launches=100)
    rep32 = dict(cost=np.array([9.0, 4.0, 1.9, 0.9]), ms=np.array([2.0, 2.0, 2.0, 2.0]), final_cost=0.9,
                 pcg_iters=np.array([10, 20, 5, 5]), matvec_ms=100.0, matvec_launches=50)
    sp = bench.equal_cost_speedup(rep32, rep64, oracle_final=1.95)
    # target 1.95 x (1 + 1e-4): FP64 after 4 iterations (16 ms, 100 matvecs), FP32-mixed after 3 (6 ms, 35)
    assert sp["target_from"] == "oracle" and sp["fp64_lm_iters"] == 4 and sp["fp32_mixed_lm_iters"] == 3
    assert sp["speedup"] == pytest.approx(16.0 / 6.0)
    assert sp["matvec_speed_ratio"] == pytest.approx(3.0 / 2.0)
    assert sp["fp64_matvecs"] == 100 and sp["fp32_mixed_matvecs"] == 35


def test_oracle_errors_and_roofline_fractions():
    golden = dict(iters_run=3, cost=[5.0, 4.0, 2.0],
                  params=dict(cameras=np.ones((4, 9)), point_index=np.array([1, 3]), points=np.ones((2, 3))))
    cams = np.ones((4, 9))
    cams[0, 0] = 1.0 + 6.0   # |delta| = 6 over |ref| = 6
    pts = np.ones((5, 3))
    e = bench.oracle_errors(dict(final_cost=2.002), (cams, pts), golden, 3)
    assert e["final_cost_rel_err"] == pytest.approx(1e-3)
    assert e["cameras_rel_err"] == pytest.approx(1.0) and e["points_rel_err"] == 0.0
    # per camera: camera 0 is off by 6/3 = 2 of its own norm, the others exact
    assert e["cameras_rel_err_max"] == pytest.approx(2.0) and e["cameras_rel_err_median"] == 0.0
    assert e["points_rel_err_max"] == 0.0
    assert bench.oracle_errors(dict(final_cost=4.0), None, golden, 2)["final_cost_rel_err"] == 0.0
    assert bench.oracle_errors(dict(final_cost=4.0), None, golden, 4) is None
    m, n, N = 13_700, 4_500_000, 29_000_000
    s = dict(hot_kernel_ms=0.5, matvec_ms=0.6)
    r = bench.roofline(s, m, n, N, False, dict(hot_kernel_ms=1.0, matvec_ms=1.2))
    alg = bench.hot_pass_algorithmic_bytes(n, N, 4)
    assert r["bound"] == "hbm" and r["achieved"] == pytest.approx(alg / 0.5e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["matvec_frac"] == pytest.approx(bench.matvec_algorithmic_bytes(m, n, N, 4) / 0.6e-3 / 8e12)
    assert r["alu_peak_tflops"] == pytest.approx(78.6432)
    assert r["fp64"]["frac"] == pytest.approx(bench.hot_pass_algorithmic_bytes(n, N, 8) / 1e-3 / 8e12)
