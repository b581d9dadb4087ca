"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this module.  The solver package never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ba_oracle.c")
LIB = os.path.join(HERE, "libba_oracle.so")

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)   # a process that has the old library loaded keeps it
    return LIB


class Options(C.Structure):
    _fields_ = [("huber_delta", C.c_double), ("damping", C.c_int32),
                ("max_lm_iters", C.c_int32), ("max_pcg_iters", C.c_int32),
                ("pcg_rtol", C.c_double), ("pcg_schedule", C.c_void_p),
                ("lambda_init", C.c_double), ("min_relative_decrease", C.c_double),
                ("preconditioner", C.c_int32), ("solver", C.c_int32)]


class Trace(C.Structure):
    _fields_ = [("iters_run", C.c_int32), ("initial_cost", C.c_double),
                ("final_cost", C.c_double), ("cost", C.c_void_p), ("trial_cost", C.c_void_p),
                ("lambda_", C.c_void_p), ("pred", C.c_void_p), ("pcg_iters", C.c_void_p),
                ("accepted", C.c_void_p), ("pcg_stop", C.c_void_p)]


# how each PCG solve ended (trace["pcg_stop"])
PCG_CONVERGED, PCG_CAP, PCG_BREAKDOWN, PCG_FIXED, PCG_DIRECT = 0, 1, 2, 3, 4


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        L.orc_project.argtypes = [_f64p, _f64p, _f64p]
        L.orc_residual_jacobian.argtypes = [_f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.orc_rho.argtypes = [C.c_double, C.c_double]
        L.orc_rho.restype = C.c_double
        L.orc_rho_prime.argtypes = [C.c_double, C.c_double]
        L.orc_rho_prime.restype = C.c_double
        L.orc_cost.argtypes = [C.c_int64, _f64p, _f64p, _i32p, _i32p, _f64p, C.c_double]
        L.orc_cost.restype = C.c_double
        L.orc_cost_subset.argtypes = [_i64p, C.c_int64, _f64p, _f64p, _i32p, _i32p, _f64p,
                                      C.c_double]
        L.orc_cost_subset.restype = C.c_double
        L.orc_gradient.argtypes = [C.c_int32, C.c_int32, C.c_int64, _f64p, _f64p, _i32p, _i32p,
                                   _f64p, C.c_double, _f64p, _f64p]
        L.orc_gradient.restype = C.c_double
        L.orc_assemble.argtypes = [C.c_int32, C.c_int32, C.c_int64, _f64p, _f64p, _i32p, _i32p,
                                   _f64p, C.c_double, _f64p, _f64p, _f64p, _f64p, _f64p,
                                   C.POINTER(C.c_double)]
        L.orc_subset_sums.argtypes = [_i64p, C.c_int64, _f64p, _f64p, _i32p, _i32p, _f64p,
                                      C.c_double, _f64p, _f64p, _f64p, _f64p,
                                      C.POINTER(C.c_double)]
        L.orc_damp.argtypes = [C.c_int32, C.c_int32, _f64p, _f64p, C.c_double, C.c_int32,
                               _f64p, _f64p, _f64p, _f64p]
        L.orc_invert_points.argtypes = [C.c_int32, _f64p, _f64p]
        L.orc_schur_matvec.argtypes = [C.c_int32, C.c_int32, C.c_int64, _i32p, _i32p, _f64p,
                                       _f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.orc_reduced_rhs.argtypes = [C.c_int32, C.c_int32, C.c_int64, _i32p, _i32p, _f64p,
                                      _f64p, _f64p, _f64p, _f64p, _f64p]
        L.orc_pcg.argtypes = [C.c_int32, C.c_int32, C.c_int64, _i32p, _i32p, _f64p, _f64p,
                              _f64p, _f64p, C.c_double, C.c_int32, C.c_int32, _f64p,
                              C.POINTER(C.c_int32)]
        L.orc_pcg_m.argtypes = [C.c_int32, C.c_int32, C.c_int64, _i32p, _i32p, _f64p, _f64p,
                                _f64p, _f64p, _f64p, C.c_double, C.c_int32, C.c_int32, _f64p,
                                C.POINTER(C.c_int32)]
        L.orc_schur_jacobi.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p,
                                       _f64p]
        L.orc_back_substitute.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _f64p, _f64p,
                                          _f64p, _f64p, _f64p]
        L.orc_lm_solve.argtypes = [C.c_int32, C.c_int32, C.c_int64, _f64p, _f64p, _i32p, _i32p,
                                   _f64p, C.POINTER(Options), C.POINTER(Trace)]
        L.orc_schur_row.argtypes = [C.c_int32, _f64p, _f64p, _i32p, _i32p, _f64p, C.c_double,
                                    C.c_double, C.c_int32, _i64p, _i64p, _i64p, _i64p, _f64p,
                                    _f64p]
        L.orc_schur_row.restype = C.c_double
        L.orc_schur_dense.argtypes = [C.c_int32, C.c_int32, C.c_int64, _i32p, _i32p, _f64p, _f64p,
                                      _f64p, _f64p]
        L.orc_dense_solve.argtypes = [C.c_int64, _f64p, _f64p, _f64p]
        _lib = L
    return _lib


def _f(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def project(cam, X):
    out = np.zeros(2)
    lib().orc_project(_f(cam), _f(X), out)
    return out


def residual_jacobian(cam, X, uv):
    e, Jc, Jp = np.zeros(2), np.zeros(18), np.zeros(6)
    lib().orc_residual_jacobian(_f(cam), _f(X), _f(uv), e, Jc, Jp)
    return e, Jc.reshape(2, 9), Jp.reshape(2, 3)


def rho(s, delta):
    return lib().orc_rho(float(s), float(delta))


def rho_prime(s, delta):
    return lib().orc_rho_prime(float(s), float(delta))


def cost(cams, pts, oc, op, uv, delta=0.0):
    return lib().orc_cost(len(oc), _f(cams), _f(pts), _i(oc), _i(op), _f(uv), float(delta))


def cost_subset(obs_list, cams, pts, oc, op, uv, delta=0.0):
    lst = np.ascontiguousarray(obs_list, dtype=np.int64)
    return lib().orc_cost_subset(lst, len(lst), _f(cams), _f(pts), _i(oc), _i(op), _f(uv),
                                 float(delta))


def gradient(cams, pts, oc, op, uv, delta=0.0):
    m, n = len(cams), len(pts)
    gc, gp = np.zeros((m, 9)), np.zeros((n, 3))
    F = lib().orc_gradient(m, n, len(oc), _f(cams), _f(pts), _i(oc), _i(op), _f(uv),
                           float(delta), gc, gp)
    return F, gc, gp


def assemble(cams, pts, oc, op, uv, delta=0.0):
    m, n, N = len(cams), len(pts), len(oc)
    B, Cm = np.zeros((m, 9, 9)), np.zeros((n, 3, 3))
    E, v, w = np.zeros((N, 9, 3)), np.zeros((m, 9)), np.zeros((n, 3))
    F = C.c_double(0.0)
    lib().orc_assemble(m, n, N, _f(cams), _f(pts), _i(oc), _i(op), _f(uv), float(delta),
                       B, Cm, E, v, w, C.byref(F))
    return dict(B=B, C=Cm, E=E, v=v, w=w, cost=F.value)


def subset_sums(obs_list, cams, pts, oc, op, uv, delta=0.0):
    lst = np.ascontiguousarray(obs_list, dtype=np.int64)
    Bs, vs, Cs, ws = np.zeros((9, 9)), np.zeros(9), np.zeros((3, 3)), np.zeros(3)
    F = C.c_double(0.0)
    lib().orc_subset_sums(lst, len(lst), _f(cams), _f(pts), _i(oc), _i(op), _f(uv),
                          float(delta), Bs, vs, Cs, ws, C.byref(F))
    return dict(B=Bs, v=vs, C=Cs, w=ws, cost=F.value)


def damp(B, Cm, lam, damping=0):
    m, n = len(B), len(Cm)
    Bd, Cd, Dc, Dp = np.zeros_like(B), np.zeros_like(Cm), np.zeros((m, 9)), np.zeros((n, 3))
    lib().orc_damp(m, n, _f(B), _f(Cm), float(lam), int(damping), Bd, Cd, Dc, Dp)
    return Bd, Cd, Dc, Dp


def invert_points(Cd):
    Ci = np.zeros_like(Cd)
    rc = lib().orc_invert_points(len(Cd), _f(Cd), Ci)
    if rc:
        raise FloatingPointError("point block not positive definite")
    return Ci


def schur_matvec(oc, op, Bd, E, Ci, x):
    m, n, N = len(Bd), len(Ci), len(oc)
    out = np.zeros((m, 9))
    lib().orc_schur_matvec(m, n, N, _i(oc), _i(op), _f(Bd), _f(E), _f(Ci), _f(x), out,
                           np.zeros(3 * max(n, 1)), np.zeros(3 * max(n, 1)))
    return out


def reduced_rhs(oc, op, v, w, E, Ci):
    m, n, N = len(v), len(w), len(oc)
    g = np.zeros((m, 9))
    lib().orc_reduced_rhs(m, n, N, _i(oc), _i(op), _f(v), _f(w), _f(E), _f(Ci), g,
                          np.zeros(3 * max(n, 1)))
    return g


def pcg(oc, op, Bd, E, Ci, b, rtol=1e-8, max_iters=50, fixed_iters=0, M=None):
    """Alg. 2; M: preconditioner blocks [m][9][9] (default: the damped camera blocks Bd)."""
    m, n, N = len(Bd), len(Ci), len(oc)
    x = np.zeros((m, 9))
    it = C.c_int32(0)
    rc = lib().orc_pcg_m(m, n, N, _i(oc), _i(op), _f(Bd), _f(E), _f(Ci), _f(Bd if M is None else M), _f(b),
                         float(rtol), int(max_iters), int(fixed_iters), x, C.byref(it))
    return x, it.value, rc


def schur_jacobi(oc, op, Bd, E, Ci):
    """Schur-Jacobi preconditioner blocks M_j = B~_j - sum_k E_k C~^-1 E_k^T."""
    m = len(Bd)
    M = np.zeros((m, 9, 9))
    lib().orc_schur_jacobi(m, len(oc), _i(oc), _i(op), _f(Bd), _f(E), _f(Ci), M)
    return M


def back_substitute(oc, op, E, Ci, w, dc):
    n, N = len(w), len(oc)
    dp = np.zeros((n, 3))
    lib().orc_back_substitute(n, N, _i(oc), _i(op), _f(E), _f(Ci), _f(w), _f(dc), dp)
    return dp


def schur_dense(oc, op, Bd, E, Ci):
    """The reduced camera system written out: dense [9m][9m] S."""
    m, n, N = len(Bd), len(Ci), len(oc)
    S = np.zeros((9 * m, 9 * m))
    rc = lib().orc_schur_dense(m, n, N, _i(oc), _i(op), _f(Bd), _f(E), _f(Ci), S)
    if rc:
        raise MemoryError("orc_schur_dense")
    return S


def dense_solve(A, b):
    """A^-1 b through the Cholesky factor of a dense SPD A."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    x = np.zeros(len(A))
    rc = lib().orc_dense_solve(len(A), A, _f(b), x)
    if rc:
        raise FloatingPointError("matrix not positive definite")
    return x


def lm_solve(cams, pts, oc, op, uv, huber_delta=0.0, damping=0, max_lm_iters=10,
             max_pcg_iters=50, pcg_rtol=1e-8, pcg_schedule=None, lambda_init=1e-4,
             min_relative_decrease=1e-3, preconditioner=0, solver=0):
    """Runs the LM loop; returns (cams, pts, trace dict, status).  preconditioner:
    0 = the damped camera blocks (Alg. 2), 1 = Schur-Jacobi blocks; solver: 0 =
    PCG, 1 = the reduced camera system written out and factored."""
    cams = np.array(cams, dtype=np.float64, order="C", copy=True)
    pts = np.array(pts, dtype=np.float64, order="C", copy=True)
    K = int(max_lm_iters)
    sched = None
    if pcg_schedule is not None:
        sched = np.ascontiguousarray(pcg_schedule, dtype=np.int32)
        assert len(sched) >= K
    opt = Options(float(huber_delta), int(damping), K, int(max_pcg_iters), float(pcg_rtol),
                  sched.ctypes.data if sched is not None else None, float(lambda_init),
                  float(min_relative_decrease), int(preconditioner), int(solver))
    arrs = dict(cost=np.zeros(K), trial_cost=np.zeros(K), lambda_=np.zeros(K), pred=np.zeros(K),
                pcg_iters=np.zeros(K, np.int32), accepted=np.zeros(K, np.int32),
                pcg_stop=np.zeros(K, np.int32))
    tr = Trace(0, 0.0, 0.0, *(arrs[k].ctypes.data for k in
                              ("cost", "trial_cost", "lambda_", "pred", "pcg_iters", "accepted", "pcg_stop")))
    rc = lib().orc_lm_solve(len(cams), len(pts), len(oc), cams, pts, _i(oc), _i(op), _f(uv),
                            C.byref(opt), C.byref(tr))
    n_it = tr.iters_run
    trace = {k.rstrip("_"): arrs[k][:n_it].copy() for k in arrs}
    trace.update(iters_run=n_it, initial_cost=tr.initial_cost, final_cost=tr.final_cost)
    return cams, pts, trace, rc


def csr(index, count):
    """Observation lists grouped by index (e.g. camera or point): offsets and
    a stable ordering (library sort)."""
    order = np.argsort(index, kind="stable").astype(np.int64)
    off = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(np.bincount(index, minlength=count), out=off[1:])
    return off, order


def schur_rows(cams_idx, cams, pts, oc, op, uv, x, lam, delta=0.0, damping=0,
               cam_csr=None, pt_csr=None):
    m, n = len(cams), len(pts)
    cam_off, cam_obs = cam_csr if cam_csr is not None else csr(oc, m)
    pt_off, pt_obs = pt_csr if pt_csr is not None else csr(op, n)
    out = np.zeros((len(cams_idx), 9))
    q = np.zeros(9)
    for t, j in enumerate(cams_idx):
        rc = lib().orc_schur_row(int(j), _f(cams), _f(pts), _i(oc), _i(op), _f(uv), float(delta),
                                 float(lam), int(damping), cam_off, cam_obs, pt_off, pt_obs,
                                 _f(x), q)
        if rc != 0.0:
            raise FloatingPointError("point block not positive definite")
        out[t] = q
    return out
