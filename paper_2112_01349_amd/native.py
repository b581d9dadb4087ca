"""ctypes binding of libba.so (include/ba.h): argument marshalling only.

Every step of the solve runs in the HIP library; this module converts numpy
arrays and torch tensors to pointers and the C structs to Python values.  It
raises if the library is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libba.so")

BA_OK, BA_EINVAL, BA_ENOMEM, BA_EDEVICE, BA_ENUMERIC = 0, 1, 2, 3, 4
FP64, FP32_MIXED = 0, 1
DAMP_MARQUARDT, DAMP_IDENTITY = 0, 1
SOLVER_PCG, SOLVER_DENSE = 0, 1
PRECOND_CAMERA_BLOCKS, PRECOND_SCHUR_JACOBI = 0, 1
# how each iteration's PCG solve ended (report["pcg_stop"])
PCG_CONVERGED, PCG_CAP, PCG_BREAKDOWN, PCG_FIXED, PCG_DIRECT = 0, 1, 2, 3, 4
PCG_STOP_NAMES = ("converged", "cap", "breakdown", "fixed", "direct")
DENSE_MAX_CAMERAS = 2048

EXPORTED = ("ba_options_default", "ba_create", "ba_set_params", "ba_get_params", "ba_eval_cost_grad",
            "ba_lm_solve", "ba_schur_matvec", "ba_cost_fwd_device", "ba_cost_bwd_device", "ba_cost_device_noalloc",
            "ba_memory_bytes", "ba_destroy", "ba_status_str", "ba_last_error")


class BAError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("precision", C.c_int32), ("damping", C.c_int32),
                ("huber_delta", C.c_double), ("max_lm_iters", C.c_int32), ("max_pcg_iters", C.c_int32),
                ("pcg_rtol", C.c_double), ("pcg_fixed_iters", C.c_int32), ("jacobian", C.c_int32),
                ("pcg_schedule", C.c_void_p), ("lambda_init", C.c_double),
                ("min_relative_decrease", C.c_double), ("time_kernels", C.c_int32),
                ("solver", C.c_int32), ("preconditioner", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("iters_run", C.c_int32), ("initial_cost", C.c_double),
                ("final_cost", C.c_double), ("cost", C.c_void_p), ("trial_cost", C.c_void_p),
                ("lambda_", C.c_void_p), ("pred", C.c_void_p), ("ms", C.c_void_p),
                ("pcg_iters", C.c_void_p), ("accepted", C.c_void_p), ("pcg_stop", C.c_void_p),
                ("total_ms", C.c_double),
                ("pcg_ms", C.c_double), ("pcg_iters_total", C.c_int64), ("matvec_ms", C.c_double),
                ("matvec_launches", C.c_int64), ("schur_hot_ms", C.c_double)]


_lib = None


def lib():
    """Loads libba.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2112_01349_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.ba_options_default.argtypes = [C.POINTER(Options)]
        L.ba_create.argtypes = [C.c_int32, C.c_int32, C.c_int64, vp, vp, vp, vp, vp, C.POINTER(Options), vp,
                                C.POINTER(vp)]
        L.ba_set_params.argtypes = [vp, vp, vp]
        L.ba_get_params.argtypes = [vp, vp, vp]
        L.ba_eval_cost_grad.argtypes = [vp, vp, vp, vp]
        L.ba_lm_solve.argtypes = [vp, C.POINTER(Options), C.POINTER(Report)]
        L.ba_schur_matvec.argtypes = [vp, C.c_double, C.c_int32, vp, vp]
        L.ba_cost_fwd_device.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
        L.ba_cost_bwd_device.argtypes = [vp, C.c_int32, vp, vp, C.c_double, vp, vp, vp, vp]
        L.ba_cost_device_noalloc.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.c_int32, vp, vp, vp, vp, vp,
                                             C.c_double, vp, vp]
        L.ba_memory_bytes.argtypes = [vp, C.POINTER(C.c_int64)]
        L.ba_destroy.argtypes = [vp]
        L.ba_destroy.restype = None
        L.ba_status_str.argtypes = [C.c_int]
        L.ba_status_str.restype = C.c_char_p
        L.ba_last_error.argtypes = [vp]
        L.ba_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("ba_destroy", "ba_status_str", "ba_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def status_name(status):
    try:
        return lib().ba_status_str(int(status)).decode()
    except Exception:  # noqa: BLE001 - naming only
        return f"status {status}"


def _ptr(a):
    return None if a is None else a.ctypes.data


def make_options(precision=FP64, damping=DAMP_MARQUARDT, huber_delta=0.0, max_lm_iters=10,
                 max_pcg_iters=50, pcg_rtol=1e-8, pcg_fixed_iters=0, pcg_schedule=None,
                 lambda_init=1e-4, min_relative_decrease=1e-3, time_kernels=False, jacobian=0,
                 solver=0, preconditioner=0):
    o = Options()
    lib().ba_options_default(C.byref(o))
    o.precision = int(precision)
    o.damping = int(damping)
    o.huber_delta = float(huber_delta)
    o.max_lm_iters = int(max_lm_iters)
    o.max_pcg_iters = int(max_pcg_iters)
    o.pcg_rtol = float(pcg_rtol)
    o.pcg_fixed_iters = int(pcg_fixed_iters)
    keep = None
    if pcg_schedule is not None:
        keep = np.ascontiguousarray(pcg_schedule, dtype=np.int32)
        if keep.shape[0] < o.max_lm_iters:
            raise ValueError("pcg_schedule shorter than max_lm_iters")
        o.pcg_schedule = keep.ctypes.data
    o.lambda_init = float(lambda_init)
    o.min_relative_decrease = float(min_relative_decrease)
    o.time_kernels = 1 if time_kernels else 0
    o.jacobian = int(jacobian)
    o.solver = int(solver)
    o.preconditioner = int(preconditioner)
    return o, keep


class Problem:
    """A bundle-adjustment problem held on the GPU (one libba handle)."""

    def __init__(self, cameras, points, obs_camera, obs_point, obs_uv, precision=FP64, stream=None,
                 **options):
        cams = np.ascontiguousarray(cameras, dtype=np.float64)
        pts = np.ascontiguousarray(points, dtype=np.float64)
        oc = np.ascontiguousarray(obs_camera, dtype=np.int32)
        op = np.ascontiguousarray(obs_point, dtype=np.int32)
        uv = np.ascontiguousarray(obs_uv, dtype=np.float64)
        if cams.ndim != 2 or cams.shape[1] != 9 or pts.ndim != 2 or pts.shape[1] != 3:
            raise ValueError("cameras must be [m,9] and points [n,3]")
        if oc.shape != op.shape or uv.shape != (oc.shape[0], 2):
            raise ValueError("observation arrays disagree in length")
        self.m, self.n, self.N = cams.shape[0], pts.shape[0], oc.shape[0]
        self.precision = int(precision)
        opt, self._sched = make_options(precision=precision, **options)
        self.options = dict(options)
        h = C.c_void_p()
        st = lib().ba_create(self.m, self.n, self.N, _ptr(cams), _ptr(pts), _ptr(oc), _ptr(op), _ptr(uv),
                             C.byref(opt), stream, C.byref(h))
        if st != BA_OK:
            raise BAError(st, lib().ba_last_error(None).decode())
        self._h = h

    # -------------------------------------------------------------- basics
    def _check(self, st):
        if st != BA_OK:
            raise BAError(st, lib().ba_last_error(self._h).decode())

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().ba_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def memory_bytes(self):
        b = C.c_int64()
        self._check(lib().ba_memory_bytes(self._h, C.byref(b)))
        return b.value

    def set_params(self, cameras=None, points=None):
        c = None if cameras is None else np.ascontiguousarray(cameras, dtype=np.float64)
        p = None if points is None else np.ascontiguousarray(points, dtype=np.float64)
        self._check(lib().ba_set_params(self._h, _ptr(c), _ptr(p)))

    def get_params(self):
        c = np.zeros((self.m, 9))
        p = np.zeros((self.n, 3))
        self._check(lib().ba_get_params(self._h, _ptr(c), _ptr(p)))
        return c, p

    def eval_cost_grad(self, grad=True):
        cost = np.zeros(1)
        gc = np.zeros((self.m, 9)) if grad else None
        gp = np.zeros((self.n, 3)) if grad else None
        self._check(lib().ba_eval_cost_grad(self._h, _ptr(cost), _ptr(gc), _ptr(gp)))
        return (float(cost[0]), gc, gp) if grad else float(cost[0])

    def cost(self):
        return self.eval_cost_grad(grad=False)

    # --------------------------------------------------------------- solve
    def lm_solve(self, **options):
        merged = dict(self.options)
        merged.update(options)
        opt, keep = make_options(precision=self.precision, **merged)
        K = max(opt.max_lm_iters, 1)
        arrs = dict(cost=np.zeros(K), trial_cost=np.zeros(K), lambda_=np.zeros(K), pred=np.zeros(K),
                    ms=np.zeros(K), pcg_iters=np.zeros(K, np.int32), accepted=np.zeros(K, np.int32),
                    pcg_stop=np.zeros(K, np.int32))
        rep = Report()
        rep.capacity = K
        for k, a in arrs.items():
            setattr(rep, k, a.ctypes.data)
        st = lib().ba_lm_solve(self._h, C.byref(opt), C.byref(rep))
        del keep
        n_it = rep.iters_run
        out = {k.rstrip("_"): arrs[k][:n_it].copy() for k in arrs}
        out.update(iters_run=n_it, initial_cost=rep.initial_cost, final_cost=rep.final_cost,
                   total_ms=rep.total_ms, pcg_ms=rep.pcg_ms, pcg_iters_total=rep.pcg_iters_total,
                   matvec_ms=rep.matvec_ms, matvec_launches=rep.matvec_launches,
                   schur_hot_ms=rep.schur_hot_ms, status=st,
                   error=lib().ba_last_error(self._h).decode() if st != BA_OK else "")
        if st not in (BA_OK, BA_ENUMERIC):
            self._check(st)
        return out

    def schur_matvec(self, x, lam, damping=DAMP_MARQUARDT):
        """q = (B~ - E C~^-1 E^T) x at the current state (caller camera order)."""
        xx = np.ascontiguousarray(x, dtype=np.float64).reshape(self.m, 9)
        q = np.zeros((self.m, 9))
        self._check(lib().ba_schur_matvec(self._h, float(lam), int(damping), _ptr(xx), _ptr(q)))
        return q

    # --------------------------------------------------- device-pointer forms
    def cost_fwd_device(self, dtype, cams_ptr, pts_ptr, cost_ptr, stream=None):
        self._check(lib().ba_cost_fwd_device(self._h, int(dtype), cams_ptr, pts_ptr, cost_ptr, stream))

    def cost_bwd_device(self, dtype, cams_ptr, pts_ptr, gout, gcam_ptr, gpt_ptr, stream=None, gout_ptr=None):
        self._check(lib().ba_cost_bwd_device(self._h, int(dtype), cams_ptr, pts_ptr, float(gout), gout_ptr,
                                             gcam_ptr, gpt_ptr, stream))


def cost_device_noalloc(m, n, N, dtype, cams_ptr, pts_ptr, oc_ptr, op_ptr, uv_ptr, huber_delta, cost_ptr,
                        stream=None):
    """ba_cost_device_noalloc: the robust cost from device arrays (pointers),
    with no handle and no allocation; raises BAError on a bad argument."""
    st = lib().ba_cost_device_noalloc(int(m), int(n), int(N), int(dtype), cams_ptr, pts_ptr, oc_ptr, op_ptr, uv_ptr,
                                      float(huber_delta), cost_ptr, stream)
    if st != BA_OK:
        raise BAError(st, "ba_cost_device_noalloc")
