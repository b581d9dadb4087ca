"""The C ABI library loads and exports every function include/ba.h declares;
argument validation runs on the host (no GPU needed for these calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def native():
    from paper_2112_01349_amd import native as nat
    if not os.path.exists(nat.LIB_PATH):
        from paper_2112_01349_amd import build
        build.build()
    return nat


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ba.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ba_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(native):
    names = declared_functions()
    assert len(names) >= 13
    L = C.CDLL(native.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(native.EXPORTED) == set(names)


def test_struct_sizes_match_header(native):
    # ba_options: 88 bytes, ba_report: 136 bytes on LP64 (natural alignment)
    assert C.sizeof(native.Options) == 88
    assert C.sizeof(native.Report) == 136
    o = native.Options()
    assert native.lib().ba_options_default(C.byref(o)) == 0
    assert o.struct_size == 88 and o.max_lm_iters == 10 and o.pcg_rtol == 1e-8 and o.lambda_init == 1e-4


def _create(native, cams, pts, oc, op, uv, opt=None):
    h = C.c_void_p()
    ptr = lambda a: a.ctypes.data  # noqa: E731
    st = native.lib().ba_create(len(cams), len(pts), len(oc), ptr(cams), ptr(pts), ptr(oc), ptr(op), ptr(uv),
                                opt, None, C.byref(h))
    return st, h


def test_invalid_inputs_are_rejected_on_the_host(native):
    cams = np.zeros((2, 9))
    cams[:, 5] = -10.0
    cams[:, 6] = 500.0
    pts = np.zeros((3, 3))
    oc = np.array([0, 1, 1], np.int32)
    op = np.array([0, 1, 2], np.int32)
    uv = np.zeros((3, 2))
    bad = oc.copy()
    bad[2] = 2
    st, h = _create(native, cams, pts, bad, op, uv)
    assert st == native.BA_EINVAL and not h.value
    assert b"out of range" in native.lib().ba_last_error(None)
    nan_uv = uv.copy()
    nan_uv[1, 0] = np.nan
    st, h = _create(native, cams, pts, oc, op, nan_uv)
    assert st == native.BA_EINVAL and b"non-finite" in native.lib().ba_last_error(None)
    neg = op.copy()
    neg[0] = -1
    st, h = _create(native, cams, pts, oc, neg, uv)
    assert st == native.BA_EINVAL
    o = native.Options()
    native.lib().ba_options_default(C.byref(o))
    o.struct_size = 12
    st, h = _create(native, cams, pts, oc, op, uv, C.byref(o))
    assert st == native.BA_EINVAL and b"struct_size" in native.lib().ba_last_error(None)
    native.lib().ba_options_default(C.byref(o))
    o.precision = 7
    st, h = _create(native, cams, pts, oc, op, uv, C.byref(o))
    assert st == native.BA_EINVAL
    native.lib().ba_options_default(C.byref(o))
    assert o.jacobian == 0
    o.jacobian = 2
    st, h = _create(native, cams, pts, oc, op, uv, C.byref(o))
    assert st == native.BA_EINVAL and b"jacobian" in native.lib().ba_last_error(None)
    native.lib().ba_options_default(C.byref(o))
    assert o.solver == native.SOLVER_PCG
    o.solver = 2
    st, h = _create(native, cams, pts, oc, op, uv, C.byref(o))
    assert st == native.BA_EINVAL and b"solver" in native.lib().ba_last_error(None)
    # the dense reduced system is limited to BA_DENSE_MAX_CAMERAS cameras
    o.solver = native.SOLVER_DENSE
    many = np.tile(cams[:1], (native.DENSE_MAX_CAMERAS + 1, 1))
    st, h = _create(native, many, pts, oc, op, uv, C.byref(o))
    assert st == native.BA_EINVAL and b"at most 2048 cameras" in native.lib().ba_last_error(None)
    native.lib().ba_options_default(C.byref(o))
    assert o.preconditioner == native.PRECOND_CAMERA_BLOCKS
    o.preconditioner = 2
    st, h = _create(native, cams, pts, oc, op, uv, C.byref(o))
    assert st == native.BA_EINVAL and b"preconditioner" in native.lib().ba_last_error(None)
    assert native.lib().ba_status_str(4) == b"BA_ENUMERIC"


def test_oracle_and_solver_share_no_code():
    """The oracle sources neither include nor name the solver's sources and
    the solver sources never reference the oracle."""
    csrc = os.path.join(ROOT, "paper_2112_01349_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "oracle" not in text.lower(), f
    for f in ("ba_oracle.c", "ba_oracle.h"):
        text = open(os.path.join(ROOT, "oracle", f)).read()
        assert "camera_model.h" not in text and "ba_internal" not in text and "ba.h\"" not in text
    for f in os.listdir(os.path.join(ROOT, "paper_2112_01349_amd")):
        if f.endswith(".py"):
            text = open(os.path.join(ROOT, "paper_2112_01349_amd", f)).read()
            assert "import oracle" not in text and "from oracle" not in text, f
