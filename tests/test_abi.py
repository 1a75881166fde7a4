"""The C ABI library loads and exports every symbol include/hom.h declares; argument
validation answers without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hom.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hom_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    import paper_2111_14317_amd as hom
    names = _declared()
    assert set(names) == set(hom.EXPORTED), names
    lib = ctypes.CDLL(hom.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_invalid_arguments_rejected_without_gpu():
    import paper_2111_14317_amd as hom
    lib = hom.lib
    out = ctypes.c_void_p()
    m = np.array([2, 2], np.int32)
    A = np.zeros((4, 2), np.int8)
    w = np.zeros(4)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.hom_create(0, P(m), P(A), P(w), 0, ctypes.byref(out)) == hom.HOM_EINVAL
    assert lib.hom_create(33, P(m), P(A), P(w), 0, ctypes.byref(out)) == hom.HOM_EINVAL
    assert b"n must be" in lib.hom_last_error()
    bad_m = np.array([2, 0], np.int32)
    assert lib.hom_create(2, P(bad_m), P(A), P(w), 0, ctypes.byref(out)) == hom.HOM_EINVAL
    bad_w = np.array([0.0, -1.0, 0.0, 0.0])
    assert lib.hom_create(2, P(m), P(A), P(bad_w), 0, ctypes.byref(out)) == hom.HOM_EINVAL
    bad_A = A.copy(); bad_A[0, 0] = -128
    assert lib.hom_create(2, P(m), P(bad_A), P(w), 0, ctypes.byref(out)) == hom.HOM_EINVAL
    assert lib.hom_create(2, P(m), P(A), P(w), 8, ctypes.byref(out)) == hom.HOM_EINVAL
    # projective handles: n <= 29 and homogenising exponents <= 127 (checked before the GPU)
    m30 = np.full(30, 1, np.int32)
    A30 = np.zeros((30, 30), np.int8)
    assert lib.hom_create(30, P(m30), P(A30), P(np.zeros(30)), hom.CREATE_PROJECTIVE,
                          ctypes.byref(out)) == hom.HOM_EINVAL
    big = np.array([[100, 100], [-100, -100], [0, 0], [1, 0]], np.int8)  # d = 200: 400 > 127
    assert lib.hom_create(2, P(m), P(big), P(w), hom.CREATE_PROJECTIVE,
                          ctypes.byref(out)) == hom.HOM_EINVAL
    assert b"homogenising exponent" in lib.hom_last_error()
    assert lib.hom_create(2, None, P(A), P(w), 0, ctypes.byref(out)) == hom.HOM_EINVAL
    assert lib.hom_eval(None, None, 0, None, None, None, None, 0, None) == hom.HOM_EINVAL
    assert lib.hom_step(None, None, 0, None, None, None, None, None, 0, None) == hom.HOM_EINVAL
    assert lib.hom_step_proj(None, None, 0, None, None, None, None, None, None) == hom.HOM_EINVAL
    assert lib.hom_destroy(None) == hom.HOM_OK
    p = hom.TrackParams()
    assert lib.hom_track_params_default(ctypes.byref(p), 7) == hom.HOM_EINVAL
    assert lib.hom_track_params_default(ctypes.byref(p), hom.MIXED) == hom.HOM_OK
    assert p.tol_track == 1e-5 and p.res_tol == 1e-10


def test_default_params_match_oracle_defaults():
    """Both sides run the same tracker rules with the same constants."""
    import oracle
    import paper_2111_14317_amd as hom
    p = hom.default_params(hom.FP64)
    o = oracle.TrackParams()
    for f in ("ds0", "ds_max", "ds_min", "tol_polish", "tol_track", "tol_end", "res_tol", "div_re",
              "sing_ratio", "tol_predict", "predictor", "max_polish", "max_newton", "max_end",
              "max_steps",
              "max_iters"):
        assert getattr(p, f) == getattr(o, f), f


def test_binomial_starts_argument_errors_without_gpu():
    """hom_binomial_starts refuses bad arguments before it touches the GPU."""
    import paper_2111_14317_amd as hom
    lib = hom.lib
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
    D = np.array([[[2, 0], [0, 3]]], np.int32)
    beta = np.ones((1, 2), np.complex128)
    num = np.zeros(1, np.int64)
    E = hom.HOM_EINVAL
    assert lib.hom_binomial_starts(0, 1, P(D), P(beta), None, None, P(num), None, 0, None) == E
    assert lib.hom_binomial_starts(33, 1, P(D), P(beta), None, None, P(num), None, 0, None) == E
    assert lib.hom_binomial_starts(2, 0, P(D), P(beta), None, None, P(num), None, 0, None) == E
    assert lib.hom_binomial_starts(2, 1, None, P(beta), None, None, P(num), None, 0, None) == E
    assert lib.hom_binomial_starts(2, 1, P(D), P(beta), None, None, None, None, 0, None) == E
    f = np.array([0], np.int64)
    assert lib.hom_binomial_starts(2, 1, P(D), P(beta), P(f), None, P(num), None, 0, None) == E
    assert b"first and count" in lib.hom_last_error()
