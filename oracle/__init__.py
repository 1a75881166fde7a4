"""Plain FP64 CPU oracle for the polyhedral-homotopy hot path (arXiv 2111.14317).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's
CPU-baseline leg; never by the library.  The arithmetic lives in `hom_oracle.c` (plain C99,
double complex): monomials by repeated multiplication, explicit derivatives (Sec. 5.1), one
partially pivoted LU for the Euler and Newton directions (Sec. 2.3, Sec. 6), a predictor-corrector
tracker whose constants come from `TrackParams`, and the implicit-function-theorem gradient.

Parity status of each function (what pins it is in tests/test_oracle_*.py):
  eval            pinned: central finite differences, 50-digit mpmath, exact values at x = +-1,
                  branch invariance, J_x = J_z diag(e^{-z}), zeros at binomial roots
  step            pinned: LAPACK solve, Cramer's rule, closed-form directions of binomial systems
  track           pinned: closed-form binomial paths, mixed-volume root count, residuals; the
                  Hermite predictor against scipy's CubicHermiteSpline and exactness on cubics;
                  the Runge-Kutta predictor's fourth order on a closed-form trinomial path
  endpoint_grad   pinned: central finite differences of re-solved endpoints
  step_proj       pinned: homogeneity of degree one under y -> lambda y, the affine directions
                  mapped into homogeneous coordinates (from the affine evaluation and numpy
                  solves, through Euler's identity), exact rational Cramer solutions
  residual        pinned: hand-worked exact values (tests/golden/residual_2x2.json), exact
                  rational arithmetic at rational points, the closed form at perturbed binomial
                  roots, zeros at roots, coefficient-scale and branch invariance
  binomial_roots  (oracle/binomial.py, Python) pinned: every root's residual from the
                  definition, |det D| pairwise distinct roots, closed forms for n = 1 and diagonal
                  D, equation-order invariance, the input generator's Smith-form roots
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hom_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

# path status codes (same meaning as the library's)
OK, START, RUNNING = 0, 1, 2
SINGULAR, STEP_MIN, DIVERGED, NONFINITE, POLISH_FAIL, ENDGAME_FAIL, MAX_ITERS = -1, -2, -3, -4, -5, -6, -7


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over independent points)."""
    if force or not os.path.exists(_LIB_PATH):
        os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        _lib.oracle_eval.argtypes = [i32, P, P, P, P, i64, P, P, i32, P, P, P, i32]
        _lib.oracle_step.argtypes = [i32, P, P, P, P, i64, P, P, P, P, P, P, i32]
        _lib.oracle_track.argtypes = [i32, P, P, P, P, i64, P, P, P, P, P, P, P, i32]
        _lib.oracle_residual.argtypes = [i32, P, P, P, i64, P, P, i32]
        _lib.oracle_endpoint_grad.argtypes = [i32, P, P, P, P, i64, P, P, P]
        _lib.oracle_step_proj.argtypes = [i32, P, P, P, P, i64, P, P, P, P, P, P, P, i32]
        _lib.oracle_hermite.argtypes = [i32, i64, P, P, P, P, P, P, P, P]
        _lib.oracle_hermite.restype = i32
        _lib.oracle_rk4_predict.argtypes = [i32, P, P, P, P, i64, P, P, P, P]
        _lib.oracle_rk4_predict.restype = i32
        for name in ("oracle_eval", "oracle_step", "oracle_track", "oracle_residual",
                     "oracle_endpoint_grad", "oracle_step_proj"):
            getattr(_lib, name).restype = i32
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


NMAX = 32  # the C oracle keeps per-point arrays on the stack


def _checked(code):
    if code < 0:
        raise ValueError("oracle: n must be in [1, 32]")
    return code


def _sys_arrays(sys):
    if not 1 <= sys.n <= NMAX:
        raise ValueError(f"oracle: n = {sys.n} outside [1, {NMAX}]")
    return (np.ascontiguousarray(sys.m, np.int32), np.ascontiguousarray(sys.A, np.int8),
            np.ascontiguousarray(sys.w, np.float64))


def default_threads() -> int:
    return os.cpu_count() or 1


def eval(sys, c, z, s, scaled=True, threads=None, with_den=False):
    """G [P][n][n+2] = [J_z | H_s | H] (rows scaled by e^{-logscale} when `scaled`), logscale
    [P][n], and optionally den[P][n][n+2] = sum_a |term_a| |C_{a,col}| (the componentwise scale
    used by the parity metric)."""
    lib = _load()
    m, A, w = _sys_arrays(sys)
    c = np.ascontiguousarray(c, np.complex128)
    z = np.ascontiguousarray(z, np.complex128).reshape(-1, sys.n)
    s = np.ascontiguousarray(s, np.float64).reshape(-1)
    P, n = z.shape[0], sys.n
    G = np.zeros((P, n, n + 2), np.complex128)
    L = np.zeros((P, n), np.float64)
    den = np.zeros((P, n, n + 2), np.float64) if with_den else None
    _checked(lib.oracle_eval(n, _ptr(m), _ptr(A), _ptr(w), _ptr(c), P, _ptr(z), _ptr(s),
                             int(scaled), _ptr(G), _ptr(L), _ptr(den), threads or default_threads()))
    return (G, L, den) if with_den else (G, L)


def step(sys, c, z, s, threads=None):
    """Euler and Newton directions dE = -J_z^{-1} H_s, dN = -J_z^{-1} H at every point, status
    (0, or -1 when a pivot is exactly zero) and the pivot ratio min|u_jj| / max|u_jj|."""
    lib = _load()
    m, A, w = _sys_arrays(sys)
    c = np.ascontiguousarray(c, np.complex128)
    z = np.ascontiguousarray(z, np.complex128).reshape(-1, sys.n)
    s = np.ascontiguousarray(s, np.float64).reshape(-1)
    P, n = z.shape[0], sys.n
    dE = np.zeros((P, n), np.complex128)
    dN = np.zeros((P, n), np.complex128)
    st = np.zeros(P, np.int32)
    ratio = np.zeros(P, np.float64)
    _checked(lib.oracle_step(n, _ptr(m), _ptr(A), _ptr(w), _ptr(c), P, _ptr(z), _ptr(s), _ptr(dE),
                             _ptr(dN), _ptr(st), _ptr(ratio), threads or default_threads()))
    return dE, dN, st, ratio


def hermite(s0, z0, e0, s1, z1, e1, s):
    """The tracker's cubic Hermite predictor: the cubic through (s0, z0), (s1, z1) with slopes
    e0, e1, at s.  Arrays [P][n] (complex) and [P] (s values)."""
    lib = _load()
    z0 = np.ascontiguousarray(z0, np.complex128)
    P, n = z0.shape
    args = [np.ascontiguousarray(np.broadcast_to(v, (P,)), np.float64) for v in (s0, s1, s)]
    e0, z1, e1 = (np.ascontiguousarray(v, np.complex128) for v in (e0, z1, e1))
    out = np.zeros((P, n), np.complex128)
    _checked(lib.oracle_hermite(n, P, _ptr(args[0]), _ptr(z0), _ptr(e0), _ptr(args[1]), _ptr(z1),
                                _ptr(e1), _ptr(args[2]), _ptr(out)))
    return out


def rk4_predict(sys, c, za, sa, h):
    """The tracker's Runge-Kutta predictor from points za [P][n] at sa [P] with steps h [P]
    (the classical fourth-order scheme on dz/ds = dE(z, s)); NaN rows where a stage point is
    singular."""
    lib = _load()
    m, A, w = _sys_arrays(sys)
    za = np.ascontiguousarray(za, np.complex128)
    P = za.shape[0]
    sa = np.ascontiguousarray(np.broadcast_to(np.asarray(sa, np.float64), (P,)))
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, np.float64), (P,)))
    c = np.ascontiguousarray(c, np.complex128)
    out = np.zeros_like(za)
    _checked(lib.oracle_rk4_predict(sys.n, _ptr(m), _ptr(A), _ptr(w), _ptr(c), P, _ptr(za),
                                    _ptr(sa), _ptr(h), _ptr(out)))
    return out


def step_proj(sys, c, y, s, threads=None):
    """Euler and Newton directions in homogeneous coordinates (Sec. 2.2, eq. (3)-(5)) at points
    y [P][n+1] (y_j pairs with x_j for j < n; y_n is the homogenising coordinate, so an affine
    point x is y = (x, 1)): [dH~/dy; y^*] dE = [-dH~/ds; 0] and [dH~/dy; y^*] dN = [-H~; 0].
    Returns (dE, dN, status, ratio, d) with d [n] the homogenising degrees."""
    lib = _load()
    m, A, w = _sys_arrays(sys)
    c = np.ascontiguousarray(c, np.complex128)
    y = np.ascontiguousarray(y, np.complex128).reshape(-1, sys.n + 1)
    s = np.ascontiguousarray(np.broadcast_to(np.asarray(s, np.float64), (y.shape[0],)))
    P, nu = y.shape
    dE = np.zeros((P, nu), np.complex128)
    dN = np.zeros((P, nu), np.complex128)
    st = np.zeros(P, np.int32)
    ratio = np.zeros(P, np.float64)
    d = np.zeros(sys.n, np.int32)
    code = lib.oracle_step_proj(sys.n, _ptr(m), _ptr(A), _ptr(w), _ptr(c), P, _ptr(y), _ptr(s),
                                _ptr(dE), _ptr(dN), _ptr(st), _ptr(ratio), _ptr(d),
                                threads or default_threads())
    if code == -2:
        raise ValueError("oracle: a homogenising exponent exceeds 127")
    _checked(code)
    return dE, dN, st, ratio, d


@dataclasses.dataclass
class TrackParams:
    """Tracker constants (the paper fixes none; these are this implementation's choices)."""

    ds0: float = 0.05
    ds_max: float = 0.5
    ds_min: float = 1e-10
    tol_polish: float = 1e-12
    tol_track: float = 1e-8
    tol_end: float = 1e-14
    res_tol: float = 1e-10
    div_re: float = 40.0
    sing_ratio: float = 1e-14
    tol_predict: float = 1e-2
    max_polish: int = 10
    max_newton: int = 3
    max_end: int = 8
    max_steps: int = 100000
    max_iters: int = 100000
    predictor: int = 0  # 0 Euler, 1 cubic Hermite through the last two accepted points,
    #                     2 classical Runge-Kutta (three more evaluations per step)

    def arrays(self):
        d = np.array([self.ds0, self.ds_max, self.ds_min, self.tol_polish, self.tol_track,
                      self.tol_end, self.res_tol, self.div_re, self.sing_ratio,
                      self.tol_predict], np.float64)
        i = np.array([self.max_polish, self.max_newton, self.max_end, self.max_steps,
                      self.max_iters, self.predictor], np.int32)
        return d, i


def track(sys, c, z0, s0, params: TrackParams | None = None, status=None, ds=None, threads=None):
    """Track every path from (z0, s0) to s = 0.  Returns (z, s, ds, status, counters[P][4] =
    accepted steps, rejected steps, corrector iterations, eval+solves)."""
    lib = _load()
    params = params or TrackParams()
    m, A, w = _sys_arrays(sys)
    c = np.ascontiguousarray(c, np.complex128)
    z = np.array(z0, np.complex128).reshape(-1, sys.n)
    P = z.shape[0]
    s = np.array(np.broadcast_to(np.asarray(s0, np.float64), (P,)))
    ds = np.zeros(P, np.float64) if ds is None else np.array(ds, np.float64)
    st = np.full(P, START, np.int32) if status is None else np.array(status, np.int32)
    cnt = np.zeros((P, 4), np.int32)
    d, i = params.arrays()
    _checked(lib.oracle_track(sys.n, _ptr(m), _ptr(A), _ptr(w), _ptr(c), P, _ptr(z), _ptr(s),
                              _ptr(ds), _ptr(d), _ptr(i), _ptr(st), _ptr(cnt),
                              threads or default_threads()))
    return z, s, ds, st, cnt


def residual(sys, c, z, threads=None):
    """Relative backward error r(x) = max_k |f_k(x)| / sum_a |c_{k,a} x^a| at t = 1."""
    lib = _load()
    m, A, _ = _sys_arrays(sys)
    c = np.ascontiguousarray(c, np.complex128)
    z = np.ascontiguousarray(z, np.complex128).reshape(-1, sys.n)
    out = np.zeros(z.shape[0], np.float64)
    _checked(lib.oracle_residual(sys.n, _ptr(m), _ptr(A), _ptr(c), z.shape[0], _ptr(z),
                                 _ptr(out), threads or default_threads()))
    return out


def endpoint_grad(sys, c, z_end, grad_x):
    """grad_c [M] (PyTorch convention dL/dRe c + i dL/dIm c) of a loss on the endpoints x = e^z,
    given grad_x = dL/dRe x + i dL/dIm x.  Returns (grad_c, number of singular paths skipped)."""
    lib = _load()
    m, A, w = _sys_arrays(sys)
    c = np.ascontiguousarray(c, np.complex128)
    z = np.ascontiguousarray(z_end, np.complex128).reshape(-1, sys.n)
    g = np.ascontiguousarray(grad_x, np.complex128).reshape(-1, sys.n)
    out = np.zeros(sys.M, np.complex128)
    ns = _checked(lib.oracle_endpoint_grad(sys.n, _ptr(m), _ptr(A), _ptr(w), _ptr(c), z.shape[0],
                                           _ptr(z), _ptr(g), _ptr(out)))
    return out, int(ns)


from .binomial import binomial_roots  # noqa: E402  (plain Python; no C)
