"""Independent references used to pin the oracle (test helpers, no library code).

  * mp_eval       - 50-digit mpmath evaluation of [J_z | H_s | H] straight from eq. (1)-(2);
  * exact_eval    - exact rational evaluation at rational points x, t (fractions.Fraction);
  * np_newton     - a numpy Newton solver for F(x) = H(x, 1) in affine x coordinates, used to
                    re-solve perturbed systems for finite-difference gradients;
  * mixed_volume  - Bernshtein's count as the alternating sum of Minkowski-sum volumes
                    MV = sum_{T != {}} (-1)^{n-|T|} Vol(sum_{k in T} conv S_k)  (scipy ConvexHull);
  * cramer        - Cramer's rule for n <= 3.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import mpmath
import numpy as np
from scipy.spatial import ConvexHull, QhullError


def mp_eval(sys, c, z, s, dps=50, shift=None):
    """G = [J_z | H_s | H] at one point with mpmath at `dps` digits; row k is multiplied by
    exp(-shift[k]) before rounding to double when `shift` is given."""
    with mpmath.workdps(dps):
        n = sys.n
        zz = [mpmath.mpc(complex(v)) for v in z]
        ss = mpmath.mpf(float(s))
        G = [[mpmath.mpc(0)] * (n + 2) for _ in range(n)]
        off = sys.offsets
        for k in range(n):
            for i in range(int(off[k]), int(off[k + 1])):
                a = [int(v) for v in sys.A[i]]
                e = sum(a[j] * zz[j] for j in range(n)) + mpmath.mpf(float(sys.w[i])) * ss
                if shift is not None:
                    e -= mpmath.mpf(float(shift[k]))
                term = mpmath.mpc(complex(c[i])) * mpmath.exp(e)
                for j in range(n):
                    G[k][j] += a[j] * term
                G[k][n] += mpmath.mpf(float(sys.w[i])) * term
                G[k][n + 1] += term
        return np.array([[complex(v) for v in row] for row in G])


def exact_eval(sys, c_frac, x_frac, t_frac):
    """Exact [x-partials scaled to log coordinates | t d/dt | value] at rational x, t.

    c_frac: list of (re, im) Fractions; x_frac: list of Fractions; t_frac: Fraction; integer
    liftings.  Returns rows of (re, im) Fraction pairs."""
    n = sys.n
    off = sys.offsets

    def cmul(a, b):
        return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])

    rows = []
    for k in range(n):
        row = [(Fraction(0), Fraction(0))] * (n + 2)
        for i in range(int(off[k]), int(off[k + 1])):
            mono = Fraction(1)
            for j in range(n):
                mono *= x_frac[j] ** int(sys.A[i][j])
            mono *= t_frac ** int(sys.w[i])
            term = cmul(c_frac[i], (mono, Fraction(0)))
            mults = [int(v) for v in sys.A[i]] + [int(sys.w[i]), 1]
            row = [(r[0] + q * term[0], r[1] + q * term[1]) for r, q in zip(row, mults)]
        rows.append(row)
    return rows


def np_F_J(sys, c, x):
    """F(x) = H(x, t=1) and J_x in affine coordinates, from the definition (numpy)."""
    n = sys.n
    F = np.zeros(n, np.complex128)
    J = np.zeros((n, n), np.complex128)
    off = sys.offsets
    for k in range(n):
        for i in range(int(off[k]), int(off[k + 1])):
            a = sys.A[i].astype(np.int64)
            mono = np.prod(x ** a)
            F[k] += c[i] * mono
            J[k] += c[i] * mono * a / x
    return F, J


def np_newton(sys, c, x0, iters=30, tol=1e-15):
    x = np.array(x0, np.complex128)
    for _ in range(iters):
        F, J = np_F_J(sys, c, x)
        dx = np.linalg.solve(J, -F)
        x = x + dx
        if np.abs(dx).max() <= tol * (1 + np.abs(x).max()):
            break
    return x


def np_F_J_batch(sys, c, X):
    """F and J_x at many points X [P][n] at once (numpy, from the definition): F [P][n],
    J [P][n][n]."""
    A = sys.A.astype(np.float64)
    mono = np.exp(np.log(X) @ A.T)  # x^a = e^{<a, log x>} for integer a (any branch of log)
    terms = mono * np.asarray(c)[None, :]
    eq = np.repeat(np.arange(sys.n), np.asarray(sys.m))
    P, n = X.shape
    F = np.zeros((P, n), np.complex128)
    J = np.zeros((P, n, n), np.complex128)
    for k in range(n):
        sel = eq == k
        F[:, k] = terms[:, sel].sum(1)
        J[:, k, :] = (terms[:, sel, None] * A[None, sel, :]).sum(1) / X
    return F, J


def np_newton_batch(sys, c, X0, iters=30):
    """Newton on F(x) = H(x, t=1) from every row of X0 [P][n] (numpy, affine x), until the
    largest relative step stops shrinking (rounding level) or `iters` iterations."""
    X = np.array(X0, np.complex128)
    prev = np.inf
    for _ in range(iters):
        F, J = np_F_J_batch(sys, c, X)
        dX = np.linalg.solve(J, -F[:, :, None])[:, :, 0]
        X = X + dX
        rel = (np.abs(dX).max(1) / np.abs(X).max(1)).max()
        if rel <= 1e-15 or rel >= 0.5 * prev:
            break
        prev = rel
    return X


def mixed_volume(sys):
    n = sys.n
    supports = [sys.A[sys.equation(k)].astype(np.float64) for k in range(n)]
    total = 0.0
    for r in range(1, n + 1):
        for T in itertools.combinations(range(n), r):
            pts = np.zeros((1, n))
            for k in T:
                pts = (pts[:, None, :] + supports[k][None, :, :]).reshape(-1, n)
            pts = np.unique(pts, axis=0)
            try:
                vol = ConvexHull(pts).volume
            except (QhullError, ValueError):
                vol = 0.0  # lower-dimensional
            total += (-1) ** (n - r) * vol
    return int(round(total))


def cramer(Jm, rhs):
    Jm = np.asarray(Jm, np.complex128)
    n = Jm.shape[0]
    assert n <= 3

    def det(M):
        if n == 1:
            return M[0, 0]
        if n == 2:
            return M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0]
        return (M[0, 0] * (M[1, 1] * M[2, 2] - M[1, 2] * M[2, 1])
                - M[0, 1] * (M[1, 0] * M[2, 2] - M[1, 2] * M[2, 0])
                + M[0, 2] * (M[1, 0] * M[2, 1] - M[1, 1] * M[2, 0]))

    D0 = det(Jm)
    out = np.zeros(n, np.complex128)
    for j in range(n):
        Mj = Jm.copy()
        Mj[:, j] = rhs
        out[j] = det(Mj) / D0
    return out
