"""Oracle: every root of a binomial start system (TEST INFRASTRUCTURE ONLY).

Sec. 2: the start points of polyhedral homotopy are the roots of the binomial systems of the
mixed cells, x^{d_k} = beta_k for k = 0..n-1 (d_k the difference of the cell's two exponent
vectors in equation k, beta_k = -c_{k,j0} / c_{k,j1}); the paper treats them as given.  In log
coordinates z = log x the system reads D z = log(beta) + 2 pi i k over integer vectors k, and
its roots in (C*)^n are |det D| points.

Method (plain, exact where it matters):
  * Re z is the same for every root: D^{-1} log|beta| (numpy solve), and one root is
    z_base = D^{-1} log(beta) with the principal logarithm.
  * The others are z_base + 2 pi i y with y = D^{-1} k mod 1.  Two integer vectors give the same
    root iff they differ by an element of D Z^n.  With the lower-triangular Hermite form
    H = D V (V unimodular, column operations, exact Python integers), D Z^n = H Z^n, whose
    representatives are the box 0 <= k_i < H_ii; so the roots are indexed by that box, and
    y = D^{-1} k = V H^{-1} k is formed in exact rationals (forward substitution with H).
  * Imaginary parts are reduced into [-pi, pi).

Slow by design (Python integers and Fractions per root); for the small systems of the tests.
Parity status: pinned by tests/test_oracle_binomial.py (residuals of every root from the
definition, count = |det D| with pairwise distinct roots, closed forms for n = 1 and diagonal D,
invariance under reordering the equations, agreement with the Smith-form generator of the
input workloads).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def hermite_lower(D):
    """Lower-triangular Hermite form by integer column operations: returns (H, V) with
    H = D V, V unimodular, H[i][j] = 0 for j > i and H[i][i] > 0.  D must be nonsingular."""
    H = [[int(v) for v in row] for row in np.asarray(D)]
    n = len(H)
    V = [[int(i == j) for j in range(n)] for i in range(n)]

    def col_op(i, j, a, b, c, d):
        # (col i, col j) <- (a col i + b col j, c col i + d col j), a d - b c = +-1
        for X in (H, V):
            for row in X:
                x, y = row[i], row[j]
                row[i], row[j] = a * x + b * y, c * x + d * y

    for i in range(n):
        for j in range(i + 1, n):  # clear H[i][j] against H[i][i] with an extended gcd
            x, y = H[i][i], H[i][j]
            if y == 0:
                continue
            g, s, t = _ext_gcd(x, y)  # s x + t y = g
            # new col i = s col i + t col j; new col j = (-y/g) col i + (x/g) col j
            col_op(i, j, s, t, -y // g, x // g)
        if H[i][i] == 0:
            raise ValueError("singular matrix")
        if H[i][i] < 0:
            for X in (H, V):
                for row in X:
                    row[i] = -row[i]
    return H, V


def _ext_gcd(a, b):
    """(g, s, t) with s a + t b = g = gcd(a, b) >= 0."""
    s0, s1, t0, t1 = 1, 0, 0, 1
    while b:
        q = a // b
        a, b = b, a - q * b
        s0, s1 = s1, s0 - q * s1
        t0, t1 = t1, t0 - q * t1
    if a < 0:
        a, s0, t0 = -a, -s0, -t0
    return a, s0, t0


def binomial_roots(D, beta):
    """All |det D| roots of x^{d_k} = beta_k as z = log x, complex128 [count][n], in the order of
    the Hermite box (k_0 slowest)."""
    D = np.asarray(D, dtype=np.int64)
    beta = np.asarray(beta, dtype=np.complex128)
    n = D.shape[0]
    assert D.shape == (n, n) and beta.shape == (n,)
    if not np.all(np.isfinite(beta)) or np.any(beta == 0):
        raise ValueError("beta must be finite and nonzero")
    H, V = hermite_lower(D)
    z_base = np.linalg.solve(D.astype(np.float64), np.log(beta))
    out = []
    for k in itertools.product(*[range(H[i][i]) for i in range(n)]):
        u = []  # u = H^{-1} k, exact
        for i in range(n):
            acc = Fraction(k[i]) - sum((H[i][j] * u[j] for j in range(i)), Fraction(0))
            u.append(acc / H[i][i])
        y = [sum((V[i][j] * u[j] for j in range(n)), Fraction(0)) for i in range(n)]
        frac = np.array([float(v - (v.numerator // v.denominator)) for v in y])
        z = z_base + 2j * np.pi * frac
        out.append(z.real + 1j * (np.mod(z.imag + np.pi, 2.0 * np.pi) - np.pi))
    return np.array(out, dtype=np.complex128).reshape(-1, n)
