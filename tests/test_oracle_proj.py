"""Pins of the oracle's projective step (Sec. 2.2, eq. (3)-(5); the unified system of Sec. 6):
the Euler and Newton directions in homogeneous coordinates y in C^{n+1}.

- exact rational values: a one-variable system at rational points, Cramer's rule on the 2 x 2
  system in Gaussian rationals (Fractions), from the homogenised polynomial written out by hand;
- the affine form carried into homogeneous coordinates: at y = (x, 1) the Jacobian's first n
  columns are J_x = J_z diag(1/x) from the (pinned) affine evaluation, and the homogenising
  column follows from Euler's identity sum_j y_j dh~/dy_j = d_k h~ (no homogenising exponent
  is used), so the two directions are numpy solves of an independently built system;
- homogeneity: both directions are homogeneous of degree one in y;
- on a path (closed-form binomial points, H = 0): dN = 0 and dE is the affine Euler direction
  dx/ds = x * dz/ds projected orthogonally to y.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W


def _sys(n, m, seed, lo=-2, hi=2, lift=15):
    rng = np.random.default_rng(seed)
    return W.random_system(n, m, W._uniform_exps(lo, hi), "unit", lift, rng, rng, rng)


def _points(n, P, seed, s_lo=-3.0):
    rng = np.random.default_rng(seed)
    y = (np.exp(rng.normal(0, 0.5, (P, n + 1))) *
         np.exp(1j * rng.uniform(0, 2 * np.pi, (P, n + 1))))
    s = rng.uniform(s_lo, 0.0, P)
    return y, s


def _rel(a, b):
    return np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)


# ---- exact rational values ------------------------------------------------------------------
class Q:
    """Gaussian rational"""

    def __init__(self, re, im=0):
        self.re, self.im = Fraction(re), Fraction(im)

    def __add__(self, o):
        return Q(self.re + o.re, self.im + o.im)

    def __sub__(self, o):
        return Q(self.re - o.re, self.im - o.im)

    def __mul__(self, o):
        return Q(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def __truediv__(self, o):
        den = o.re * o.re + o.im * o.im
        return Q((self.re * o.re + self.im * o.im) / den, (self.im * o.re - self.re * o.im) / den)

    def conj(self):
        return Q(self.re, -self.im)

    def powi(self, e):
        r = Q(1)
        b = self if e >= 0 else Q(1) / self
        for _ in range(abs(e)):
            r = r * b
        return r

    def c(self):
        return complex(float(self.re), float(self.im))


def test_exact_rational_one_variable():
    """f(x) = c0 x^-1 + c1 x^2 + c2 with liftings (3, 0, 5): d = 2, homogenised exponents
    (-1, 3), (2, 0), (0, 2), so h~(y0, y1, s) = c0 y0^-1 y1^3 t^3 + c1 y0^2 + c2 y1^2 t^5.
    At s = 0 (t = 1), for Gaussian-rational c and y, Cramer's rule on
    [[dh/dy0, dh/dy1], [conj y0, conj y1]] v = [-rhs, 0] gives the exact directions."""
    A = np.array([[-1], [2], [0]], np.int8)
    w = np.array([3.0, 0.0, 5.0])
    cq = [Q(1, 2), Q(-3, 1), Q(Fraction(1, 2), -1)]
    sys_ = W.System(1, np.array([3], np.int32), A, w, np.array([q.c() for q in cq]))
    for y0, y1 in ((Q(1, 1), Q(2, -1)), (Q(Fraction(3, 2), 0), Q(-1, Fraction(1, 3))),
                   (Q(0, 2), Q(Fraction(5, 4), Fraction(1, 4)))):
        terms = [cq[0] * y0.powi(-1) * y1.powi(3), cq[1] * y0.powi(2), cq[2] * y1.powi(2)]
        H = terms[0] + terms[1] + terms[2]
        Hs = terms[0] * Q(3) + terms[2] * Q(5)
        d0 = cq[0] * Q(-1) * y0.powi(-2) * y1.powi(3) + cq[1] * Q(2) * y0
        d1 = cq[0] * Q(3) * y0.powi(-1) * y1.powi(2) + cq[2] * Q(2) * y1
        a, b, cc, dd = d0, d1, y0.conj(), y1.conj()
        det = a * dd - b * cc

        def cramer(rhs0):  # [[a, b], [cc, dd]] v = [rhs0, 0]
            return [rhs0 * dd / det, (Q(0) - cc * rhs0) / det]

        eE = cramer(Q(0) - Hs)
        eN = cramer(Q(0) - H)
        dE, dN, st, _, d = oracle.step_proj(sys_, sys_.c, np.array([[y0.c(), y1.c()]]), 0.0)
        assert st[0] == 0 and d[0] == 2
        np.testing.assert_allclose(dE[0], [v.c() for v in eE], rtol=1e-13)
        np.testing.assert_allclose(dN[0], [v.c() for v in eN], rtol=1e-13)


# ---- the affine form carried into homogeneous coordinates -----------------------------------
@pytest.mark.parametrize("n,m,seed", [(3, 4, 1), (5, 7, 2), (8, 16, 3)])
def test_matches_affine_through_euler_identity(n, m, seed):
    sys_ = _sys(n, m, seed)
    P = 200
    rng = np.random.default_rng(seed + 100)
    z = rng.normal(0, 0.5, (P, n)) + 1j * rng.uniform(0, 2 * np.pi, (P, n))
    s = rng.uniform(-3.0, 0.0, P)
    x = np.exp(z)
    G, _ = oracle.eval(sys_, sys_.c, z, s)  # rows scaled by e^{-M_k}: directions unchanged
    Jz, Hs, H = G[:, :, :n], G[:, :, n], G[:, :, n + 1]
    d = np.array([int(sys_.A[sys_.equation(k)].astype(int).sum(1).max()) for k in range(n)])
    Jy = np.zeros((P, n + 1, n + 1), complex)
    Jy[:, :n, :n] = Jz / x[:, None, :]
    Jy[:, :n, n] = d[None, :] * H - Jz.sum(2)  # Euler's identity at y_n = 1
    Jy[:, n, :n] = np.conj(x)
    Jy[:, n, n] = 1.0
    rhs = np.zeros((P, n + 1, 2), complex)
    rhs[:, :n, 0] = -Hs
    rhs[:, :n, 1] = -H
    ref = np.linalg.solve(Jy, rhs)
    y = np.concatenate([x, np.ones((P, 1))], axis=1)
    dE, dN, st, ratio, dd = oracle.step_proj(sys_, sys_.c, y, s)
    assert np.array_equal(dd, d)
    kappa = np.linalg.cond(Jy, p=np.inf)
    ok = (st == 0) & (kappa < 1e6)
    assert ok.sum() >= P // 2
    tol = 1e-15 * kappa[ok] * 100
    assert (_rel(dE[ok], ref[ok, :, 0]) <= np.maximum(tol, 1e-12)).all()
    assert (_rel(dN[ok], ref[ok, :, 1]) <= np.maximum(tol, 1e-12)).all()


@pytest.mark.parametrize("n,m,seed", [(3, 4, 4), (8, 16, 5)])
def test_homogeneous_of_degree_one(n, m, seed):
    sys_ = _sys(n, m, seed)
    y, s = _points(n, 100, seed + 7)
    rng = np.random.default_rng(seed + 9)
    lam = np.exp(rng.normal(0, 0.7, 100)) * np.exp(1j * rng.uniform(0, 2 * np.pi, 100))
    a = oracle.step_proj(sys_, sys_.c, y, s)
    b = oracle.step_proj(sys_, sys_.c, y * lam[:, None], s)
    ok = (a[2] == 0) & (a[3] > 1e-8)
    assert ok.sum() >= 50
    assert (_rel(b[0][ok], lam[ok, None] * a[0][ok]) <= 1e-10).all()
    assert (_rel(b[1][ok], lam[ok, None] * a[1][ok]) <= 1e-10).all()
    # the constraint row: y^* d = 0
    for v in (a[0], a[1]):
        dot = np.abs(np.sum(np.conj(y[ok]) * v[ok], axis=1))
        assert (dot <= 1e-12 * np.abs(y[ok]).max(1) * np.abs(v[ok]).max(1)).all()


def test_on_a_binomial_path():
    """Closed-form points of a raw-lifted binomial system's path (H = 0): dN = 0 and dE is the
    projection of (x * dz/ds, 0) orthogonal to y = (x, 1), dz/ds = D^{-1} (w_{k,0} - w_{k,1})."""
    rng = np.random.default_rng(77)
    n = 3
    Dm = np.array([[2, 1, 0], [0, 1, -1], [1, 0, 3]])
    A = np.zeros((2 * n, n), np.int8)
    for k in range(n):
        A[2 * k + 1] = Dm[k]
    w = rng.integers(0, 6, 2 * n).astype(float)
    c = np.exp(1j * rng.uniform(0, 2 * np.pi, 2 * n))
    sys_ = W.System(n, np.full(n, 2, np.int32), A, w, c)
    delta = w[1::2] - w[0::2]
    beta = -c[0::2] / c[1::2]
    dz = np.linalg.solve(Dm.astype(float), -delta)  # dz/ds on the path
    for s in (-2.0, -0.7, 0.0):
        # D z = log(beta) - delta s (one branch)
        z = np.linalg.solve(Dm.astype(float), np.log(beta) - delta * s)
        x = np.exp(z)
        y = np.concatenate([x, [1.0]])
        dE, dN, st, _, _ = oracle.step_proj(sys_, sys_.c, y[None], s)
        assert st[0] == 0
        assert np.abs(dN[0]).max() <= 1e-13 * np.abs(y).max()
        v = np.concatenate([x * dz, [0.0]])
        proj = v - (np.vdot(y, v) / np.vdot(y, y)) * y
        np.testing.assert_allclose(dE[0], proj, rtol=0, atol=1e-13 * np.abs(proj).max())
