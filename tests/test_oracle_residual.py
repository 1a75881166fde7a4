"""Pins of the oracle's relative residual r(x) = max_k |f_k(x)| / sum_a |c_{k,a} x^a| at t = 1.

f_k is the target system, eq. (1) at t = 1 (Sec. 2).  The residual is the endpoint test of every
tracking check, so it is pinned by references that share nothing with it:
  * hand-worked exact values (tests/golden/residual_2x2.json);
  * exact rational arithmetic (fractions.Fraction for f_k, 50-digit mpmath for the moduli) at
    rational points, including negative coordinates and negative exponents;
  * the closed form at perturbed roots of a binomial system: with x = x* e^delta and
    c_0 x*^{a_0} = -c_1 x*^{a_1}, row k equals |e^{<a_0,d>} - e^{<a_1,d>}| / (|e^{<a_0,d>}| +
    |e^{<a_1,d>}|), whatever the coefficients;
  * zeros at closed-form roots; invariance under per-equation scaling of the coefficients and
    under z_j -> z_j + 2 pi i.
"""
import json
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _sys_from_json(d):
    c = np.array([complex(a, b) for a, b in d["c"]])
    return W.System(d["n"], np.array(d["m"]), np.array(d["A"]), np.array(d["w"], float), c)


def test_golden_hand_worked_values():
    g = json.load(open(os.path.join(GOLD, "residual_2x2.json")))
    sys = _sys_from_json(g["system"])
    for pt in g["points"]:
        x = np.array([complex(a, b) for a, b in pt["x"]])
        z = np.log(x)
        r = oracle.residual(sys, sys.c, z[None])[0]
        want = float(Fraction(pt["r_squared"])) ** 0.5
        assert abs(r - want) <= 1e-15, (pt["x"], r, want)


def _msqrt(q):
    """square root of an exact non-negative Fraction, at the current mpmath precision"""
    return mpmath.sqrt(mpmath.mpf(q.numerator) / q.denominator)


def _exact_residual(sys, c_int, x_frac):
    """max_k |f_k| / sum |terms| with f_k exact (Fractions) and the moduli at 50 digits."""
    off = sys.offsets
    best = mpmath.mpf(0)
    with mpmath.workdps(50):
        for k in range(sys.n):
            fr, fi = Fraction(0), Fraction(0)
            den = mpmath.mpf(0)
            for i in range(int(off[k]), int(off[k + 1])):
                mono = Fraction(1)
                for j in range(sys.n):
                    mono *= x_frac[j] ** int(sys.A[i][j])
                tr, ti = c_int[i][0] * mono, c_int[i][1] * mono
                fr += tr
                fi += ti
                den += _msqrt(tr * tr + ti * ti)
            num = _msqrt(fr * fr + fi * fi)
            best = max(best, num / den)
        return float(best)


@pytest.mark.parametrize("n,m", [(2, 3), (3, 4), (4, 6)])
def test_exact_rational_points(n, m):
    rng = np.random.default_rng(100 + n)
    sys = W.random_system(n, m, W._uniform_exps(-3, 3), "unit", 7, rng, rng, rng)
    cre = rng.integers(-6, 7, size=sys.M)
    cim = rng.integers(-6, 7, size=sys.M)
    sys = sys.with_coefficients(cre + 1j * cim)
    c_int = [(Fraction(int(a)), Fraction(int(b))) for a, b in zip(cre, cim)]
    for _ in range(12):
        num = rng.choice([-3, -2, -1, 1, 2, 3], n)
        den = rng.integers(1, 4, n)
        xf = [Fraction(int(a), int(b)) for a, b in zip(num, den)]
        x = np.array([float(v) for v in xf], complex)
        r = oracle.residual(sys, sys.c, np.log(x)[None])[0]
        want = _exact_residual(sys, c_int, xf)
        assert abs(r - want) <= 1e-14 * max(1.0, n * m), (xf, r, want)


def _binomial(seed, n):
    rng = np.random.default_rng(seed)
    sys = W.random_system(n, 2, W._uniform_exps(-3, 3), "unit", 0, rng, rng, rng)
    D, beta = W.cell_binomial(sys, [(0, 1)] * n)
    while W.int_det(D) == 0:
        sys = W.random_system(n, 2, W._uniform_exps(-3, 3), "unit", 0, rng, rng, rng)
        D, beta = W.cell_binomial(sys, [(0, 1)] * n)
    det = abs(W.int_det(D))
    roots = W.binomial_roots(D, beta, min(det, 8), rng)
    return sys, roots, rng


@pytest.mark.parametrize("n", [2, 3, 5])
def test_zero_at_binomial_roots_and_closed_form_when_perturbed(n):
    sys, roots, rng = _binomial(7 + n, n)
    assert oracle.residual(sys, sys.c, roots).max() <= 1e-14
    a0 = sys.A[0::2].astype(float)  # equation k's monomials are rows 2k, 2k + 1
    a1 = sys.A[1::2].astype(float)
    for scale in (1e-9, 1e-6, 1e-3, 0.1):
        d = scale * (rng.standard_normal(roots.shape) + 1j * rng.standard_normal(roots.shape))
        r = oracle.residual(sys, sys.c, roots + d)
        e0, e1 = np.exp(d @ a0.T), np.exp(d @ a1.T)
        want = (np.abs(e0 - e1) / (np.abs(e0) + np.abs(e1))).max(axis=1)
        assert np.all(np.abs(r - want) <= 1e-14 + 1e-10 * want), (scale, r, want)
        assert want.min() > 0


def test_invariances():
    """Per-equation coefficient scaling and the branch of log change nothing; a point with a
    huge |x| stays finite."""
    rng = np.random.default_rng(3)
    sys = W.random_system(4, 5, W._uniform_exps(-3, 3), "unit", 7, rng, rng, rng)
    z, _ = W.random_points(4, 64, rng)
    r = oracle.residual(sys, sys.c, z)
    lam = np.repeat(rng.uniform(0.1, 10, 4) * np.exp(1j * rng.uniform(0, 6.3, 4)), sys.m)
    np.testing.assert_allclose(oracle.residual(sys, sys.c * lam, z), r, rtol=1e-13, atol=0)
    zb = z + 2j * np.pi * rng.integers(-3, 4, z.shape)
    np.testing.assert_allclose(oracle.residual(sys, sys.c, zb), r, rtol=1e-12, atol=0)
    assert np.all((r >= 0) & (r <= 1))


def test_rejects_too_many_unknowns():
    rng = np.random.default_rng(4)
    sys = W.random_system(33, 2, W._uniform_exps(-1, 1), "unit", 3, rng, rng, rng)
    with pytest.raises(ValueError):
        oracle.residual(sys, sys.c, np.zeros((1, 33), complex))
    with pytest.raises(ValueError):
        oracle.eval(sys, sys.c, np.zeros((1, 33), complex), np.zeros(1))
