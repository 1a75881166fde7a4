"""Pins of the oracle's evaluation of [J_z | H_s | H] (eq. (1)-(2), Sec. 5.1)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import pins
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _small(seed=0, n=3, m=4, lo=-2, hi=2, lift=31, P=32):
    rng = np.random.default_rng(seed)
    sys = W.random_system(n, m, W._uniform_exps(lo, hi), "unit", lift, rng, rng, rng)
    z, s = W.random_points(n, P, rng)
    return sys, z, s


def _scaled_err(G, ref, den):
    """componentwise error relative to sum_a |term_a| |C_a,col| (0/0 where a column is empty)"""
    diff = np.abs(G - ref)
    return np.where(den > 0, diff / np.where(den > 0, den, 1.0), diff)


def _sys_from_json(d):
    c = np.array([complex(a, b) for a, b in d["c"]])
    return W.System(d["n"], np.array(d["m"]), np.array(d["A"]), np.array(d["w"], float), c)


def test_golden_binomial_point():
    """Hand-worked values at x = (2, -1), t = 1/2 (tests/golden/binomial_2x2.json)."""
    g = json.load(open(os.path.join(GOLD, "binomial_2x2.json")))
    sys = _sys_from_json(g["system"])
    x = np.array(g["point"]["x"], float)
    t = float(Fraction(g["point"]["t"]))
    z = np.log(x.astype(complex))
    G, L = oracle.eval(sys, sys.c, z[None], np.array([np.log(t)]), scaled=False)
    want = np.array([[float(Fraction(v)) for v in row] for row in g["G_at_point"]])
    np.testing.assert_allclose(G[0], want, rtol=0, atol=1e-14)
    dE, dN, st, _ = oracle.step(sys, sys.c, z[None], np.array([np.log(t)]))
    np.testing.assert_allclose(dE[0], [float(Fraction(v)) for v in g["euler_at_point"]], atol=1e-14)
    np.testing.assert_allclose(dN[0], [float(Fraction(v)) for v in g["newton_at_point"]], atol=1e-14)


def test_exact_rational_points():
    """Exact rational evaluation (Fractions) at rational x, t with small integer coefficients."""
    rng = np.random.default_rng(5)
    for n, m in ((2, 3), (3, 4), (4, 5)):
        sys = W.random_system(n, m, W._uniform_exps(-2, 2), "unit", 7, rng, rng, rng)
        cre = rng.integers(-5, 6, size=sys.M)
        cim = rng.integers(-5, 6, size=sys.M)
        sys = sys.with_coefficients(cre + 1j * cim)
        xs = [Fraction(int(v), int(d)) for v, d in zip(rng.choice([-3, -2, -1, 1, 2, 3], n),
                                                        rng.integers(1, 4, n))]
        t = Fraction(1, 2)
        exact = pins.exact_eval(sys, [(Fraction(int(a)), Fraction(int(b))) for a, b in zip(cre, cim)], xs, t)
        want = np.array([[float(a) + 1j * float(b) for a, b in row] for row in exact])
        z = np.log(np.array([float(v) for v in xs], dtype=complex))
        G, _ = oracle.eval(sys, sys.c, z[None], np.array([np.log(0.5)]), scaled=False)
        scale = np.abs(want).max()
        np.testing.assert_allclose(G[0], want, rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mpmath_50_digits(seed):
    sys, z, s = _small(seed, P=8)
    G, L, den = oracle.eval(sys, sys.c, z, s, scaled=False, with_den=True)
    for p in range(len(s)):
        ref = pins.mp_eval(sys, sys.c, z[p], s[p])
        err = _scaled_err(G[p], ref, den[p])
        assert err.max() <= 1e-14, err.max()


def test_scaled_equals_unscaled():
    sys, z, s = _small(3, P=64)
    Gs, L = oracle.eval(sys, sys.c, z, s, scaled=True)
    Gu, L0 = oracle.eval(sys, sys.c, z, s, scaled=False)
    assert np.all(L0 == 0)
    np.testing.assert_allclose(Gs * np.exp(L)[:, :, None], Gu, rtol=1e-13, atol=1e-300)
    # scaled rows have their largest term magnitude at most |c| (= 1 here)
    _, _, den = oracle.eval(sys, sys.c, z, s, scaled=True, with_den=True)
    assert den[:, :, -1].max() <= sys.M


@pytest.mark.parametrize("imag_step", [False, True])
def test_central_differences(imag_step):
    """H is holomorphic in z: central differences along real and imaginary steps, and in s."""
    sys, z, s = _small(4, P=16)
    G, _ = oracle.eval(sys, sys.c, z, s, scaled=False)
    n = sys.n
    for j in range(n):
        h = 1e-5
        e = np.zeros(n, complex)
        e[j] = 1j * h if imag_step else h
        Gp, _ = oracle.eval(sys, sys.c, z + e, s, scaled=False)
        Gm, _ = oracle.eval(sys, sys.c, z - e, s, scaled=False)
        fd = (Gp[:, :, -1] - Gm[:, :, -1]) / (2 * e[j])
        np.testing.assert_allclose(fd, G[:, :, j], rtol=1e-8, atol=1e-8 * np.abs(G[:, :, j]).max())
    h = 1e-5
    Gp, _ = oracle.eval(sys, sys.c, z, s + h, scaled=False)
    Gm, _ = oracle.eval(sys, sys.c, z, s - h, scaled=False)
    fd = (Gp[:, :, -1] - Gm[:, :, -1]) / (2 * h)
    np.testing.assert_allclose(fd, G[:, :, n], rtol=1e-8, atol=1e-8 * np.abs(G[:, :, n]).max())


def test_branch_invariance():
    """Any branch of log gives the same values (Sec. 5.1): z_j + 2 pi i changes nothing."""
    sys, z, s = _small(6, P=32)
    G, L = oracle.eval(sys, sys.c, z, s)
    rng = np.random.default_rng(0)
    shift = 2j * np.pi * rng.integers(-3, 4, size=z.shape)
    G2, L2 = oracle.eval(sys, sys.c, z + shift, s)
    np.testing.assert_allclose(L2, L, atol=1e-14)
    np.testing.assert_allclose(G2, G, atol=1e-12)


def test_affine_jacobian_relation():
    """J_x = J_z diag(e^{-z}) (Sec. 5.1): compare with the numpy definition in x coordinates."""
    sys, z, _ = _small(7, P=8)
    G, _ = oracle.eval(sys, sys.c, z, np.zeros(len(z)), scaled=False)
    for p in range(len(z)):
        F, Jx = pins.np_F_J(sys, sys.c, np.exp(z[p]))
        np.testing.assert_allclose(G[p, :, :sys.n] * np.exp(-z[p])[None, :], Jx, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(G[p, :, -1], F, rtol=1e-12, atol=1e-13)


def test_zero_at_binomial_roots():
    rng = np.random.default_rng(11)
    sys = W.random_system(4, 5, W._uniform_exps(-2, 2), "unit", 15, rng, rng, rng)
    csys, cell = W.plant_cell(sys, 15, rng, min_det=8)
    z0 = W.binomial_start_points(csys, cell, 8, rng)
    # only the cell's two monomials per equation: the binomial system itself
    keep = np.concatenate([[csys.offsets[k] + j0, csys.offsets[k] + j1] for k, (j0, j1) in enumerate(cell)])
    bsys = W.System(4, np.full(4, 2), csys.A[keep], np.zeros(8), csys.c[keep])
    G, _, den = oracle.eval(bsys, bsys.c, z0, np.zeros(len(z0)), with_den=True)
    assert (np.abs(G[:, :, -1]) / den[:, :, -1]).max() < 1e-13


def test_monomial_permutation():
    sys, z, s = _small(8, P=16)
    G, L = oracle.eval(sys, sys.c, z, s)
    perm = np.concatenate([np.random.default_rng(1).permutation(np.arange(sys.offsets[k], sys.offsets[k + 1]))
                           for k in range(sys.n)])
    sys2 = W.System(sys.n, sys.m, sys.A[perm], sys.w[perm], sys.c[perm])
    G2, L2 = oracle.eval(sys2, sys2.c, z, s)
    np.testing.assert_allclose(G2, G, rtol=1e-13, atol=1e-14)


def test_scaled_underflow_regime():
    """t^w far below the FP64 range (s w ~ -2000): the scaled rows stay finite and nonzero and
    agree with a 50-digit evaluation carrying the same row scale."""
    sys, z, s = _small(9, lift=255, P=4)
    s = np.full(len(s), -8.0)
    sys = sys.with_lifting(sys.w + 250.0)
    G, L, den = oracle.eval(sys, sys.c, z, s, with_den=True)
    assert np.isfinite(G).all() and (np.abs(G[:, :, -1]) > 0).all()
    assert L.max() < -1900
    for p in range(len(s)):
        ref = pins.mp_eval(sys, sys.c, z[p], s[p], shift=L[p])
        err = _scaled_err(G[p], ref, den[p])
        assert err.max() <= 1e-13, err.max()
