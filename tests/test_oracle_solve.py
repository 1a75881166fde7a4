"""Pins of the oracle's consolidated Euler/Newton solve (Sec. 2.3 and the unified system of Sec. 6):
dE = -J_z^{-1} H_s, dN = -J_z^{-1} H from one partially pivoted LU of [J_z | H_s | H]."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import pins
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _cfg_small(n, m, seed, P=64):
    rng = np.random.default_rng(seed)
    sys = W.random_system(n, m, W._uniform_exps(-3, 3), "unit", 31, rng, rng, rng)
    z, s = W.random_points(n, P, rng)
    return sys, z, s


@pytest.mark.parametrize("n,m", [(2, 3), (3, 4), (6, 8), (10, 12)])
def test_lapack(n, m):
    """Against LAPACK zgesv (numpy.linalg.solve) on the unscaled system."""
    sys, z, s = _cfg_small(n, m, n)
    G, _ = oracle.eval(sys, sys.c, z, s, scaled=False)
    dE, dN, st, ratio = oracle.step(sys, sys.c, z, s)
    assert (st == 0).all()
    ref = np.linalg.solve(G[:, :, :n], -G[:, :, n:n + 2])
    cond = np.linalg.cond(G[:, :, :n])
    ok = cond < 1e6
    for X, col in ((dE, 0), (dN, 1)):
        err = np.abs(X - ref[:, :, col]).max(1) / np.abs(ref[:, :, col]).max(1)
        assert (err[ok] <= 50 * cond[ok] * 2.0 ** -53).all()


def test_cramer():
    for n in (1, 2, 3):
        sys, z, s = _cfg_small(n, 4, 20 + n, P=32)
        G, _ = oracle.eval(sys, sys.c, z, s, scaled=False)
        dE, dN, st, _ = oracle.step(sys, sys.c, z, s)
        for p in range(len(s)):
            if np.linalg.cond(G[p, :, :n]) > 1e10:
                continue  # (near-)singular point: no unique directions to compare
            tol = 20 * np.linalg.cond(G[p, :, :n]) * 2.0 ** -53
            e = pins.cramer(G[p, :, :n], -G[p, :, n])
            nn = pins.cramer(G[p, :, :n], -G[p, :, n + 1])
            assert np.abs(dE[p] - e).max() <= tol * np.abs(e).max()
            assert np.abs(dN[p] - nn).max() <= tol * np.abs(nn).max()


def test_backward_error():
    """||J x + b|| / (||J|| ||x|| + ||b||) at the level of a few n eps."""
    sys, z, s = _cfg_small(10, 12, 3, P=128)
    G, _ = oracle.eval(sys, sys.c, z, s)
    dE, dN, st, _ = oracle.step(sys, sys.c, z, s)
    n = sys.n
    J = G[:, :, :n]
    for X, col in ((dE, n), (dN, n + 1)):
        b = G[:, :, col]
        r = np.abs(np.einsum("pij,pj->pi", J, X) + b).max(1)
        scale = np.abs(J).sum(2).max(1) * np.abs(X).max(1) + np.abs(b).max(1)
        assert (r / scale).max() <= 10 * n * 2.0 ** -53


def test_golden_binomial_euler_everywhere():
    """Binomial homotopy: the Euler direction is D^{-1}(w_0 - w_1) at every point."""
    g = json.load(open(os.path.join(GOLD, "binomial_2x2.json")))
    d = g["system"]
    sys = W.System(d["n"], np.array(d["m"]), np.array(d["A"]), np.array(d["w"], float),
                   np.array([complex(a, b) for a, b in d["c"]]))
    rng = np.random.default_rng(0)
    z, s = W.random_points(2, 64, rng)
    dE, dN, st, _ = oracle.step(sys, sys.c, z, s)
    want = np.array([float(Fraction(v)) for v in g["euler_everywhere"]])
    np.testing.assert_allclose(dE, np.broadcast_to(want, dE.shape), atol=1e-13)


def test_binomial_closed_form_directions():
    """Raw-lifted binomial systems (m_k = 2): dE = D^{-1}(w_{k,0} - w_{k,1}) and dN = 0 on the path."""
    rng = np.random.default_rng(4)
    for n in (2, 4, 7):
        A = rng.integers(-3, 4, size=(2 * n, n))
        D = A[1::2] - A[0::2]
        if W.int_det(D) == 0:
            continue
        w = rng.integers(0, 20, size=2 * n).astype(float)
        c = np.exp(2j * np.pi * rng.random(2 * n))
        sys = W.System(n, np.full(n, 2), A, w, c)
        delta = w[1::2] - w[0::2]
        beta = -c[0::2] / c[1::2]
        s = rng.uniform(-5, 0, size=16)
        z = np.array([np.linalg.solve(D.astype(float), np.log(beta) - delta * sv) for sv in s])
        dE, dN, st, _ = oracle.step(sys, sys.c, z, s)
        want = np.linalg.solve(D.astype(float), w[0::2] - w[1::2])
        tol = 1e-13 * np.linalg.cond(D.astype(float)) * max(1.0, np.abs(want).max())
        assert np.abs(dE - want[None, :]).max() <= tol
        assert np.abs(dN).max() <= tol


def test_row_scaling_invariance():
    """The directions do not depend on the per-row scale e^{-M_k}."""
    sys, z, s = _cfg_small(6, 8, 9)
    dE, dN, _, _ = oracle.step(sys, sys.c, z, s)
    G, _ = oracle.eval(sys, sys.c, z, s, scaled=False)
    ref = np.linalg.solve(G[:, :, :6], -G[:, :, 6:8])
    np.testing.assert_allclose(dE, ref[:, :, 0], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(dN, ref[:, :, 1], rtol=1e-9, atol=1e-12)


def test_singular_detected():
    """Two proportional equations give a singular J_z (status -1)."""
    rng = np.random.default_rng(2)
    sys = W.random_system(3, 4, W._uniform_exps(-2, 2), "unit", 5, rng, rng, rng)
    A = sys.A.copy()
    c = sys.c.copy()
    A[4:8] = A[0:4]
    c[4:8] = 2.0 * c[0:4]
    w = sys.w.copy()
    w[4:8] = w[0:4]
    bad = W.System(3, sys.m, A, w, c)
    z, s = W.random_points(3, 8, rng)
    _, _, st, ratio = oracle.step(bad, bad.c, z, s)
    assert (ratio < 1e-12).all()
