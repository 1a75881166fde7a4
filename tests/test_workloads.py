"""The seeded input generators: Smith normal form, binomial start roots, planted cells."""
import numpy as np
import pytest
from sympy import Matrix
from sympy.matrices.normalforms import invariant_factors

import pins
import workloads as W


def test_smith_normal_form_vs_sympy():
    rng = np.random.default_rng(0)
    done = 0
    while done < 25:
        n = int(rng.integers(2, 9))
        D = rng.integers(-6, 7, size=(n, n))
        if W.int_det(D) == 0:
            continue
        U, sigma, V = W.smith_normal_form(D)
        S = np.array(U, dtype=object) @ np.array(D, dtype=object) @ np.array(V, dtype=object)
        assert (S == np.diag(sigma)).all()
        assert [abs(int(v)) for v in invariant_factors(Matrix(D.tolist()))] == sigma
        assert abs(int(Matrix(U).det())) == 1 and abs(int(Matrix(V).det())) == 1
        done += 1


def test_int_det_vs_sympy():
    rng = np.random.default_rng(1)
    for _ in range(20):
        D = rng.integers(-6, 7, size=(7, 7))
        assert W.int_det(D) == int(Matrix(D.tolist()).det())


def test_binomial_roots_count_and_distinct():
    rng = np.random.default_rng(2)
    for _ in range(6):
        n = int(rng.integers(2, 5))
        D = rng.integers(-3, 4, size=(n, n))
        det = abs(W.int_det(D))
        if det == 0 or det > 400:
            continue
        beta = np.exp(2j * np.pi * rng.random(n)) * rng.uniform(0.5, 2, n)
        z = W.binomial_roots(D, beta, det, rng)
        key = {tuple(v) for v in np.round(np.c_[z.real, np.mod(z.imag + 1e-9, 2 * np.pi)] * 1e8)}
        assert len(key) == det
        lhs = np.exp(z @ D.T.astype(float))  # x^{d_k} = exp(<d_k, z>)
        np.testing.assert_allclose(lhs, np.broadcast_to(beta, lhs.shape), rtol=1e-12)


def test_planted_cell_is_mixed_cell():
    """The planted pair has lifting 0 and every other monomial a positive one, so with inner
    normal (0, 1) the pair is the unique minimiser in each equation."""
    csys, cell, z0 = W.planted_config("c5", P=64)
    off = csys.offsets
    for k, (j0, j1) in enumerate(cell):
        wk = csys.w[off[k]:off[k + 1]]
        assert wk[j0] == 0 and wk[j1] == 0
        assert (np.delete(wk, [j0, j1]) >= 1).all()
    D, _ = W.cell_binomial(csys, cell)
    assert abs(W.int_det(D)) >= 64


def test_configs_shapes():
    for cfg, (n, m) in {"c1": (3, 4), "c2": (10, 12), "c5": (8, 16)}.items():
        sys, z, s = W.config_system(cfg, P=128)
        assert sys.n == n and (sys.m == m).all()
        assert z.shape == (128, n) and s.min() >= -8 and s.max() <= 0
        for k in range(n):  # no duplicate monomials inside an equation
            rows = {tuple(r) for r in sys.A[sys.equation(k)]}
            assert len(rows) == m
    sys, _, _ = W.config_system("c3", P=16)
    frac0 = (sys.A == 0).mean()
    assert 0.25 < frac0 < 0.35 and np.abs(sys.A).max() == 4
    # the sizes of the paper's timing systems: n = 14 with 184 monomials, n = 24 with 324, split
    # as evenly as possible over the equations, 0/1 exponents with about 30% ones, distinct rows
    for cfg, (n, M) in {"ps14": (14, 184), "ps24": (24, 324)}.items():
        sys, z, s = W.config_system(cfg, P=1000)
        assert sys.n == n and int(sys.m.sum()) == M and sys.m.max() - sys.m.min() <= 1
        assert set(np.unique(sys.A)) <= {0, 1} and 0.25 < sys.A.mean() < 0.35
        assert z.shape == (1000, n)
        for k in range(n):
            rows = {tuple(r) for r in sys.A[sys.equation(k)]}
            assert len(rows) == sys.m[k]


def test_seeded_reproducible():
    a = W.config_system("c2", P=64)
    b = W.config_system("c2", P=64)
    assert np.array_equal(a[0].A, b[0].A) and np.array_equal(a[1], b[1])
