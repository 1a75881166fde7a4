"""Pins of the oracle's binomial start-system roots (Sec. 2: the start points of polyhedral
homotopy are the roots of each mixed cell's binomial system x^{d_k} = beta_k)."""
import numpy as np
import pytest

import oracle
import workloads as W


def _residual(D, beta, z):
    """max_k |e^{<d_k, z>} - beta_k| / |beta_k| per root, from the definition."""
    return (np.abs(np.exp(z @ np.asarray(D, np.float64).T) - beta[None, :]) / np.abs(beta)).max(1)


def _mod2pi_pairwise_min(z):
    """smallest distance between two roots, imaginary parts compared mod 2 pi"""
    d = z[:, None, :] - z[None, :, :]
    d = np.maximum(np.abs(d.real), np.abs(np.angle(np.exp(1j * d.imag)))).max(2)
    d[np.arange(len(z)), np.arange(len(z))] = np.inf
    return d.min()


def _same_set(a, b, tol=1e-10):
    assert a.shape == b.shape
    for row in a:
        d = np.maximum(np.abs(b.real - row.real), np.abs(np.angle(np.exp(1j * (b.imag - row.imag)))))
        assert d.max(1).min() <= tol


def _random_cell(rng, n, lo=-3, hi=3, max_det=400):
    while True:
        D = rng.integers(lo, hi + 1, size=(n, n))
        det = round(abs(np.linalg.det(D)))
        if 0 < det <= max_det:
            beta = rng.normal(size=n) + 1j * rng.normal(size=n)
            return D, beta, det


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (4, 3), (6, 4), (8, 5)])
def test_roots_satisfy_the_system_count_and_distinct(n, seed):
    """Every root solves x^{d_k} = beta_k; there are |det D| of them, pairwise distinct."""
    rng = np.random.default_rng(seed)
    D, beta, det = _random_cell(rng, n)
    z = oracle.binomial_roots(D, beta)
    assert z.shape == (det, n)
    assert _residual(D, beta, z).max() <= 1e-11
    if det > 1:
        assert _mod2pi_pairwise_min(z) > 1e-6
    assert (z.imag >= -np.pi).all() and (z.imag < np.pi).all()


def test_one_variable_closed_form():
    """x^d = beta: the d roots e^{(log beta + 2 pi i k) / d}."""
    for d, beta in ((1, 2.0 + 1j), (5, -3.0), (-4, 0.5j), (12, 1.0)):
        z = oracle.binomial_roots([[d]], [beta])
        k = np.arange(abs(d))
        ref = (np.log(complex(beta)) + 2j * np.pi * k) / d
        ref = ref.real + 1j * (np.mod(ref.imag + np.pi, 2 * np.pi) - np.pi)
        _same_set(z, ref[:, None])


def test_diagonal_closed_form():
    """D = diag(d): the product of the one-variable root sets."""
    d, beta = [2, -3, 4], np.array([1.5 - 0.5j, -2.0, 0.25j])
    z = oracle.binomial_roots(np.diag(d), beta)
    per = []
    for dj, bj in zip(d, beta):
        r = (np.log(bj) + 2j * np.pi * np.arange(abs(dj))) / dj
        per.append(r.real + 1j * (np.mod(r.imag + np.pi, 2 * np.pi) - np.pi))
    ref = np.array([list(t) for t in __import__("itertools").product(*per)])
    _same_set(z, ref)


def test_equation_order_invariance():
    """Permuting the equations (rows of D with their beta) leaves the root set unchanged."""
    rng = np.random.default_rng(7)
    D, beta, _ = _random_cell(rng, 4)
    perm = rng.permutation(4)
    _same_set(oracle.binomial_roots(D, beta), oracle.binomial_roots(D[perm], beta[perm]))


def test_agrees_with_smith_form_generator():
    """The input workloads' Smith-form generator (a different lattice enumeration) gives the
    same root set for a planted cell and for random cells."""
    csys, cell, _ = W.planted_config("c1", P=4)
    cases = [W.cell_binomial(csys, cell)]
    rng = np.random.default_rng(8)
    for n in (2, 3, 5):
        D, beta, _ = _random_cell(rng, n, max_det=120)
        cases.append((D, beta))
    for D, beta in cases:
        z = oracle.binomial_roots(D, beta)
        ref = W.binomial_roots(D, beta, len(z), np.random.default_rng(0))
        _same_set(z, ref)


def test_planted_mistakes_fail_the_pins(monkeypatch):
    """Plausible mistakes planted in the oracle fail the pins: dropping V (z = H^{-1} k instead of
    V H^{-1} k) fails the residual; a box one short in its last coordinate fails the count."""
    import oracle.binomial as B
    rng = np.random.default_rng(9)
    D, beta, det = _random_cell(rng, 4, max_det=60)
    H, V = B.hermite_lower(D)
    assert np.array_equal(np.asarray(D, dtype=object) @ np.asarray(V, dtype=object),
                          np.asarray(H, dtype=object))
    assert int(np.prod([H[i][i] for i in range(4)])) == det
    orig = B.hermite_lower

    def no_v(D):
        H, _ = orig(D)
        return H, [[int(i == j) for j in range(len(H))] for i in range(len(H))]
    monkeypatch.setattr(B, "hermite_lower", no_v)
    assert _residual(D, beta, B.binomial_roots(D, beta)).max() > 1e-3

    def short_box(D):
        H, V = orig(D)
        H = [row[:] for row in H]
        H[-1][-1] -= 1
        return H, V
    monkeypatch.setattr(B, "hermite_lower", short_box)
    bad = B.binomial_roots(D, beta)
    assert len(bad) != det or _residual(D, beta, bad).max() > 1e-3
