"""Pins of the oracle's endpoint gradient with respect to the coefficients (implicit function
theorem, the argument behind the Davidenko equation of Sec. 2.3): J_x^H nu = -g,
grad c_{k,a} = sum_paths nu_k conj(x^a), PyTorch's convention dL/dRe c + i dL/dIm c."""
import numpy as np

import oracle
import pins
import workloads as W


def _endpoints(cfg="c5", P=16):
    csys, cell, z0 = W.planted_config(cfg, P=P)
    ze, _, _, st, _ = oracle.track(csys, csys.c, z0, -32.0)
    ok = st == oracle.OK
    return csys, ze[ok]


def _loss(sys, c, z_end):
    """L = sum |x*|^2 with x* re-solved by a numpy Newton from the given endpoints."""
    tot = 0.0
    for z in z_end:
        x = pins.np_newton(sys, c, np.exp(z))
        tot += float(np.sum(np.abs(x) ** 2))
    return tot


def test_grad_vs_central_differences():
    sys, ze = _endpoints()
    x = np.exp(ze)
    g, nsing = oracle.endpoint_grad(sys, sys.c, ze, 2 * x)
    assert nsing == 0
    rng = np.random.default_rng(3)
    h = 1e-6
    for i in rng.choice(sys.M, size=8, replace=False):
        fd = 0j
        for unit in (1.0, 1j):
            cp = sys.c.copy(); cp[i] += unit * h
            cm = sys.c.copy(); cm[i] -= unit * h
            d = (_loss(sys, cp, ze) - _loss(sys, cm, ze)) / (2 * h)
            fd += d * (1.0 if unit == 1.0 else 1j)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.abs(g).max()), (i, fd, g[i])


def test_grad_linear_in_upstream_and_additive_over_paths():
    sys, ze = _endpoints(P=12)
    rng = np.random.default_rng(1)
    g1 = rng.normal(size=ze.shape) + 1j * rng.normal(size=ze.shape)
    g2 = rng.normal(size=ze.shape) + 1j * rng.normal(size=ze.shape)
    a, _ = oracle.endpoint_grad(sys, sys.c, ze, g1)
    b, _ = oracle.endpoint_grad(sys, sys.c, ze, g2)
    ab, _ = oracle.endpoint_grad(sys, sys.c, ze, 2.0 * g1 - 3.0 * g2)
    np.testing.assert_allclose(ab, 2.0 * a - 3.0 * b, atol=1e-10 * np.abs(ab).max())
    h1, _ = oracle.endpoint_grad(sys, sys.c, ze[:5], g1[:5])
    h2, _ = oracle.endpoint_grad(sys, sys.c, ze[5:], g1[5:])
    np.testing.assert_allclose(h1 + h2, a, atol=1e-12 * np.abs(a).max())


def test_grad_scale_invariance():
    """Scaling all coefficients of one equation by lambda leaves the roots unchanged, so the
    gradient is orthogonal to that direction: Re sum_a conj(grad c_{k,a}) c_{k,a} = 0."""
    sys, ze = _endpoints(P=10)
    g, _ = oracle.endpoint_grad(sys, sys.c, ze, 2 * np.exp(ze))
    for k in range(sys.n):
        sl = sys.equation(k)
        v = np.vdot(g[sl], sys.c[sl])
        assert abs(v) <= 1e-9 * np.abs(g).max() * np.abs(sys.c[sl]).sum()
