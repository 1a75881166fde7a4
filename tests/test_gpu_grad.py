"""GPU parity of hom_endpoint_grad and the HomTrack autograd.Function."""
import numpy as np
import pytest

import oracle
import pins
import workloads as W
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hom():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    import paper_2111_14317_amd as hom
    return hom


def _endpoints(P=256):
    csys, cell, z0 = W.planted_config("c5", P=P)
    ze, _, _, st, _ = oracle.track(csys, csys.c, z0, -32.0)
    return csys, ze[st == 0], z0[st == 0]


def test_grad_vs_oracle(hom):
    say("[grad] c5 P=256 fp64 and mixed vs oracle")
    sys, ze, _ = _endpoints()
    g = 2 * np.exp(ze)
    ref, ns = oracle.endpoint_grad(sys, sys.c, ze, g)
    assert ns == 0
    h = hom.System.from_workload(sys)
    for prec, tol in ((hom.FP64, 1e-10), (hom.MIXED, 1e-4)):
        got = hom.endpoint_grad(h, sys.c, ze, g, precision=prec).cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"  prec {prec}: rel err {err:.3e}")
        assert err <= tol


def test_grad_deterministic_and_chunked(hom):
    say("[grad determinism] c5 P=256")
    sys, ze, _ = _endpoints()
    h = hom.System.from_workload(sys)
    g = 2 * np.exp(ze)
    a = hom.endpoint_grad(h, sys.c, ze, g).cpu().numpy()
    b = hom.endpoint_grad(h, sys.c, ze, g).cpu().numpy()
    assert np.array_equal(a, b)
    z0 = hom.endpoint_grad(h, sys.c, ze[:0], g[:0]).cpu().numpy()
    assert (z0 == 0).all()


def test_homtrack_autograd_vs_finite_differences(hom):
    """torch.autograd through HomTrack: loss sum |x*|^2, gradient w.r.t. c vs central
    differences (h = 1e-6) of re-solved endpoints on 8 seeded coefficients."""
    import torch
    say("[grad autograd] c5 P=64 vs FD")
    csys, cell, z0 = W.planted_config("c5", P=64)
    h = hom.System.from_workload(csys)
    c = torch.tensor(csys.c, dtype=torch.complex128, device="cuda", requires_grad=True)
    x, st = hom.HomTrack.apply(c, h, z0, -32.0)
    ok = (st == 0)
    loss = (x.abs() ** 2)[ok].sum()
    loss.backward()
    g = c.grad.cpu().numpy()
    xe = x.detach().cpu().numpy()[ok.cpu().numpy()]
    rng = np.random.default_rng(5)
    hh = 1e-6
    for i in rng.choice(csys.M, 8, replace=False):
        fd = 0j
        for unit in (1.0, 1j):
            vals = []
            for sgn in (1, -1):
                cp = csys.c.copy()
                cp[i] += sgn * unit * hh
                vals.append(sum(np.sum(np.abs(pins.np_newton(csys, cp, x0)) ** 2) for x0 in xe))
            fd += (vals[0] - vals[1]) / (2 * hh) * (1 if unit == 1.0 else 1j)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.abs(g).max()), (i, fd, g[i])
