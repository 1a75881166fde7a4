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
        err = np.abs(got - ref) / np.abs(ref)  # per entry, relative to the entry itself
        say(f"  prec {prec}: max per-entry rel err {err.max():.3e} (|ref| >= {np.abs(ref).min():.2e})")
        assert (err <= tol).all()


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


def test_grad_c5_full_size(hom):
    """The differentiation workload at full size: 16384 paths (n = 8, 16 monomials per equation)
    tracked in FP64, loss sum |x*|^2 over the OK paths with a well-conditioned endpoint
    (kappa <= 1e4).  The gradient w.r.t. all 128 coefficients in FP64 and in the mixed form
    against the oracle's, entry by entry (1e-10 / 1e-4 relative); and central differences
    (h = 1e-6 on Re and Im, endpoints re-solved by Newton) of the loss over a seeded 4096-path
    subset on 16 seeded coefficients against the GPU gradient of that subset (1e-6 relative)."""
    say("[grad c5 full] P=16384 fp64 + mixed vs oracle; FD on 16 coefficients")
    csys, cell, z0 = W.planted_config("c5", P=16384)
    h = hom.System.from_workload(csys)
    st = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.FP64))
    z, sg = st.z.cpu().numpy(), st.status.cpu().numpy()
    G, _ = oracle.eval(csys, csys.c, z, np.zeros(len(z)))
    kappa = np.abs(np.linalg.cond(G[:, :, :csys.n], p=np.inf))
    use = (sg == 0) & (kappa <= 1e4)
    say(f"  paths used {int(use.sum())} of {len(z)}")
    assert use.sum() >= 0.999 * len(z)
    x = np.exp(z)
    g = np.where(use[:, None], 2 * x, 0)
    ref, ns = oracle.endpoint_grad(csys, csys.c, z, g)
    assert ns == 0
    for prec, tol in ((hom.FP64, 1e-10), (hom.MIXED, 1e-4)):
        got = hom.endpoint_grad(h, csys.c, z, g, precision=prec).cpu().numpy()
        err = np.abs(got - ref) / np.abs(ref)
        say(f"  prec {prec}: max per-entry rel err {err.max():.3e} over {len(ref)} coefficients")
        assert (err <= tol).all()
    rng = np.random.default_rng(16384)
    sub = rng.choice(np.nonzero(use)[0], 4096, replace=False)
    gs = hom.endpoint_grad(h, csys.c, z[sub], 2 * x[sub], precision=hom.FP64).cpu().numpy()
    hh = 1e-6
    for i in rng.choice(csys.M, 16, replace=False):
        fd = 0j
        for unit in (1.0, 1j):
            vals = []
            for sgn in (1, -1):
                cp = csys.c.copy()
                cp[i] += sgn * unit * hh
                vals.append(np.sum(np.abs(pins.np_newton_batch(csys, cp, x[sub])) ** 2))
            fd += (vals[0] - vals[1]) / (2 * hh) * (1 if unit == 1.0 else 1j)
        say(f"  coefficient {i}: FD rel err {abs(fd - gs[i]) / abs(gs[i]):.2e}")
        assert abs(fd - gs[i]) <= 1e-6 * abs(gs[i]), (i, fd, gs[i])
