"""GPU parity of the dense-support paths: the matrix-core engines (FP64 MFMA, BF16x3 MFMA) and
the vector-unit kernels on global-memory tables, at the n = 32, 128-monomials-per-equation shape
and on ragged shapes (n not a multiple of 16, m_k not a multiple of 32, P not a multiple of 16)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import check_dirs as _check_dirs, dir_err as _dir_err, cond_inf, eval_err, eval_err_fp32, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hom():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    import paper_2111_14317_amd as hom
    return hom


def _np(t):
    return t.cpu().numpy()


def _ragged(seed=11, n=20, lift=12):
    rng = np.random.default_rng(seed)
    m = rng.integers(30, 71, size=n)  # padded to 32 / 64 / 96 per equation
    sys = W.random_system(n, m, W._uniform_exps(-3, 3), "unit", lift, rng, rng, rng)
    z, s = W.random_points(n, 37, rng)
    return sys, z, s


ENGINES = [("mfma-fp64", 0, 1e-12), ("mfma-bf16x3", 4, 1e-5), ("valu-fp64", 8, 1e-12),
           ("valu-fp32", 12, 1e-5)]


@pytest.mark.parametrize("name,flags,tol", ENGINES)
def test_dense_eval_c3_shape(hom, name, flags, tol):
    """n = 32, 128 monomials per equation (exponents in [-4, 4], 30% zeros, Gaussian c, lifting
    U{0..255}), 200 points: every engine against the FP64 oracle."""
    say(f"[dense eval c3] {name} P=200")
    sys, z, s = W.config_system("c3", P=200)
    h = hom.System.from_workload(sys)
    G, L = hom.eval(h, sys.c, z, s, flags=flags)
    Go, Lo, den = oracle.eval(sys, sys.c, z, s, with_den=True)
    G, L = _np(G), _np(L)
    metric = eval_err if tol < 1e-6 else eval_err_fp32
    err = metric(G, L, Go, Lo, den)
    say(f"  max scaled err {err.max():.3e}  median {np.median(err):.3e}  "
        f"shift |L - Lo| <= {np.abs(L - Lo).max():.3e}")
    assert np.isfinite(G).all()
    assert err.max() <= tol
    if flags & 8:
        np.testing.assert_allclose(L, Lo, rtol=0, atol=1e-12 * (1 + np.abs(Lo).max()))
    else:  # the matrix-core shift is the row maximum to within about 0.1
        assert np.abs(L - Lo).max() <= 0.25


def test_dense_bf16_rational_liftings(hom):
    """The BF16x3 engine stages the liftings as float only when every one is exactly a float; with
    liftings k + 1/3 (not floats) it reads the FP64 liftings instead and stays within its bound."""
    import dataclasses
    say("[dense eval bf16x3] liftings k + 1/3, P=200")
    sys0, z, s = W.config_system("c3", P=200)
    sys = dataclasses.replace(sys0, w=sys0.w + 1.0 / 3.0)
    assert np.any(sys.w.astype(np.float32).astype(np.float64) != sys.w)
    h = hom.System.from_workload(sys)
    G, L = hom.eval(h, sys.c, z, s, flags=4)
    Go, Lo, den = oracle.eval(sys, sys.c, z, s, with_den=True)
    err = eval_err_fp32(_np(G), _np(L), Go, Lo, den)
    say(f"  max scaled err {err.max():.3e}")
    assert np.isfinite(_np(G)).all() and err.max() <= 1e-5


@pytest.mark.parametrize("name,flags,tol", ENGINES)
def test_dense_eval_ragged(hom, name, flags, tol):
    say(f"[dense eval ragged] {name} n=20 m_k in [30,70] P=37")
    sys, z, s = _ragged()
    h = hom.System.from_workload(sys)
    G, L = hom.eval(h, sys.c, z, s, flags=flags)
    Go, Lo, den = oracle.eval(sys, sys.c, z, s, with_den=True)
    metric = eval_err if tol < 1e-6 else eval_err_fp32
    err = metric(_np(G), _np(L), Go, Lo, den)
    say(f"  max scaled err {err.max():.3e}")
    assert err.max() <= tol
    # P = 1 and P = 0
    G1, L1 = hom.eval(h, sys.c, z[:1], s[:1], flags=flags)
    assert metric(_np(G1), _np(L1), Go[:1], Lo[:1], den[:1]).max() <= tol
    G0, _ = hom.eval(h, sys.c, z[:0], s[:0], flags=flags)
    assert G0.shape[0] == 0


def test_dense_eval_flags(hom):
    """HOM_UNSCALED and HOM_AFFINE on the matrix-core FP64 engine (small liftings, so t^w stays in
    range)."""
    say("[dense eval flags] ragged n=20 unscaled/affine")
    sys, z, s = _ragged(lift=3)
    h = hom.System.from_workload(sys)
    Go, _ = oracle.eval(sys, sys.c, z, s, scaled=False)
    Gu, Lu = hom.eval(h, sys.c, z, s, flags=hom.UNSCALED)
    assert np.all(_np(Lu) == 0)
    _, _, den = oracle.eval(sys, sys.c, z, s, with_den=True, scaled=False)
    assert (np.abs(_np(Gu) - Go) / np.where(den > 0, den, 1)).max() <= 1e-12
    Ga, _ = hom.eval(h, sys.c, z, s, flags=hom.UNSCALED | hom.AFFINE)
    Ga, n = _np(Ga), sys.n
    ref = Go.copy()
    ref[:, :, :n] *= np.exp(-z)[:, None, :]
    ref[:, :, n] *= np.exp(-s)[:, None]
    scale = den.copy()
    scale[:, :, :n] *= np.abs(np.exp(-z))[:, None, :]
    scale[:, :, n] *= np.exp(-s)[:, None]
    assert (np.abs(Ga - ref) / np.where(scale > 0, scale, 1)).max() <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_dense_step_c3_shape(hom, prec):
    say(f"[dense step c3] {prec} P=200")
    sys, z, s = W.config_system("c3", P=200)
    h = hom.System.from_workload(sys)
    precision = hom.FP64 if prec == "fp64" else hom.MIXED
    dE, dN, st = hom.step(h, sys.c, z, s, precision=precision)
    oE, oN, ost, ratio = oracle.step(sys, sys.c, z, s)
    kappa = cond_inf(sys, sys.c, z, s)
    _check_dirs(_np(dE), _np(dN), oE, oN, ost, kappa, prec == "mixed", sys.n,
                min_well=10 if prec == "fp64" else 0)
    if prec == "fp64":
        assert np.array_equal(_np(st) == 0, (ost == 0) & (ratio >= 1e-14))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_dense_step_well_conditioned(hom, prec):
    """A dense-support handle (40 monomials per equation: matrix-core tables) at n = 8, where most
    random points are well conditioned: the mixed step is within 1e-5 of the oracle on at least
    100 points with kappa <= 1e2 (FP64: 1e-12 where kappa <= 1e3), and within the LU bound on
    every point."""
    say(f"[dense step well-conditioned] n=8 m=40 P=512 {prec}")
    rng = np.random.default_rng(31)
    sys = W.random_system(8, 40, W._uniform_exps(-2, 2), "unit", 15, rng, rng, rng)
    z, s = W.random_points(8, 512, rng, s_lo=-2.0)
    h = hom.System.from_workload(sys)
    precision = hom.FP64 if prec == "fp64" else hom.MIXED
    dE, dN, st = hom.step(h, sys.c, z, s, precision=precision)
    oE, oN, ost, _ = oracle.step(sys, sys.c, z, s)
    kappa = cond_inf(sys, sys.c, z, s)
    _check_dirs(_np(dE), _np(dN), oE, oN, ost, kappa, prec == "mixed", sys.n, min_well=100)


def test_dense_step_ragged_and_valu_handle(hom):
    """Ragged dense system, both precisions; a handle without matrix-core tables (vector units,
    global-memory tables) gives the same directions."""
    say("[dense step ragged] n=20 P=37")
    sys, z, s = _ragged()
    oE, oN, ost, _ = oracle.step(sys, sys.c, z, s)
    kappa = cond_inf(sys, sys.c, z, s)
    for valu in (False, True):
        h = hom.System.from_workload(sys, valu=valu)
        for prec in (hom.FP64, hom.MIXED):
            dE, dN, st = hom.step(h, sys.c, z, s, precision=prec)
            _check_dirs(_np(dE), _np(dN), oE, oN, ost, kappa, prec == hom.MIXED, sys.n,
                        f"valu={valu} prec={prec}")


def test_step_mixed_redo_near_singular(hom):
    """Mixed-form step at points whose FP32 pivot ratio is below the redo threshold: equation 1 is
    equation 0 with its coefficients perturbed by 1e-6, so every Jacobian has two nearly equal rows
    (pivot ratio 1e-9 .. 3e-6, condition 1e7 .. 3e10).  The FP32 LU alone would lose every digit
    there; the FP64 redo must give directions within kappa * 1e-13 of the oracle, on both the
    matrix-core handle and the vector-unit handle."""
    say("[mixed redo] n=20 m=64 P=40, near-duplicate equations")
    rng = np.random.default_rng(23)
    n = 20
    sy = W.random_system(n, 64, W._uniform_exps(-3, 3), "unit", 12, rng, rng, rng)
    A, w, c = sy.A.copy(), sy.w.copy(), sy.c.copy()
    e0, e1 = sy.equation(0), sy.equation(1)
    A[e1], w[e1] = A[e0], w[e0]
    c[e1] = c[e0] * (1 + 1e-6 * (rng.standard_normal(64) + 1j * rng.standard_normal(64)))
    ns = W.System(n, sy.m.copy(), A, w, c)
    z, s = W.random_points(n, 40, rng)
    oE, oN, ost, ratio = oracle.step(ns, ns.c, z, s)
    kappa = np.abs(cond_inf(ns, ns.c, z, s))
    assert ratio.max() < 1e-4 and (ost == 0).all() and kappa.min() > 1e6
    for valu in (False, True):
        h = hom.System.from_workload(ns, valu=valu)
        dE, dN, st = hom.step(h, ns.c, z, s, precision=hom.MIXED)
        e = np.maximum(_dir_err(_np(dE), oE), _dir_err(_np(dN), oN))
        say(f"  valu={valu}: max err/kappa {(e / kappa).max():.3e}")
        assert (_np(st) == 0).all()
        assert (e <= kappa * 1e-13).all()


def test_dense_full_size_sampled(hom):
    """The full 262144-point n = 32 workload in both matrix-core engines; a seeded sample of 128
    points against the oracle (G of the whole batch is 4.6 GB on the device)."""
    import torch
    say("[dense full] c3 P=262144 sampled")
    sys, z, s = W.config_system("c3")
    h = hom.System.from_workload(sys)
    idx = np.random.default_rng(5).choice(len(s), 128, replace=False)
    Go, Lo, den = oracle.eval(sys, sys.c, z[idx], s[idx], with_den=True)
    ti = torch.as_tensor(idx, device="cuda")
    for flags, metric, tol in ((0, eval_err, 1e-12), (hom.EVAL_FP32, eval_err_fp32, 1e-5)):
        G, L = hom.eval(h, sys.c, z, s, flags=flags)
        Gs, Ls = _np(G[ti]), _np(L[ti])
        del G, L
        torch.cuda.empty_cache()
        err = metric(Gs, Ls, Go, Lo, den)
        say(f"  flags {flags}: max scaled err {err.max():.3e}")
        assert err.max() <= tol
    oE, oN, ost, _ = oracle.step(sys, sys.c, z[idx], s[idx])
    kappa = cond_inf(sys, sys.c, z[idx], s[idx])
    for prec in (hom.FP64, hom.MIXED):
        dE, dN, st = hom.step(h, sys.c, z, s, precision=prec)
        _check_dirs(_np(dE)[idx], _np(dN)[idx], oE, oN, ost, kappa, prec == hom.MIXED, sys.n,
                    f"prec={prec}")


def test_global_table_track(hom):
    """A system whose tables exceed the LDS budget (n = 24, 64 monomials per equation) tracked on a
    single-system handle: the same endpoints as its run inside a batch handle, roots of the
    target."""
    say("[global-table track] n=24 m=64 P=24")
    rng = np.random.default_rng(13)
    sy = W.random_system(24, 64, W._uniform_exps(-3, 3), "unit", 63, rng, rng, rng)
    csys, cell = W.plant_cell(sy, 63, rng, min_det=24)
    z0 = W.binomial_start_points(csys, cell, 24, rng)
    h = hom.System.from_workload(csys)
    a = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.FP64))
    b = hom.track(hom.Batch([csys]), csys.c, z0, -32.0, hom.default_params(hom.FP64),
                  sys_idx=np.zeros(len(z0), np.int32))
    assert np.array_equal(_np(a.status), _np(b.status))
    assert np.array_equal(_np(a.z), _np(b.z))
    ok = _np(a.status) == 0
    assert ok.mean() >= 0.9
    assert oracle.residual(csys, csys.c, _np(a.z)[ok]).max() <= 1e-10


@pytest.mark.parametrize("which", ["valu-n3", "bf16x3-n20"])
def test_eval_flags_fp32(hom, which):
    """HOM_UNSCALED and HOM_AFFINE with the FP32 evaluation: the vector-unit kernel (c1 shape, n = 3)
    and the BF16x3 matrix-core engine (ragged n = 20, liftings up to 3), componentwise against the
    oracle's unscaled values at the FP32 tolerance (1e-5 of each entry's term mass, floored at
    1e-30 of the row's total as in the scaled comparison)."""
    say(f"[eval flags fp32] {which}")
    if which == "valu-n3":
        sys, z, s = W.config_system("c1", P=257)
    else:
        sys, z, s = _ragged(lift=3)
    h = hom.System.from_workload(sys)
    n = sys.n
    Go, _ = oracle.eval(sys, sys.c, z, s, scaled=False)
    _, _, den = oracle.eval(sys, sys.c, z, s, with_den=True, scaled=False)
    for affine in (False, True):
        flags = hom.EVAL_FP32 | hom.UNSCALED | (hom.AFFINE if affine else 0)
        G, L = hom.eval(h, sys.c, z, s, flags=flags)
        assert np.all(_np(L) == 0)
        ref, scale = Go.copy(), den.copy()
        if affine:
            ref[:, :, :n] *= np.exp(-z)[:, None, :]
            ref[:, :, n] *= np.exp(-s)[:, None]
            scale[:, :, :n] *= np.abs(np.exp(-z))[:, None, :]
            scale[:, :, n] *= np.exp(-s)[:, None]
        scale = np.maximum(scale, 1e-30 * scale[:, :, -1:])
        err = np.abs(_np(G) - ref) / np.where(scale > 0, scale, 1.0)
        say(f"  affine={affine}: max {err.max():.2e}")
        assert err.max() <= 1e-5
