"""Pins of the oracle's predictor-corrector tracker and of the start systems it is given."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import pins
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _mod2pi_key(z, digits=6):
    return {tuple(v) for v in np.round(np.c_[z.real, np.mod(z.imag + 1e-7, 2 * np.pi)] * 10 ** digits)}


def test_golden_binomial_roots():
    """Tracking the hand-worked binomial homotopy from s0 = -32 ends at the 6 closed-form roots."""
    g = json.load(open(os.path.join(GOLD, "binomial_2x2.json")))
    d = g["system"]
    sys = W.System(d["n"], np.array(d["m"]), np.array(d["A"]), np.array(d["w"], float),
                   np.array([complex(a, b) for a, b in d["c"]]))
    want = np.array([[1j * np.pi * float(Fraction(v)) for v in r] for r in g["roots_im_over_pi"]])
    # start points on the closed-form paths z(s) = z(0) - s dE
    dE = np.array([float(Fraction(v)) for v in g["euler_everywhere"]])
    s0 = -32.0
    z0 = want + s0 * dE[None, :]
    ze, se, _, st, cnt = oracle.track(sys, sys.c, z0, s0)
    assert (st == oracle.OK).all() and (se == 0).all()
    dz = np.abs(np.exp(ze) - np.exp(want)).max()
    assert dz < 1e-13


def test_binomial_path_closed_form():
    """Raw-lifted binomial systems: every endpoint is D^{-1}(log beta + 2 pi i k)."""
    rng = np.random.default_rng(12)
    n = 4
    for _ in range(3):
        A = rng.integers(-2, 3, size=(2 * n, n))
        D = A[1::2] - A[0::2]
        det = W.int_det(D)
        if det == 0:
            continue
        w = rng.integers(0, 10, size=2 * n).astype(float)
        c = np.exp(2j * np.pi * rng.random(2 * n))
        sys = W.System(n, np.full(n, 2), A, w, c)
        beta = -c[0::2] / c[1::2]
        delta = w[1::2] - w[0::2]
        z_end = W.binomial_roots(D, beta, min(abs(det), 16), rng)
        s0 = -10.0
        z0 = z_end - s0 * np.linalg.solve(D.astype(float), delta)[None, :]
        # these straight paths may run far from |x| = 1: lift the divergence guard
        ze, se, _, st, _ = oracle.track(sys, sys.c, z0, s0, oracle.TrackParams(div_re=1e4))
        assert (st == oracle.OK).all()
        err = np.abs(ze.real - z_end.real) + np.abs(np.angle(np.exp(1j * (ze.imag - z_end.imag))))
        assert err.max() <= 1e-11 * np.linalg.cond(D.astype(float))


def test_mixed_volume_and_c1_cells():
    """Sum of |det| over brute-force cells = mixed volume by Minkowski volumes (Bernshtein)."""
    base, cells = W.c1_cells()
    mv = pins.mixed_volume(base)
    assert sum(info["det"] for _, info, _ in cells) == mv
    for csys, info, z0 in cells:
        assert len(z0) == info["det"] and len(_mod2pi_key(z0)) == info["det"]


def test_c1_all_paths():
    """All mixed-volume paths of c1 end at distinct roots with residual <= 1e-10."""
    base, cells = W.c1_cells()
    ends = []
    for csys, info, z0 in cells:
        ze, se, _, st, cnt = oracle.track(csys, csys.c, z0, -32.0)
        assert (st == oracle.OK).all()
        ends.append(ze)
    ze = np.concatenate(ends)
    assert len(_mod2pi_key(ze)) == pins.mixed_volume(base) == len(ze)
    assert oracle.residual(base, base.c, ze).max() <= 1e-10
    # the roots are roots of F in affine coordinates too (numpy definition)
    for x in np.exp(ze[:10]):
        F, _ = pins.np_F_J(base, base.c, x)
        assert np.abs(F).max() < 1e-12


def test_random_systems_mv_count():
    """Small random systems: tracked endpoints = mixed volume, all distinct (property test)."""
    for seed in range(4):
        rng = np.random.default_rng(100 + seed)
        n = 2 + seed % 2
        sys = W.random_system(n, 3, W._uniform_exps(-2, 2), "unit", 15, rng, rng, rng)
        try:
            sys, cells = W.generic_lifting_cells(sys, rng, 15)
        except RuntimeError:
            continue
        ends = []
        for info in cells:
            csys = W.cell_homotopy(sys, info)
            z0 = W.binomial_start_points(csys, info["cell"], info["det"], rng)
            ze, _, _, st, _ = oracle.track(csys, csys.c, z0, -32.0)
            assert (st == oracle.OK).all()
            ends.append(ze)
        ze = np.concatenate(ends)
        assert len(ze) == pins.mixed_volume(sys) == len(_mod2pi_key(ze))


def test_endpoint_set_independent_of_lifting():
    """A different generic lifting gives the same endpoint set."""
    base, cells = W.c1_cells()
    rng = np.random.default_rng(77)
    sys2, cells2 = W.generic_lifting_cells(base.with_lifting(rng.integers(0, 32, base.M).astype(float)), rng, 31)
    sets = []
    for s_, cl in ((base, None), (sys2, cells2)):
        ends = []
        for info in (cl if cl is not None else [i for _, i, _ in cells]):
            csys = W.cell_homotopy(s_, info)
            z0 = W.binomial_start_points(csys, info["cell"], info["det"], rng)
            ze, _, _, st, _ = oracle.track(csys, csys.c, z0, -32.0)
            ends.append(ze)
        sets.append(_mod2pi_key(np.concatenate(ends), digits=5))
    assert sets[0] == sets[1]


def test_step_size_independence():
    csys, cell, z0 = W.planted_config("c5", P=64)
    a = oracle.track(csys, csys.c, z0, -32.0, oracle.TrackParams(ds0=0.05, ds_max=0.5))
    b = oracle.track(csys, csys.c, z0, -32.0, oracle.TrackParams(ds0=0.01, ds_max=0.25))
    ok = (a[3] == 0) & (b[3] == 0)
    assert ok.mean() > 0.95
    assert _mod2pi_key(a[0][ok], 5) == _mod2pi_key(b[0][ok], 5)


def test_resume_bitwise():
    """Calling with max_steps = k repeatedly equals one long call (z, s bitwise)."""
    csys, cell, z0 = W.planted_config("c5", P=32)
    full = oracle.track(csys, csys.c, z0, -32.0)
    p = oracle.TrackParams(max_steps=7)
    z, s, ds, st = z0.copy(), np.full(32, -32.0), None, None
    for _ in range(1000):
        z, s, ds, st, cnt = oracle.track(csys, csys.c, z, s, p, status=st, ds=ds)
        if not (st == oracle.RUNNING).any():
            break
    assert np.array_equal(z, full[0]) and np.array_equal(s, full[1])
    assert np.array_equal(st, full[3])


def test_failure_modes_forced():
    """Host-forced outcomes: a start point far off the path fails polishing; a NaN input is
    NONFINITE; a zero step budget leaves the path RUNNING at its polished start."""
    csys, cell, z0 = W.planted_config("c5", P=8)
    bad = z0.copy()
    bad[0] += 0.7
    bad[1, 0] = np.nan
    z, s, ds, st, cnt = oracle.track(csys, csys.c, bad, -32.0)
    assert st[0] in (oracle.POLISH_FAIL, oracle.OK)
    assert st[1] in (oracle.NONFINITE, oracle.SINGULAR)
    assert (st[2:] == oracle.OK).all()
    z, s, ds, st, cnt = oracle.track(csys, csys.c, z0, -32.0, oracle.TrackParams(max_steps=0))
    assert (st == oracle.RUNNING).all() and (s == -32.0).all()


# ---- the cubic Hermite predictor (Sec. 2.3: predictors built on the Euler direction) -----------
def test_hermite_predictor_matches_scipy():
    """The tracker's predictor against scipy's CubicHermiteSpline (extrapolating past s1), real
    and imaginary parts separately."""
    from scipy.interpolate import CubicHermiteSpline
    rng = np.random.default_rng(3)
    P, n = 50, 4
    s0 = rng.uniform(-10, -1, P)
    s1 = s0 + rng.uniform(0.01, 0.7, P)
    s = s1 + (s1 - s0) * rng.uniform(0.0, 3.0, P)
    z0, z1, e0, e1 = (rng.normal(size=(P, n)) + 1j * rng.normal(size=(P, n)) for _ in range(4))
    got = oracle.hermite(s0, z0, e0, s1, z1, e1, s)
    for p in range(P):
        for part in (np.real, np.imag):
            sp = CubicHermiteSpline([s0[p], s1[p]], np.stack([part(z0[p]), part(z1[p])]),
                                    np.stack([part(e0[p]), part(e1[p])]), extrapolate=True)
            np.testing.assert_allclose(part(got[p]), sp(s[p]), rtol=1e-12, atol=1e-12)


def test_hermite_predictor_exact_on_cubics():
    """A cubic path is reproduced exactly from two points and their slopes, at any s."""
    rng = np.random.default_rng(4)
    P, n = 40, 3
    a = [rng.normal(size=(P, n)) + 1j * rng.normal(size=(P, n)) for _ in range(4)]

    def z(s):
        return a[0] + a[1] * s[:, None] + a[2] * s[:, None] ** 2 + a[3] * s[:, None] ** 3

    def dz(s):
        return a[1] + 2 * a[2] * s[:, None] + 3 * a[3] * s[:, None] ** 2

    s0 = rng.uniform(-3, -1, P)
    s1 = s0 + rng.uniform(0.1, 0.5, P)
    s = s1 + rng.uniform(0.0, 1.0, P)
    got = oracle.hermite(s0, z(s0), dz(s0), s1, z(s1), dz(s1), s)
    np.testing.assert_allclose(got, z(s), rtol=1e-10, atol=1e-10)


def test_hermite_tracker_same_roots():
    """Tracking with the Hermite predictor ends every path on the Euler predictor's endpoint
    (path by path; the c1 cells and 300 n = 8 planted-cell paths), with fewer eval+solves."""
    base, cells = W.c1_cells()
    ev = {0: 0, 1: 0}
    for csys, info, z0 in cells:
        res = {}
        for pred in (0, 1):
            ze, _, _, st, cnt = oracle.track(csys, csys.c, z0, -32.0, oracle.TrackParams(predictor=pred))
            assert (st == oracle.OK).all()
            res[pred] = ze
            ev[pred] += int(cnt[:, 3].sum())
        d = np.abs(res[0] - res[1])
        d = np.maximum(np.abs(d.real), np.abs(np.angle(np.exp(1j * (res[0].imag - res[1].imag)))))
        assert d.max() <= 1e-12
    csys, cell, z0 = W.planted_config("c5", P=300)
    a = oracle.track(csys, csys.c, z0, -32.0, oracle.TrackParams(predictor=0))
    b = oracle.track(csys, csys.c, z0, -32.0, oracle.TrackParams(predictor=1))
    assert (a[3] == 0).all() and (b[3] == 0).all()
    dre = np.abs(a[0].real - b[0].real).max(1)
    dim = np.abs(np.angle(np.exp(1j * (a[0].imag - b[0].imag)))).max(1)
    assert np.maximum(dre, dim).max() <= 1e-12
    assert b[4][:, 3].sum() < a[4][:, 3].sum() and ev[1] < ev[0]


# ---- the Runge-Kutta predictor (Sec. 2.3: Runge-Kutta methods on the Euler direction) ---------
def _trinomial():
    """n = 1: c0 + c1 x t^{w1} + c2 x^2 t^{w2}; its paths have the closed form of the quadratic
    formula, z(s) = log x(s)."""
    c = np.array([1.0 + 0.0j, -3.0 + 0.5j, 2.0 - 0.25j])
    w = np.array([0.0, 1.0, 3.0])
    sys_ = W.System(1, np.array([3], np.int32), np.array([[0], [1], [2]], np.int8), w, c)

    def z_exact(s, near):
        t = np.exp(s)
        a, b, cc = c[2] * t ** w[2], c[1] * t ** w[1], c[0] * t ** w[0]
        d = np.sqrt(b * b - 4 * a * cc + 0j)
        roots = np.log(np.array([(-b + d) / (2 * a), (-b - d) / (2 * a)]))
        roots = roots.real + 1j * (near.imag + np.angle(np.exp(1j * (roots.imag - near.imag))))
        return roots[np.argmin(np.abs(roots - near))]
    return sys_, z_exact


def _order(err):
    return np.log2(err[:-1] / err[1:])


def test_rk4_predictor_fourth_order():
    """The predictor's error against the closed-form path shrinks like h^5 (local error of a
    fourth-order method): halving h divides it by about 32; a plausible mistake in the weights
    (equal weights) or the stage points (all at s_a + h/2) loses that order."""
    sys_, z_exact = _trinomial()
    sa = -1.0
    z0 = np.array([z_exact(sa, 0.0 + 0.0j)])  # the path through the root nearest z = 0
    hs = np.array([0.2, 0.1, 0.05, 0.025])
    got = np.array([oracle.rk4_predict(sys_, sys_.c, z0[None, :], sa, h)[0, 0] for h in hs])
    ref = np.array([z_exact(sa + h, z0[0]) for h in hs])
    err = np.abs(got - ref)
    order = _order(err)
    assert (order > 4.5).all() and (order < 5.6).all(), order

    def de(z, s):
        return oracle.step(sys_, sys_.c, np.array([[z]]), np.array([s]))[0][0, 0]

    def bad_rk(h, weights=(1, 2, 2, 1), mid=(0.5, 0.5, 1.0)):
        z = z0[0]
        k1 = de(z, sa)
        k2 = de(z + mid[0] * h * k1, sa + mid[0] * h)
        k3 = de(z + mid[1] * h * k2, sa + mid[1] * h)
        k4 = de(z + mid[2] * h * k3, sa + mid[2] * h)
        return z + h / sum(weights) * (weights[0] * k1 + weights[1] * k2 + weights[2] * k3 + weights[3] * k4)
    good = np.abs(np.array([bad_rk(h) for h in hs]) - ref)
    np.testing.assert_allclose(good, err, rtol=1e-6, atol=1e-15)  # the same scheme, by hand
    for kw in ({"weights": (1, 1, 1, 1)}, {"mid": (0.5, 0.5, 0.5)}):
        e = np.abs(np.array([bad_rk(h, **kw) for h in hs]) - ref)
        assert _order(e).min() < 4.0


def test_rk4_tracker_same_roots_fewer_steps():
    """Tracking with the Runge-Kutta predictor ends every path on the Euler predictor's endpoint
    (path by path: the c1 cells and 300 n = 8 planted-cell paths), in fewer accepted steps."""
    base, cells = W.c1_cells()
    steps = {0: 0, 2: 0}
    for csys, info, z0 in cells:
        res = {}
        for pred in (0, 2):
            ze, _, _, st, cnt = oracle.track(csys, csys.c, z0, -32.0, oracle.TrackParams(predictor=pred))
            assert (st == oracle.OK).all()
            res[pred] = ze
            steps[pred] += int(cnt[:, 0].sum())
        dre = np.abs(res[0].real - res[2].real)
        dim = np.abs(np.angle(np.exp(1j * (res[0].imag - res[2].imag))))
        assert np.maximum(dre, dim).max() <= 1e-12
    csys, cell, z0 = W.planted_config("c5", P=300)
    a = oracle.track(csys, csys.c, z0, -32.0, oracle.TrackParams(predictor=0))
    b = oracle.track(csys, csys.c, z0, -32.0, oracle.TrackParams(predictor=2))
    assert (a[3] == 0).all() and (b[3] == 0).all()
    dre = np.abs(a[0].real - b[0].real).max(1)
    dim = np.abs(np.angle(np.exp(1j * (a[0].imag - b[0].imag)))).max(1)
    assert np.maximum(dre, dim).max() <= 1e-12
    assert b[4][:, 0].sum() < a[4][:, 0].sum() and steps[2] < steps[0]
