"""hom_track_noalloc (the tracker on the library's static device scratch, no allocation) against
hom_track: bitwise the same endpoints, statuses and counters, on two calls in a row (the second
with fewer paths), for a system staged in LDS and one whose tables stay in global memory (its
coefficient table then lives in the scratch), in both precisions."""
import numpy as np
import pytest

import workloads as W
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hom():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    import paper_2111_14317_amd as hom
    return hom


def _np(t):
    return t.cpu().numpy()


def _global_table_system():
    rng = np.random.default_rng(13)
    sy = W.random_system(24, 64, W._uniform_exps(-3, 3), "unit", 63, rng, rng, rng)
    csys, cell = W.plant_cell(sy, 63, rng, min_det=48)
    return csys, W.binomial_start_points(csys, cell, 48, rng)


@pytest.mark.parametrize("which", ["lds-tables", "global-tables"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_equals_track(hom, which, prec):
    import torch
    if which == "lds-tables":
        csys, cell, z0 = W.planted_config("c5", P=1024)
        sizes = (1024, 300)
    else:
        csys, z0 = _global_table_system()
        sizes = (48, 17)
    say(f"[noalloc] {which} {prec} n={csys.n} calls of {sizes} paths")
    precision = hom.FP64 if prec == "fp64" else hom.MIXED
    h = hom.System.from_workload(csys)
    c = torch.tensor(csys.c, dtype=torch.complex128, device="cuda")
    for P in sizes:
        ref = hom.track(h, c, z0[:P], -32.0,
                        hom.default_params(precision, flags=hom.TRACK_SERIAL))
        got = hom.track_noalloc(h, c, hom.new_state(z0[:P], -32.0), hom.default_params(precision))
        torch.cuda.synchronize()
        for f in ("z", "s", "ds", "status", "counters"):
            assert np.array_equal(_np(getattr(got, f)), _np(getattr(ref, f))), (P, f)
        ok = _np(got.status) == 0
        say(f"  P={P}: {int(ok.sum())} OK")
        assert ok.mean() >= 0.9


@pytest.mark.parametrize("prec,pred", [("mixed", "rk4"), ("fp64", "hermite")])
def test_noalloc_predictors(hom, prec, pred):
    """The same with the Runge-Kutta (mixed form) and cubic Hermite (FP64 form) predictors."""
    import torch
    csys, cell, z0 = W.planted_config("c5", P=512)
    say(f"[noalloc] {prec} {pred} n={csys.n}")
    precision = hom.FP64 if prec == "fp64" else hom.MIXED
    predictor = hom.PREDICT_RK4 if pred == "rk4" else hom.PREDICT_HERMITE
    h = hom.System.from_workload(csys)
    c = torch.tensor(csys.c, dtype=torch.complex128, device="cuda")
    for P in (512, 130):
        ref = hom.track(h, c, z0[:P], -32.0, hom.default_params(
            precision, flags=hom.TRACK_SERIAL, predictor=predictor))
        got = hom.track_noalloc(h, c, hom.new_state(z0[:P], -32.0),
                                hom.default_params(precision, predictor=predictor))
        torch.cuda.synchronize()
        for f in ("z", "s", "ds", "status", "counters"):
            assert np.array_equal(_np(getattr(got, f)), _np(getattr(ref, f))), (P, f)
        assert (_np(got.status) == 0).mean() >= 0.9


def test_noalloc_rejects_what_it_cannot_hold(hom):
    """A coefficient table beyond the scratch (one equation with 6000 monomials at n = 32) and a
    batch handle are refused with a clear error before any launch."""
    say("[noalloc] refusals")
    import torch
    rng = np.random.default_rng(3)
    n = 32
    m = np.ones(n, np.int32)
    m[0] = 6000
    M = int(m.sum())
    A = rng.integers(-2, 3, size=(M, n)).astype(np.int8)
    w = rng.integers(0, 8, size=M).astype(np.float64)
    h = hom.System(n, m, A, w, valu=True)
    c = torch.ones(M, dtype=torch.complex128, device="cuda")
    st = hom.new_state(np.zeros((4, n), complex), -1.0)
    with pytest.raises(hom.HomError, match="exceeds the static scratch"):
        hom.track_noalloc(h, c, st)
    csys, cell, z0 = W.planted_config("c5", P=8)
    b = hom.Batch([csys])
    with pytest.raises(hom.HomError, match="batch handles"):
        hom.track_noalloc(b, torch.tensor(csys.c, dtype=torch.complex128, device="cuda"),
                          hom.new_state(z0, -32.0))
