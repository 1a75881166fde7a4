"""GPU parity of the batched form: many systems of uneven n and support size in one launch."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import mod2pi_dist, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hom():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    import paper_2111_14317_amd as hom
    return hom


def _np(t):
    return t.cpu().numpy()


def _batch(seed=7, specs=((3, 4, 40), (6, 9, 60), (10, 12, 90), (7, 5, 0), (13, 10, 70),
                          (24, 64, 24), (9, 16, 50), (17, 8, 30))):
    """Planted-cell systems (n, m per equation, paths); (24, 64) exceeds the LDS table budget,
    the (7, 5) system has no paths."""
    rng = np.random.default_rng(seed)
    systems, starts = [], []
    for n, m, P in specs:
        sys = W.random_system(n, m, W._uniform_exps(-3, 3), "unit", 63, rng, rng, rng)
        csys, cell = W.plant_cell(sys, 63, rng, min_det=max(P, 1))
        systems.append(csys)
        starts.append(W.binomial_start_points(csys, cell, P, rng) if P else np.zeros((0, n), complex))
    n_max = max(s.n for s in systems)
    z = np.zeros((sum(len(z0) for z0 in starts), n_max), complex)
    idx = np.concatenate([np.full(len(z0), q, np.int32) for q, z0 in enumerate(starts)])
    row = 0
    for z0 in starts:
        z[row:row + len(z0), :z0.shape[1]] = z0
        row += len(z0)
    c = np.concatenate([s.c for s in systems])
    return systems, starts, z, idx, c


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_single_system_runs(hom, prec):
    say(f"[batch] 8 systems, one launch, {prec}")
    systems, starts, z, idx, c = _batch()
    precision = hom.FP64 if prec == "fp64" else hom.MIXED
    b = hom.Batch(systems)
    st = hom.track(b, c, z, -32.0, hom.default_params(precision), sys_idx=idx)
    zb, sb = _np(st.z), _np(st.status)
    row = 0
    for q, (sy, z0) in enumerate(zip(systems, starts)):
        P = len(z0)
        if P == 0:
            continue
        say(f"  system {q}: n={sy.n} m={int(sy.m[0])} P={P}")
        got = zb[row:row + P, :sy.n]
        assert np.all(zb[row:row + P, sy.n:] == 0)  # padding untouched
        h = hom.System.from_workload(sy)  # tables in LDS or, for (24, 64), in global memory
        ref = hom.track(h, sy.c, z0, -32.0, hom.default_params(precision))
        assert np.array_equal(_np(ref.status), sb[row:row + P])
        if prec == "fp64":
            assert np.array_equal(_np(ref.z), got)
        ze, _, _, ost, _ = oracle.track(sy, sy.c, z0, -32.0)
        ok = (ost == 0) & (sb[row:row + P] == 0)
        assert ok.mean() >= 0.9, (q, ok.mean())
        assert np.quantile(mod2pi_dist(got[ok], ze[ok]), 0.95) <= 1e-10
        assert oracle.residual(sy, sy.c, got[sb[row:row + P] == 0]).max() <= 1e-10
        row += P


def test_batch_rejects_bad_use(hom):
    say("[batch] argument checks")
    systems, starts, z, idx, c = _batch(specs=((3, 4, 8), (4, 5, 8)))
    b = hom.Batch(systems)
    with pytest.raises(ValueError):
        hom.track(b, c, z, -32.0)  # no sys_idx
    with pytest.raises(hom.HomError):
        hom.eval(b, c, z[:, :3], np.zeros(len(z)))  # batch handles: track only
