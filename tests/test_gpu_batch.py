"""GPU parity of the batched form: many systems of uneven n and support size in one launch."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import (check_fp64_per_path, check_mixed_set, distinct_count, mod2pi_dist, say,
                      status_hist)

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
        if prec == "fp64":  # path by path: same statuses, <= 1e-12 where kappa <= 1e4
            check_fp64_per_path(sy, got, sb[row:row + P], ze, ost, f"system {q}",
                                max_excluded=0.05)
        else:  # as a set, at most one path of the system not OK
            check_mixed_set(sy, got, sb[row:row + P], ze, ost, f"system {q}",
                            min_ok=(P - 1) / P, max_swaps=0.0)
        row += P


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_rk4_equals_single_system_runs(hom, prec):
    """The Runge-Kutta predictor in the batched form: statuses equal to single-system runs with the
    same predictor (FP64: endpoints bitwise, and path by path against the oracle's tracker with
    that predictor)."""
    say(f"[batch rk4] 8 systems, one launch, {prec}")
    systems, starts, z, idx, c = _batch()
    precision = hom.FP64 if prec == "fp64" else hom.MIXED
    params = hom.default_params(precision, predictor=hom.PREDICT_RK4)
    b = hom.Batch(systems)
    st = hom.track(b, c, z, -32.0, params, sys_idx=idx)
    zb, sb = _np(st.z), _np(st.status)
    row = 0
    for q, (sy, z0) in enumerate(zip(systems, starts)):
        P = len(z0)
        if P == 0:
            continue
        got = zb[row:row + P, :sy.n]
        h = hom.System.from_workload(sy)
        ref = hom.track(h, sy.c, z0, -32.0, params)
        assert np.array_equal(_np(ref.status), sb[row:row + P])
        if prec == "fp64":
            assert np.array_equal(_np(ref.z), got)
            ze, _, _, ost, _ = oracle.track(sy, sy.c, z0, -32.0, oracle.TrackParams(predictor=2))
            check_fp64_per_path(sy, got, sb[row:row + P], ze, ost, f"system {q}",
                                max_excluded=0.05)
        row += P


def test_batch_rejects_bad_use(hom):
    say("[batch] argument checks")
    systems, starts, z, idx, c = _batch(specs=((3, 4, 8), (4, 5, 8)))
    b = hom.Batch(systems)
    with pytest.raises(ValueError):
        hom.track(b, c, z, -32.0)  # no sys_idx
    with pytest.raises(hom.HomError):
        hom.eval(b, c, z[:, :3], np.zeros(len(z)))  # batch handles: track only


def _state(hom, torch, z, P):
    return hom.TrackState(torch.tensor(z, dtype=torch.complex128, device="cuda"),
                          torch.full((P,), -32.0, dtype=torch.float64, device="cuda"),
                          torch.zeros(P, dtype=torch.float64, device="cuda"),
                          torch.full((P,), hom.PATH_START, dtype=torch.int32, device="cuda"),
                          torch.zeros((P, 4), dtype=torch.int32, device="cuda"))


def test_batch_tile_independent(hom):
    """The work-item size changes only the schedule: FP64 endpoints are bitwise equal for every
    tile the autotuner may pick."""
    say("[batch] tiles 1, 2, 8, 16 vs default")
    systems, starts, z, idx, c = _batch(seed=8, specs=((5, 6, 60), (12, 9, 80), (24, 40, 30)))
    b = hom.Batch(systems)
    ref = hom.track(b, c, z, -32.0, hom.default_params(hom.FP64), sys_idx=idx)
    for t in (1, 2, 8, 16):
        st = hom.track(b, c, z, -32.0, hom.default_params(hom.FP64, tile=t), sys_idx=idx)
        assert np.array_equal(_np(st.z), _np(ref.z)), t
        assert np.array_equal(_np(st.status), _np(ref.status)), t


def test_autotune_picks_and_caches(hom, tmp_path):
    from paper_2111_14317_amd import autotune
    say("[batch] autotune, 3 systems")
    systems, starts, z, idx, c = _batch(seed=9, specs=((6, 8, 200), (10, 12, 300), (16, 20, 100)))
    b = hom.Batch(systems)
    cache = str(tmp_path / "tiles.json")
    best, times = autotune.tune(hom, b, c, z, -32.0, idx, hom.MIXED, candidates=(1, 4),
                                sample_every=2, cache_path=cache)
    say(f"  times {times} -> tile {best}")
    assert best in (1, 4) and set(times) == {1, 4} and all(v > 0 for v in times.values())
    again, times2 = autotune.tune(hom, b, c, z, -32.0, idx, hom.MIXED, candidates=(1, 4),
                                  sample_every=2, cache_path=cache)
    assert again == best and times2 == times  # served from the cache


def test_batch_graph_replay(hom):
    """The batched launch captured in a HIP graph: three replays, each after an eager reset of the
    state (and eager tracking work in between), equal the eager run bitwise (FP64)."""
    import torch
    say("[batch] hipGraph capture and replay")
    systems, starts, z, idx, c = _batch(seed=10, specs=((4, 5, 40), (9, 10, 60), (20, 36, 20)))
    b = hom.Batch(systems)
    P = len(z)
    params = hom.default_params(hom.FP64)
    ct = torch.tensor(c, dtype=torch.complex128, device="cuda")
    it = torch.tensor(idx, dtype=torch.int32, device="cuda")
    z0 = torch.tensor(z, dtype=torch.complex128, device="cuda")
    eager = hom.track(b, ct, z0, -32.0, params, sys_idx=it)
    ez, est = _np(eager.z), _np(eager.status)
    st = _state(hom, torch, z, P)

    def reset():
        st.z.copy_(z0)
        st.s.fill_(-32.0)
        st.ds.zero_()
        st.status.fill_(hom.PATH_START)
        st.counters.zero_()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up launch off the default stream, as capture requires
        hom.track(b, ct, None, None, params, state=st, sys_idx=it)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    reset()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hom.track(b, ct, None, None, params, state=st, sys_idx=it)
    torch.cuda.synchronize()
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        assert np.array_equal(_np(st.z), ez), rep
        assert np.array_equal(_np(st.status), est), rep
        other = hom.track(b, ct, z0, -32.0, params, sys_idx=it)  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(_np(other.z), ez)


def test_c4_full_size(hom):
    """The batched workload at full size: 256 planted-cell systems (n in 6..24, 8..64 monomials
    per equation), 584615 paths in one launch per form.  Each form ends >= 99.9% of the paths
    OK; every OK endpoint is a root (residual <= 1e-10) and distinct within its system.  A seeded
    sample (2 paths of each of 64 systems) against the oracle's tracker: FP64 path by path (same
    status, <= 1e-12 where kappa <= 1e4), the mixed form within 1e-10 unless the path ended on
    another path's root (counted)."""
    import concurrent.futures as cf
    import torch
    say("[batch c4 full] 256 systems, mixed + fp64")
    sy = W.c4_systems()
    systems, starts = [s_ for s_, _, _ in sy], [z0 for _, _, z0 in sy]
    z, idx, c = W.stack_batch(systems, starts)
    b = hom.Batch(systems)
    ct = torch.tensor(c, dtype=torch.complex128, device="cuda")
    it = torch.tensor(idx, dtype=torch.int32, device="cuda")
    zt = torch.tensor(z, dtype=torch.complex128, device="cuda")
    rows = np.concatenate([[0], np.cumsum([len(z0) for z0 in starts])])
    res = {}
    for name, prec in (("mixed", hom.MIXED), ("fp64", hom.FP64)):
        st = hom.track(b, ct, zt, -32.0, hom.default_params(prec), sys_idx=it)
        zg, sg = _np(st.z), _np(st.status)
        say(f"  {name}: {len(sg)} paths, statuses {status_hist(sg)}")
        assert (sg == 0).mean() >= 0.999
        for q, s_ in enumerate(systems):
            zq, ok = zg[rows[q]:rows[q + 1], :s_.n], sg[rows[q]:rows[q + 1]] == 0
            assert oracle.residual(s_, s_.c, zq[ok]).max(initial=0.0) <= 1e-10, (name, q)
            assert distinct_count(zq[ok]) == int(ok.sum()), (name, q)
        res[name] = (zg, sg)
    rng = np.random.default_rng(404)
    picks = [(int(q), rng.choice(len(starts[q]), 2, replace=False)) for q in
             rng.choice(len(systems), 64, replace=False)]

    def ora(item):
        q, loc = item
        ze, _, _, ost, _ = oracle.track(systems[q], systems[q].c, starts[q][loc], -32.0, threads=1)
        return ze, ost

    with cf.ThreadPoolExecutor(16) as ex:
        refs = list(ex.map(ora, picks))
    swaps = 0
    for (q, loc), (ze, ost) in zip(picks, refs):
        s_ = systems[q]
        zf, sf = res["fp64"][0][rows[q] + loc, :s_.n], res["fp64"][1][rows[q] + loc]
        check_fp64_per_path(s_, zf, sf, ze, ost, f"system {q}", max_excluded=0.5)
        zm, sm = res["mixed"][0][rows[q] + loc, :s_.n], res["mixed"][1][rows[q] + loc]
        d = mod2pi_dist(zm, ze)
        both = (sm == 0) & (ost == 0)
        swaps += int((both & (d > 1e-10)).sum())  # roots and distinct: checked above
    say(f"  sampled mixed paths ending on another path's root: {swaps} of {2 * len(picks)}")
    assert swaps == 0
