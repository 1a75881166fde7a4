"""GPU parity of hom_track against the oracle's tracker (same rules, same constants)."""
import numpy as np
import pytest

import oracle
import pins
import workloads as W
from gpu_util import (check_fp64_per_path, check_mixed_set, mod2pi_dist, say, status_hist,
                      torch_params)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hom():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    import paper_2111_14317_amd as hom
    return hom


def _np(t):
    return t.cpu().numpy()


def _key(z, digits=6):
    return {tuple(v) for v in np.round(np.c_[z.real, np.mod(z.imag + 1e-7, 2 * np.pi)] * 10 ** digits)}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c1_all_mixed_volume_paths(hom, prec):
    """Every mixed-volume path of the tiny system, one handle per mixed cell: endpoints match
    the oracle's, are distinct, and are roots (residual <= 1e-10)."""
    say(f"[track c1 all cells] {prec}")
    base, cells = W.c1_cells()
    precision = hom.FP64 if prec == "fp64" else hom.MIXED
    gpu_end, ora_end = [], []
    for csys, info, z0 in cells:
        h = hom.System.from_workload(csys)
        st = hom.track(h, csys.c, z0, -32.0, hom.default_params(precision))
        assert (_np(st.status) == 0).all(), _np(st.status)
        gpu_end.append(_np(st.z))
        ze, _, _, ost, _ = oracle.track(csys, csys.c, z0, -32.0)
        ora_end.append(ze)
    g, o = np.concatenate(gpu_end), np.concatenate(ora_end)
    assert mod2pi_dist(g, o).max() <= 1e-12
    assert len(_key(g)) == pins.mixed_volume(base) == len(g)
    assert oracle.residual(base, base.c, g).max() <= 1e-10


def test_fp64_matches_oracle_per_path(hom):
    """n=8 planted-cell paths: the same status and the same endpoint on every path; counters
    close."""
    say("[track c5 fp64 per-path] P=512")
    csys, cell, z0 = W.planted_config("c5", P=512)
    p = oracle.TrackParams()
    h = hom.System.from_workload(csys)
    st = hom.track(h, csys.c, z0, -32.0, torch_params(hom, p, hom.FP64))
    ze, se, _, ost, ocnt = oracle.track(csys, csys.c, z0, -32.0, p)
    check_fp64_per_path(csys, _np(st.z), _np(st.status), ze, ost, "fp64")
    gc = _np(st.counters)
    assert abs(gc[:, 3].mean() / ocnt[:, 3].mean() - 1) < 0.02
    assert oracle.residual(csys, csys.c, _np(st.z)[_np(st.status) == 0]).max() <= 1e-10


def test_mixed_matches_oracle_endpoints(hom):
    say("[track c5 mixed] P=512")
    csys, cell, z0 = W.planted_config("c5", P=512)
    h = hom.System.from_workload(csys)
    b = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED))
    ze, _, _, ost, _ = oracle.track(csys, csys.c, z0, -32.0)
    check_mixed_set(csys, _np(b.z), _np(b.status), ze, ost, "mixed", max_swaps=0.0)


def test_c2_full_endpoint_parity(hom):
    """The n = 10 workload at full size, 65536 planted-cell paths, against the oracle's tracker:
    FP64 path by path (same status everywhere, <= 1e-12 on every well-conditioned endpoint); the
    mixed form as a set (>= 99.9% OK, every OK endpoint distinct, a root, and within 1e-10 of an
    oracle endpoint), with its failures reported by status."""
    say("[track c2 full] P=65536 fp64 + mixed vs oracle")
    csys, cell, z0 = W.planted_config("c2", P=65536)
    h = hom.System.from_workload(csys)
    ze, _, _, ost, _ = oracle.track(csys, csys.c, z0, -32.0)
    say(f"  oracle: {status_hist(ost)}")
    a = hom.track(h, csys.c, z0, -32.0, torch_params(hom, oracle.TrackParams(), hom.FP64))
    check_fp64_per_path(csys, _np(a.z), _np(a.status), ze, ost, "fp64", max_excluded=1e-3)
    b = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED))
    check_mixed_set(csys, _np(b.z), _np(b.status), ze, ost, "mixed", max_swaps=0.0)


def test_resume_bitwise(hom):
    """With exact row shifts, max_steps-limited calls resumed until done equal one call bitwise;
    with the default (lagged) shifts they agree to rounding."""
    say("[track resume] c5 P=256")
    csys, cell, z0 = W.planted_config("c5", P=256)
    h = hom.System.from_workload(csys)
    for flags in (hom.TRACK_EXACT_SHIFT, 0):
        full = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.FP64, flags=flags))
        p = hom.default_params(hom.FP64, max_steps=9, flags=flags)
        st = hom.track(h, csys.c, z0, -32.0, p)
        for _ in range(500):
            if not (_np(st.status) == hom.PATH_RUNNING).any():
                break
            st = hom.track(h, csys.c, None, None, p, state=st)
        assert np.array_equal(_np(st.status), _np(full.status))
        if flags:
            assert np.array_equal(_np(st.z), _np(full.z)) and np.array_equal(_np(st.s), _np(full.s))
        else:
            ok = _np(st.status) == 0
            assert mod2pi_dist(_np(st.z)[ok], _np(full.z)[ok]).max() <= 1e-12


def test_mixed_beside_equals_serial(hom):
    """The mixed form re-tracks its parked paths in FP64 beside the FP32 launch by default; the
    results equal those of re-tracking them after it (TRACK_SERIAL) bit for bit, since the same
    FP64 kernel runs every parked path from the same state."""
    say("[track mixed beside vs serial] c2 P=16384")
    csys, cell, z0 = W.planted_config("c2", P=16384)
    h = hom.System.from_workload(csys)
    a = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED))
    b = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED, flags=hom.TRACK_SERIAL))
    for f in ("z", "s", "ds", "status", "counters"):
        assert np.array_equal(_np(getattr(a, f)), _np(getattr(b, f))), f
    assert (_np(a.status) == 0).mean() >= 0.999


def test_mixed_side_nowait_equals_serial(hom):
    """The side launch's hand-over: with TRACK_SIDE_NOWAIT it gives up as soon as it finds no
    parked path waiting, and the call's last launch re-tracks what it left; the results still
    equal the serial order bit for bit."""
    say("[track mixed side nowait vs serial] c2 P=16384")
    csys, cell, z0 = W.planted_config("c2", P=16384)
    h = hom.System.from_workload(csys)
    a = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED, flags=hom.TRACK_SIDE_NOWAIT))
    b = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED, flags=hom.TRACK_SERIAL))
    for f in ("z", "s", "ds", "status", "counters"):
        assert np.array_equal(_np(getattr(a, f)), _np(getattr(b, f))), f


def test_deterministic_and_batch_independent(hom):
    """Bitwise-equal endpoints across runs and when the path set is split."""
    say("[track determinism] c5 P=300")
    csys, cell, z0 = W.planted_config("c5", P=300)
    h = hom.System.from_workload(csys)
    a = hom.track(h, csys.c, z0, -32.0)
    b = hom.track(h, csys.c, z0, -32.0)
    c1 = hom.track(h, csys.c, z0[:117], -32.0)
    c2 = hom.track(h, csys.c, z0[117:], -32.0)
    assert np.array_equal(_np(a.z), _np(b.z))
    assert np.array_equal(_np(a.z), np.concatenate([_np(c1.z), _np(c2.z)]))


def test_failure_modes_forced(hom):
    """Host-forced outcomes on the GPU match the oracle's: a start point far off every path, a
    NaN start, a zero step budget."""
    say("[track failures] c5 P=8")
    csys, cell, z0 = W.planted_config("c5", P=8)
    bad = z0.copy()
    bad[0] += 0.7
    bad[1, 0] = np.nan
    h = hom.System.from_workload(csys)
    st = hom.track(h, csys.c, bad, -32.0)
    _, _, _, ost, _ = oracle.track(csys, csys.c, bad, -32.0)
    assert np.array_equal(_np(st.status), ost)
    st = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.FP64, max_steps=0))
    assert (_np(st.status) == hom.PATH_RUNNING).all() and (_np(st.s) == -32.0).all()
    st = hom.track(h, csys.c, z0[:0], -32.0)  # P = 0
    assert st.z.shape[0] == 0


@pytest.mark.parametrize("n", [2, 4, 6, 7, 12, 13, 16, 20, 24, 32])
def test_every_group_size(hom, n):
    """One planted system per compiled group size (n = 13 and 16 both run on 16-lane groups;
    n = 24, 32 read their tables from global memory), 40 paths: FP64 matches the oracle path by
    path, the mixed form matches it as a set."""
    say(f"[track group size] n={n} P=40")
    rng = np.random.default_rng(200 + n)
    sy = W.random_system(n, 10, W._uniform_exps(-3, 3), "unit", 63, rng, rng, rng)
    csys, cell = W.plant_cell(sy, 63, rng, min_det=40)
    z0 = W.binomial_start_points(csys, cell, 40, rng)
    h = hom.System.from_workload(csys)
    ze, _, _, ost, _ = oracle.track(csys, csys.c, z0, -32.0)
    a = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.FP64))
    check_fp64_per_path(csys, _np(a.z), _np(a.status), ze, ost, "fp64")
    b = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED))
    check_mixed_set(csys, _np(b.z), _np(b.status), ze, ost, "mixed", min_ok=1.0)


@pytest.mark.parametrize("cfg,P", [("c5", 2048), ("c2", 16384)])
def test_hermite_predictor_matches_oracle(hom, cfg, P):
    """The cubic Hermite predictor (from the last two accepted points and their Euler
    directions): FP64 path by path against the oracle's tracker with the same predictor, the mixed
    form path by path as well, both with fewer eval+solves than the Euler predictor."""
    say(f"[track hermite] {cfg} P={P}")
    csys, cell, z0 = W.planted_config(cfg, P=P)
    h = hom.System.from_workload(csys)
    po = oracle.TrackParams(predictor=1)
    ze, _, _, ost, ocnt = oracle.track(csys, csys.c, z0, -32.0, po)
    a = hom.track(h, csys.c, z0, -32.0, torch_params(hom, po, hom.FP64))
    check_fp64_per_path(csys, _np(a.z), _np(a.status), ze, ost, "fp64 hermite")
    gc = _np(a.counters)
    assert abs(gc[:, 3].mean() / ocnt[:, 3].mean() - 1) < 0.02
    b = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED, predictor=hom.PREDICT_HERMITE))
    check_mixed_set(csys, _np(b.z), _np(b.status), ze, ost, "mixed hermite", max_swaps=0.0)
    e = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED))
    say(f"  eval+solves per path: hermite {_np(b.counters)[:, 3].mean():.1f}, "
        f"euler {_np(e.counters)[:, 3].mean():.1f} (mixed); fp64 hermite {gc[:, 3].mean():.1f}")
    assert _np(b.counters)[:, 3].mean() < _np(e.counters)[:, 3].mean()


@pytest.mark.parametrize("cfg,P", [("c5", 2048), ("c2", 16384)])
def test_rk4_predictor_matches_oracle(hom, cfg, P):
    """The Runge-Kutta predictor (three stage evaluations per step): FP64 path by path against the
    oracle's tracker with the same predictor (eval+solve and step counts within 2%), the mixed form
    path by path as well, both in fewer accepted steps than the Euler predictor."""
    say(f"[track rk4] {cfg} P={P}")
    csys, cell, z0 = W.planted_config(cfg, P=P)
    h = hom.System.from_workload(csys)
    po = oracle.TrackParams(predictor=2)
    ze, _, _, ost, ocnt = oracle.track(csys, csys.c, z0, -32.0, po)
    a = hom.track(h, csys.c, z0, -32.0, torch_params(hom, po, hom.FP64))
    check_fp64_per_path(csys, _np(a.z), _np(a.status), ze, ost, "fp64 rk4")
    gc = _np(a.counters)
    assert abs(gc[:, 3].mean() / ocnt[:, 3].mean() - 1) < 0.02
    assert abs(gc[:, 0].mean() / ocnt[:, 0].mean() - 1) < 0.02
    b = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED, predictor=hom.PREDICT_RK4))
    check_mixed_set(csys, _np(b.z), _np(b.status), ze, ost, "mixed rk4", max_swaps=0.0)
    e = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.MIXED))
    say(f"  accepted steps per path: rk4 {_np(b.counters)[:, 0].mean():.1f}, "
        f"euler {_np(e.counters)[:, 0].mean():.1f} (mixed); eval+solves rk4 "
        f"{_np(b.counters)[:, 3].mean():.1f}, euler {_np(e.counters)[:, 3].mean():.1f}")
    assert _np(b.counters)[:, 0].mean() < _np(e.counters)[:, 0].mean()
