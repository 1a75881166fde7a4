"""Benchmark: eval + consolidated Euler/Newton solves per second while tracking paths.

Workload (one step = one full pass of the hot path): a random n = 10 Laurent system with 12
monomials per equation (exponents uniform in [-3, 3], unit-circle coefficients) and a planted
mixed cell (lifting 0 on one pair per equation, U{1..63} elsewhere); 65536 paths tracked from
s = -32 to s = 0 with the persistent predictor-corrector kernel, Euler predictor and Newton
corrector from one consolidated LU per evaluation, FP64 endgame.  Both forms run: the plain
FP64 form and the mixed form (FP32 exponentials, contraction and LU).  `value` is the mixed
form's rate; a form's number counts only when >= 99.9% of its paths end OK (residual <= 1e-10).

Timing: W untimed warmup steps, then K steps back to back, each on its own pre-staged copy of
the start state (inputs resident in HBM), bracketed by torch.cuda.synchronize().  Kernel
durations for the roofline come from hipEvents the library records around its own launches.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "eval+Euler/Newton solves/sec (n=10, 64K paths), mixed vs FP64 at 1e-10 resid"
UNIT = "eval+solve/s"
N_EQ, M_EQ = 10, 12
# algorithmic work of one eval + 2-rhs solve at n = 10, 12 monomials per equation (FMA = 2 flops)
#   A1 exponent sums  : M (2n + 1) FMA             = 120 * 21 * 2      = 5040
#   A2 c * exp(u - M) : 3 real mults per monomial  = 120 * 6           =  720   (+3 transcendentals)
#   A3 contraction    : M ((n + 1) complex FMA by a real + 1 complex add) = 120 * (11*4 + 2) = 5520
#   A5 LU, 2 rhs      : sum_j (n-1-j)(6 + 8 (n+1-j)) + 10 reciprocals (8) + 2 back-subs (45*8 + 10*6)
#                     = 3270 + 80 + 840 = 4190
FLOPS_PER_UNIT = 5040 + 720 + 5520 + 4190
FP64_SHARE = 5040  # the exponent sums stay FP64 in the mixed form
PEAK_FP64 = 78.6e12
PEAK_FP32 = 157.3e12


# HBM traffic of the dominant kernel comes from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE),
# summarised in this file together with a hash of the kernel's sources; it is reported only while
# the sources still hash to the same value (after a kernel change the counters are stale).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_track_n10_mixed_hbm.txt")
KERNEL_SOURCES = ["paper_2111_14317_amd/csrc/k_track.hip", "paper_2111_14317_amd/csrc/hom_device.h",
                  "paper_2111_14317_amd/csrc/hom_internal.h"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the mixed tracker (fetch + write, calibrated), or None when the
    summary is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("sources_sha256") != kernel_sources_sha256():
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _peak_mixed():
    # time lower bound: FP64 part at the FP64 peak, the rest at the FP32 peak
    t = FP64_SHARE / PEAK_FP64 + (FLOPS_PER_UNIT - FP64_SHARE) / PEAK_FP32
    return FLOPS_PER_UNIT / t


def _workload(P):
    import workloads as W
    csys, cell, z0 = W.planted_config("c2", P=P)
    return csys, z0


def run_form(hom, torch, h, csys, z0, precision, steps, warmup, **overrides):
    """Returns dict with rate, ms/step, ok fraction, mean evals/path, kernel timings and the last
    step's endpoints and statuses."""
    dev = "cuda"
    P = z0.shape[0]
    c = torch.tensor(csys.c, dtype=torch.complex128, device=dev)
    z_init = torch.tensor(z0, dtype=torch.complex128, device=dev)
    params = hom.default_params(precision, **overrides)
    total = warmup + steps
    states = []
    for _ in range(total):
        states.append(hom.TrackState(
            z_init.clone(), torch.full((P,), -32.0, dtype=torch.float64, device=dev),
            torch.zeros(P, dtype=torch.float64, device=dev),
            torch.full((P,), hom.PATH_START, dtype=torch.int32, device=dev),
            torch.zeros((P, 4), dtype=torch.int32, device=dev)))
    torch.cuda.synchronize()
    for i in range(warmup):
        hom.track(h, c, None, None, params, state=states[i])
    torch.cuda.synchronize()
    hom.profile_read()  # drop anything recorded so far
    hom.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, total):
        hom.track(h, c, None, None, params, state=states[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hom.set_profiling(False)
    prof = hom.profile_read()
    evals = 0
    ok = []
    evals_per_path = []
    for i in range(warmup, total):
        cnt = states[i].counters.cpu()
        evals += int(cnt[:, 3].sum())
        st = states[i].status.cpu()
        ok.append(float((st == hom.PATH_OK).float().mean()))
        evals_per_path.append(float(cnt[:, 3].float().mean()))
    sec = t1 - t0
    kern, units = {}, {}  # per step: summed over the launches of one label (the mixed form
    for name, ms, u in prof:  # runs k_track<n,fp64> twice per step: polish, then finish)
        kern[name] = kern.get(name, 0.0) + ms / steps
        units[name] = units.get(name, 0.0) + u / steps
    launches = {}
    for name, _, _ in prof:
        launches[name] = launches.get(name, 0) + 1
    last = states[total - 1]
    return dict(rate=evals / sec, ms_per_step=1e3 * sec / steps, ok_frac=min(ok),
                evals_per_path=sum(evals_per_path) / len(evals_per_path),
                evals_per_step=evals / steps, kernels=kern, units=units,
                launches={k: v / steps for k, v in launches.items()}, paths_per_s=P * steps / sec,
                z_end=last.z.cpu().numpy(), status=last.status.cpu().numpy())


def status_hist(st):
    import numpy as np
    u, c = np.unique(st, return_counts=True)
    return {str(int(a)): int(b) for a, b in zip(u, c)}


def _mod2pi_dist(a, b):
    import numpy as np
    dre = np.abs(a.real - b.real)
    dim = np.abs(np.angle(np.exp(1j * (a.imag - b.imag))))
    return np.maximum(dre, dim).max(axis=-1)


def _projection(z, seed=20211129):
    """fixed random positive weights on Re z_j, cos Im z_j, sin Im z_j; points within d of each
    other (max modulus, mod 2 pi i) project to within W d"""
    import numpy as np
    rng = np.random.default_rng(seed)
    n = z.shape[1]
    wr, wc, ws = (rng.uniform(0.5, 1.0, n) for _ in range(3))
    return z.real @ wr + np.cos(z.imag) @ wc + np.sin(z.imag) @ ws, wr.sum() + wc.sum() + ws.sum()


def _nearest(a, b, radius=1e-6):
    """smallest max-modulus distance (mod 2 pi i) from each row of a to the rows of b within
    `radius` (inf when none)"""
    import numpy as np
    out = np.full(len(a), np.inf)
    if len(a) == 0 or len(b) == 0:
        return out
    pa, W = _projection(a)
    pb, _ = _projection(b)
    order = np.argsort(pb)
    pbs = pb[order]
    lo = np.searchsorted(pbs, pa - radius * W, side="left")
    hi = np.searchsorted(pbs, pa + radius * W, side="right")
    for k in range(int((hi - lo).max(initial=0))):
        idx = np.nonzero(hi - lo > k)[0]
        out[idx] = np.minimum(out[idx], _mod2pi_dist(a[idx], b[order[lo[idx] + k]]))
    return out


def _distinct(z, tol=1e-8):
    """number of endpoints pairwise more than tol apart (mod 2 pi i)"""
    import numpy as np
    if len(z) == 0:
        return 0
    p, W = _projection(z)
    order = np.argsort(p)
    ps = p[order]
    dup = np.zeros(len(z), bool)
    k = 1
    while k < len(ps):
        near = ps[k:] - ps[:-k] <= tol * W
        if not near.any():
            break
        i, j = order[:-k][near], order[k:][near]
        dup[np.maximum(i, j)[_mod2pi_dist(z[i], z[j]) <= tol]] = True
        k += 1
    return int((~dup).sum())


def compare_endpoints(a, b):
    """Form a's endpoints against form b's, path by path (same start points): how many paths end
    OK in both, the largest distance over them, how many differ by more than 1e-10 (a path that
    ended on another path's root), and the distinct OK endpoints of each form."""
    import numpy as np
    both = (a["status"] == 0) & (b["status"] == 0)
    d = _mod2pi_dist(a["z_end"][both], b["z_end"][both])
    return {"both_ok": int(both.sum()), "max_dist": float(d.max()) if both.any() else 0.0,
            "differ_gt_1e-10": int((d > 1e-10).sum()),
            "distinct_ok": [_distinct(a["z_end"][a["status"] == 0]),
                            _distinct(b["z_end"][b["status"] == 0])]}


# dense-support configuration: n = 32, 128 monomials per equation, 262144 points (eval and step)
C3_N, C3_M = 32, 128
C3_MONO = C3_N * C3_M
#   A1 2 (2n + 1) M = 532480, A2 8 M = 32768, A3 M (4n + 6) = 548864  (FMA = 2 flops)
C3_FLOPS_EVAL = 2 * (2 * C3_N + 1) * C3_MONO + 8 * C3_MONO + C3_MONO * (4 * C3_N + 6)
#   A5 on the 32 x 32 complex J with 2 right-hand sides: (8/3) n^3 + 16 n^2
C3_FLOPS_LU = int(8 * C3_N ** 3 / 3 + 16 * C3_N ** 2)
# matrix-core work the engines issue per point (the BF16x3 split repeats products)
#   BF16x3: per 16 monomials x 16 points, 1 + 6 MFMA 16x16x32 for A1 (row maximum, then hi/mid/lo
#           of Re and of the three phase digits); per 32 monomials x 16 points 6 MFMA per
#           16-column tile for A3 (Re/Im x hi/mid/lo), two column tiles
C3_MFMA_BF16 = C3_MONO * ((1 + 6) * 16384 / 256 + 6 * 2 * 16384 / 512)
#   FP64: per 16 x 16, 8 + 8 MFMA 16x16x4 f64 (Re, Im; K = 32 in steps of 4) for A1, 4 x 2 x 2 for
#         A3 (K = 4 monomials at a time, two column tiles, Re/Im)
C3_MFMA_F64 = C3_MONO * ((8 + 8) * 2048 / 256 + 16 * 2048 / 256)
PEAK_BF16 = 2.5e15
PEAK_HBM = 8.0e12


def run_dense(hom, torch, P, reps=3):
    """Dense-support eval and step at n = 32, m = 128: per engine, kernel ms (library events),
    points/s, algorithmic TFLOP/s and the matrix-core issue rate."""
    import workloads as W
    sys_, z, s = W.config_system("c3", P=P)
    dev = "cuda"
    c = torch.tensor(sys_.c, dtype=torch.complex128, device=dev)
    zt = torch.tensor(z, dtype=torch.complex128, device=dev)
    st = torch.tensor(s, dtype=torch.float64, device=dev)
    h = hom.System.from_workload(sys_)
    out = {}
    legs = [("eval_mfma_fp64", "eval", 0), ("eval_mfma_bf16x3", "eval", hom.EVAL_FP32),
            ("eval_valu_fp64", "eval", hom.EVAL_VALU), ("step_mfma_fp64", "step", hom.FP64),
            ("step_mfma_bf16x3", "step", hom.MIXED)]
    for name, kind, arg in legs:
        def once():
            if kind == "eval":
                G, L = hom.eval(h, c, zt, st, flags=arg)
                del G, L
            else:
                r = hom.step(h, c, zt, st, precision=arg)
                del r
        once()
        torch.cuda.synchronize()
        hom.profile_read()
        hom.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            once()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        hom.set_profiling(False)
        kern = {}
        for kname, ms, _u in hom.profile_read():
            kern[kname] = kern.get(kname, 0.0) + ms / reps
        ms = sum(kern.values())
        flops = C3_FLOPS_EVAL + (C3_FLOPS_LU if kind == "step" else 0)
        rec = {"kernels_ms": kern, "ms": ms, "wall_ms": wall * 1e3, "points_per_s": P / (ms * 1e-3),
               "tflops_algorithmic": P * flops / (ms * 1e-3) / 1e12}
        ek = [k for k in kern if k.startswith("k_dense<") or k.startswith("k_eval<")]
        if ek:
            ems = sum(kern[k] for k in ek)
            rec["eval_kernel_ms"] = ems
            if "bf16x3" in name:
                rec["mfma_tflops_issued"] = P * C3_MFMA_BF16 / (ems * 1e-3) / 1e12
                rec["mfma_frac_of_bf16_peak"] = P * C3_MFMA_BF16 / (ems * 1e-3) / PEAK_BF16
            elif "mfma_fp64" in name:
                rec["mfma_tflops_issued"] = P * C3_MFMA_F64 / (ems * 1e-3) / 1e12
                rec["mfma_frac_of_fp64_peak"] = P * C3_MFMA_F64 / (ems * 1e-3) / PEAK_FP64
            rec["frac_of_fp64_peak_algorithmic"] = P * C3_FLOPS_EVAL / (ems * 1e-3) / PEAK_FP64
        out[name] = rec
        print(f"# c3 {name}: {ms:.2f} ms, {rec['points_per_s']:.3e} points/s, kernels {kern}",
              file=sys.stderr, flush=True)
    return out


# common support (every equation on one support of m = 128 monomials), per point:
#   A1 2 (2n + 1) m and A2 8 m once, then per equation c_k . E (6 m) and the contraction m (4n + 6)
U_FLOPS_EVAL = 2 * (2 * C3_N + 1) * C3_M + 8 * C3_M + C3_N * C3_M * (4 * C3_N + 12)
#   FP64 MFMA issued: A1 16 per 16 x 16 on the m common monomials, A3 16 per 16 x 16 per equation
U_MFMA_F64 = C3_M * 16 * 2048 / 256 + C3_MONO * 16 * 2048 / 256


def run_union(hom, torch, P, reps=3):
    """Common-support system at n = 32, m = 128 (exponentials shared by the equations): FP64 eval
    and step on the common-support engine against the per-equation engine on the same system."""
    import workloads as W
    sys_, z, s = W.union_config(P=P)
    dev = "cuda"
    c = torch.tensor(sys_.c, dtype=torch.complex128, device=dev)
    zt = torch.tensor(z, dtype=torch.complex128, device=dev)
    st = torch.tensor(s, dtype=torch.float64, device=dev)
    out = {}
    for per_eq in (False, True):
        h = hom.System.from_workload(sys_, per_equation=per_eq)
        for kind in ("eval", "step"):
            name = f"{kind}_{'per_equation' if per_eq else 'common_support'}_fp64"

            def once():
                r = hom.eval(h, c, zt, st) if kind == "eval" else hom.step(h, c, zt, st)
                del r
            once()
            torch.cuda.synchronize()
            hom.profile_read()
            hom.set_profiling(True)
            for _ in range(reps):
                once()
            torch.cuda.synchronize()
            hom.set_profiling(False)
            kern = {}
            for kname, ms, _u in hom.profile_read():
                kern[kname] = kern.get(kname, 0.0) + ms / reps
            ms = sum(kern.values())
            ek = [k for k in kern if k in ("k_union<fp64>", "k_dense<fp64>")]
            ems = sum(kern[k] for k in ek)
            rec = {"kernels_ms": kern, "ms": ms, "points_per_s": P / (ms * 1e-3),
                   "eval_kernel_ms": ems,
                   "eval_tflops_algorithmic": P * U_FLOPS_EVAL / (ems * 1e-3) / 1e12,
                   "eval_frac_of_fp64_peak_algorithmic": P * U_FLOPS_EVAL / (ems * 1e-3) / PEAK_FP64}
            if not per_eq:
                rec["mfma_frac_of_fp64_peak"] = P * U_MFMA_F64 / (ems * 1e-3) / PEAK_FP64
            out[name] = rec
            print(f"# union {name}: {ms:.2f} ms, {rec['points_per_s']:.3e} points/s, kernels {kern}",
                  file=sys.stderr, flush=True)
        h.close()
    return out


def run_starts(hom, torch, reps=3):
    """Start points of the n = 10 tracking workload's planted cell: all |det D| = 3,881,632 roots
    of its binomial system (Smith form and base root planned on the GPU, then one launch writing
    16 bytes per root coordinate, judged against HBM); and 1024 small random cells in one call."""
    import numpy as np
    import workloads as W
    csys, cell, _ = W.planted_config("c2", P=4)
    D, beta = W.cell_binomial(csys, cell)
    z, num = hom.binomial_starts(D, beta)
    del z
    torch.cuda.synchronize()
    hom.profile_read()
    hom.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        z, _ = hom.binomial_starts(D, beta)
        del z
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    hom.set_profiling(False)
    prof = hom.profile_read()
    ms = sum(t for k, t, _ in prof if k == "k_binomial_starts") / reps
    plan_ms = sum(t for k, t, _ in prof if k == "k_start_plan") / reps
    rows = int(num[0])
    nbytes = rows * csys.n * 16
    rec = {"roots": rows, "n": csys.n, "kernel_ms": ms, "plan_ms": plan_ms, "call_ms": wall * 1e3,
           "roots_per_s": rows / (ms * 1e-3), "hbm_gb_per_s": nbytes / (ms * 1e-3) / 1e9,
           "frac_of_hbm_peak": nbytes / (ms * 1e-3) / PEAK_HBM}
    print(f"# starts n=10 cell: {rows} roots, kernel {ms:.3f} ms ({rec['hbm_gb_per_s']:.0f} GB/s), "
          f"plan {plan_ms:.2f} ms, call {wall * 1e3:.2f} ms", file=sys.stderr, flush=True)
    # many cells in one call: 1024 n = 10 cells (random exponent differences in [-3, 3] with
    # 1 <= |det| <= 64), every root: the plan is one GPU thread per cell
    rng = np.random.default_rng(2111)
    Ds, betas = [], []
    while len(Ds) < 1024:
        Dc = rng.integers(-3, 4, size=(10, 10))
        Dc = np.triu(Dc, 1) * (rng.random((10, 10)) < 0.2) + np.diag(rng.choice([1, 1, 2, 3], 10))
        Dc = (np.tril(rng.integers(-1, 2, size=(10, 10)) * (rng.random((10, 10)) < 0.2), -1)
              + np.eye(10, dtype=np.int64)) @ Dc
        d = round(abs(np.linalg.det(Dc)))
        if 1 <= d <= 64:
            Ds.append(Dc[rng.permutation(10)])
            betas.append(rng.normal(size=10) + 1j * rng.normal(size=10))
    Ds, betas = np.stack(Ds), np.stack(betas)
    z, num = hom.binomial_starts(Ds, betas)
    del z
    torch.cuda.synchronize()
    hom.profile_read()
    hom.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        z, _ = hom.binomial_starts(Ds, betas)
        del z
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    hom.set_profiling(False)
    prof = hom.profile_read()
    rec["batch_1024_cells_n10"] = {
        "roots": int(num.sum()),
        "plan_ms": sum(t for k, t, _ in prof if k == "k_start_plan") / reps,
        "kernel_ms": sum(t for k, t, _ in prof if k == "k_binomial_starts") / reps,
        "call_ms": wall * 1e3}
    print(f"# starts 1024 n=10 cells: {rec['batch_1024_cells_n10']}", file=sys.stderr, flush=True)
    return rec


def run_eval_n10(hom, torch, P=65536, reps=5):
    """hom_eval and hom_step on P random points of the n = 10 system.  The evaluation reads z, s and
    writes G and the row scales (2168 B per point at n = 10): it is judged against HBM bandwidth."""
    import workloads as W
    sys_, z, s = W.config_system("c2", P=P)
    n = sys_.n
    dev = "cuda"
    c = torch.tensor(sys_.c, dtype=torch.complex128, device=dev)
    zt = torch.tensor(z, dtype=torch.complex128, device=dev)
    st = torch.tensor(s, dtype=torch.float64, device=dev)
    h = hom.System.from_workload(sys_)
    # bytes per point: z, s in; G, logscale out (eval) / dE, dN, status out (step)
    b_eval = 16 * n + 8 + 16 * n * (n + 2) + 8 * n
    b_step = 16 * n + 8 + 2 * 16 * n + 4
    out = {}
    for name, kind, arg, nbytes in (("eval_fp64", "eval", 0, b_eval),
                                    ("eval_fp32", "eval", hom.EVAL_FP32, b_eval),
                                    ("step_fp64", "step", hom.FP64, b_step),
                                    ("step_mixed", "step", hom.MIXED, b_step)):
        def once():
            if kind == "eval":
                return hom.eval(h, c, zt, st, flags=arg)
            return hom.step(h, c, zt, st, precision=arg)
        once()
        torch.cuda.synchronize()
        hom.profile_read()
        hom.set_profiling(True)
        for _ in range(reps):
            once()
        torch.cuda.synchronize()
        hom.set_profiling(False)
        ms = sum(t for _, t, _ in hom.profile_read()) / reps
        out[name] = {"ms": ms, "points_per_s": P / (ms * 1e-3), "bytes_per_point": nbytes,
                     "hbm_gb_per_s": P * nbytes / (ms * 1e-3) / 1e9,
                     "frac_of_hbm_peak": P * nbytes / (ms * 1e-3) / PEAK_HBM,
                     "frac_of_fp64_peak": P * (FLOPS_PER_UNIT - (4190 if kind == "eval" else 0))
                     / (ms * 1e-3) / PEAK_FP64}
        print(f"# n10 {name} P={P}: {ms:.3f} ms, {out[name]['hbm_gb_per_s']:.0f} GB/s",
              file=sys.stderr, flush=True)
    return out


def flops_step(n, M):
    """Algorithmic flops of one eval + 2-rhs solve of a system with n unknowns and M monomials
    (the same count as FLOPS_PER_UNIT, which is flops_step(10, 120))."""
    a1 = 2 * (2 * n + 1) * M
    a2 = 6 * M
    a3 = M * (4 * (n + 1) + 2)
    lu = sum((n - 1 - j) * (6 + 8 * (n + 1 - j)) for j in range(n)) + 8 * n
    back = 2 * (n * (n - 1) // 2 * 8 + 6 * n)
    return a1 + a2 + a3 + lu + back, a1


def run_c4(hom, torch, reps=3):
    """The batched form at full size: 256 planted-cell systems (n in 6..24, 8..64 monomials per
    equation), ~5.8e5 paths in one persistent launch sequence per call.  Per form: the work-item
    size from the autotuner, the call captured in a HIP graph and replayed `reps` times (the state
    is reset between replays, outside the timed region), eval+solve/s, paths/s, OK fraction, the
    batched kernel's time (library events, eager run) and its algorithmic TFLOP/s."""
    import numpy as np

    import workloads as W
    from paper_2111_14317_amd import autotune
    t0 = time.perf_counter()
    sy = W.c4_systems()
    systems, starts = [s_ for s_, _, _ in sy], [z0 for _, _, z0 in sy]
    z, idx, c = W.stack_batch(systems, starts)
    gen_s = time.perf_counter() - t0
    P = len(z)
    b = hom.Batch(systems)
    dev = "cuda"
    ct = torch.tensor(c, dtype=torch.complex128, device=dev)
    it = torch.tensor(idx, dtype=torch.int32, device=dev)
    z0 = torch.tensor(z, dtype=torch.complex128, device=dev)
    fl = np.array([flops_step(s_.n, int(np.sum(s_.m)))[0] for s_ in systems], np.float64)
    fl64 = np.array([flops_step(s_.n, int(np.sum(s_.m)))[1] for s_ in systems], np.float64)
    out = {"systems": len(systems), "paths": P, "generate_s": gen_s}
    for name, prec in (("mixed", hom.MIXED), ("fp64", hom.FP64)):
        tile, times = autotune.tune(hom, b, ct, z, -32.0, idx, prec, candidates=(1, 2, 4, 8),
                                    sample_every=8, cache_path=None)
        params = hom.default_params(prec, tile=tile)
        st = hom.TrackState(z0.clone(), torch.full((P,), -32.0, dtype=torch.float64, device=dev),
                            torch.zeros(P, dtype=torch.float64, device=dev),
                            torch.full((P,), hom.PATH_START, dtype=torch.int32, device=dev),
                            torch.zeros((P, 4), dtype=torch.int32, device=dev))

        def reset():
            st.z.copy_(z0)
            st.s.fill_(-32.0)
            st.ds.zero_()
            st.status.fill_(hom.PATH_START)
            st.counters.zero_()

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # a first launch off the default stream before capture
            hom.track(b, ct, None, None, params, state=st, sys_idx=it)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        reset()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            hom.track(b, ct, None, None, params, state=st, sys_idx=it)
        torch.cuda.synchronize()
        wall = []
        evals = ok = None
        for _ in range(reps):
            reset()
            torch.cuda.synchronize()
            t = time.perf_counter()
            g.replay()
            torch.cuda.synchronize()
            wall.append(time.perf_counter() - t)
            cnt = st.counters[:, 3].cpu().numpy().astype(np.float64)
            evals = cnt.sum()
            stt = st.status.cpu().numpy()
            ok = float((stt == 0).mean())
        del g
        # kernel time of the same call, eager, with the library's events
        reset()
        torch.cuda.synchronize()
        hom.profile_read()
        hom.set_profiling(True)
        hom.track(b, ct, None, None, params, state=st, sys_idx=it)
        torch.cuda.synchronize()
        hom.set_profiling(False)
        prof = hom.profile_read()
        kms = {}
        for kname, ms, u in prof:
            kms[kname] = kms.get(kname, 0.0) + ms
        cnt = st.counters[:, 3].cpu().numpy().astype(np.float64)
        work = float(np.sum(cnt * fl[idx]))
        work64 = float(np.sum(cnt * fl64[idx]))
        kern = f"k_track_batch<{name}>"
        ktot = sum(kms.values())
        peak = PEAK_FP64 if name == "fp64" else work / (work64 / PEAK_FP64 + (work - work64) / PEAK_FP32)
        rec = {"tile": tile, "tile_ms": times, "graph_replay_s": min(wall),
               "eval_solve_per_s": evals / min(wall), "paths_per_s": P / min(wall), "ok_frac": ok,
               "statuses": status_hist(stt), "evals_per_path": evals / P, "kernels_ms": kms,
               "tflops_algorithmic": work / (ktot * 1e-3) / 1e12,
               "frac_of_peak": work / (ktot * 1e-3) / peak, "peak_tflops": peak / 1e12,
               "dominant_kernel": kern}
        out[name] = rec
        print(f"# c4 {name}: tile {tile}, {min(wall):.3f} s/replay, {rec['eval_solve_per_s']:.3e} "
              f"{UNIT}, ok {ok:.5f}, {rec['tflops_algorithmic']:.2f} TFLOP/s", file=sys.stderr,
              flush=True)
    return out


def run_c5(hom, torch, P=16384, reps=3):
    """The differentiation workload: 16384 paths of the n = 8 system tracked in FP64, loss
    sum |x*|^2; the adjoint gradient w.r.t. all 128 coefficients in FP64 and in the mixed form:
    kernel ms (library events), paths/s, and the per-entry error against the oracle's gradient."""
    import numpy as np

    import oracle
    import workloads as W
    csys, cell, z0 = W.planted_config("c5", P=P)
    h = hom.System.from_workload(csys)
    st = hom.track(h, csys.c, z0, -32.0, hom.default_params(hom.FP64))
    z, sg = st.z.cpu().numpy(), st.status.cpu().numpy()
    ok = sg == 0
    g = np.where(ok[:, None], 2 * np.exp(z), 0)
    ref, _ = oracle.endpoint_grad(csys, csys.c, z, g)
    out = {"paths": P, "ok_frac": float(ok.mean())}
    dev = "cuda"
    zt = torch.tensor(z, dtype=torch.complex128, device=dev)
    gt = torch.tensor(g, dtype=torch.complex128, device=dev)
    ct = torch.tensor(csys.c, dtype=torch.complex128, device=dev)
    for name, prec in (("fp64", hom.FP64), ("mixed", hom.MIXED)):
        got = hom.endpoint_grad(h, ct, zt, gt, precision=prec)
        torch.cuda.synchronize()
        hom.profile_read()
        hom.set_profiling(True)
        for _ in range(reps):
            got = hom.endpoint_grad(h, ct, zt, gt, precision=prec)
        torch.cuda.synchronize()
        hom.set_profiling(False)
        ms = sum(t for _, t, _ in hom.profile_read()) / reps
        err = np.abs(got.cpu().numpy() - ref) / np.abs(ref)
        out[name] = {"kernel_ms": ms, "paths_per_s": P / (ms * 1e-3),
                     "max_rel_err_per_entry_vs_oracle": float(err.max())}
        print(f"# c5 grad {name}: {ms:.3f} ms, max per-entry rel err {err.max():.2e}",
              file=sys.stderr, flush=True)
    return out


def error_table(hom, torch, csys, mixed, fp64, ora_z, ora_st, c5):
    """The mixed form's error against the FP64 oracle, per result: G (scaled componentwise metric)
    and d_E, d_N (relative, where kappa <= 1e2; and the largest error / kappa anywhere) on 4096
    random points of the n = 10 system; endpoints (the last timed step of each form against the
    oracle's endpoints of the CPU-baseline sample, as sets; and the FP64 form path by path); the
    adjoint gradient (per entry, from the differentiation leg)."""
    import numpy as np

    import oracle
    import workloads as W
    sys_, z, s = W.config_system("c2", P=4096)
    h = hom.System.from_workload(sys_)
    G, L = hom.eval(h, sys_.c, z, s, flags=hom.EVAL_FP32)
    Go, Lo, den = oracle.eval(sys_, sys_.c, z, s, with_den=True)
    Gg = G.cpu().numpy() * np.exp(L.cpu().numpy() - Lo)[:, :, None]
    scale = np.maximum(den, 1e-30 * den[:, :, -1:])
    eG = float((np.abs(Gg - Go) / np.where(scale > 0, scale, 1.0)).max())
    dE, dN, st = hom.step(h, sys_.c, z, s, precision=hom.MIXED)
    oE, oN, ost, _ = oracle.step(sys_, sys_.c, z, s)
    kap = np.abs(np.linalg.cond(Go[:, :, :sys_.n], p=np.inf))

    def rel(a, b):
        return np.abs(a - b).max(1) / np.abs(b).max(1)

    eE, eN = rel(dE.cpu().numpy(), oE), rel(dN.cpu().numpy(), oN)
    well = (kap <= 1e2) & (ost == 0)
    fin = ost == 0
    out = {"G_scaled_max": eG,
           "dE_rel_max_kappa_le_1e2": float(eE[well].max()),
           "dN_rel_max_kappa_le_1e2": float(eN[well].max()),
           "dE_over_kappa_max": float((eE / kap)[fin].max()),
           "dN_over_kappa_max": float((eN / kap)[fin].max()), "points": len(z),
           "points_kappa_le_1e2": int(well.sum())}
    n0 = len(ora_z)
    for name, form in (("mixed", mixed), ("fp64", fp64)):
        zg, sg = form["z_end"][:n0], form["status"][:n0]
        okg = sg == 0
        d = _nearest(zg[okg], ora_z[ora_st == 0])
        both = okg & (ora_st == 0)
        out[f"endpoints_{name}"] = {
            "paths": n0, "ok": int(okg.sum()), "set_max_dist": float(d.max()),
            "path_by_path_max_dist": float(_mod2pi_dist(zg[both], ora_z[both]).max()),
            "paths_on_another_root": int((_mod2pi_dist(zg[both], ora_z[both]) > 1e-10).sum())}
    if c5:
        out["grad_rel_max_per_entry"] = c5["mixed"]["max_rel_err_per_entry_vs_oracle"]
        out["grad_rel_max_per_entry_fp64_form"] = c5["fp64"]["max_rel_err_per_entry_vs_oracle"]
    return out


def flops_step_proj(n, M):
    """Algorithmic flops of one projective step (n equations, n + 1 homogeneous unknowns, M
    monomials): A1 over n + 1 coordinates and the lifting, A2, A3 with n + 3 columns, the
    y-coordinate epilogue, the Householder LQ of the (n+1) x (n+3) unified system (complex: 4 real
    flops per multiply-add) and the two null vectors."""
    nu, cols = n + 1, n + 3
    a1 = 2 * (2 * nu + 1) * M
    a2 = 6 * M
    a3 = M * (4 * (nu + 1) + 2)
    epi = 6 * n * nu
    lq = 4 * (2 * cols * nu * nu - 2 * nu ** 3 // 3)
    null = 2 * 2 * 8 * sum(cols - i for i in range(nu))
    return a1 + a2 + a3 + epi + lq + null


def run_step_proj(hom, torch, P=65536, reps=5):
    """hom_step_proj on P random homogeneous points of the n = 10 system: kernel ms (library
    events), points/s and the algorithmic FP64 rate."""
    import numpy as np

    import workloads as W
    sys_, z, s = W.config_system("c2", P=P)
    rng = np.random.default_rng(5)
    lam = np.exp(rng.normal(0, 0.5, P) + 1j * rng.uniform(0, 2 * np.pi, P))
    y = np.concatenate([np.exp(z), np.ones((P, 1))], axis=1) * lam[:, None]
    h = hom.System.from_workload(sys_, projective=True)
    dev = "cuda"
    c = torch.tensor(sys_.c, dtype=torch.complex128, device=dev)
    yt = torch.tensor(y, dtype=torch.complex128, device=dev)
    st = torch.tensor(s, dtype=torch.float64, device=dev)
    out = hom.step_proj(h, c, yt, st)
    torch.cuda.synchronize()
    hom.profile_read()
    hom.set_profiling(True)
    for _ in range(reps):
        out = hom.step_proj(h, c, yt, st)
    torch.cuda.synchronize()
    hom.set_profiling(False)
    ms = sum(t for _, t, _ in hom.profile_read()) / reps
    fl = flops_step_proj(sys_.n, int(np.sum(sys_.m)))
    ok = float((out[2] == 0).float().mean())
    rec = {"points": P, "ms": ms, "points_per_s": P / (ms * 1e-3), "flops_per_point": fl,
           "tflops_algorithmic": P * fl / (ms * 1e-3) / 1e12,
           "frac_of_fp64_peak": P * fl / (ms * 1e-3) / PEAK_FP64, "ok_frac": ok}
    print(f"# step_proj n10 P={P}: {ms:.3f} ms, {rec['points_per_s']:.3e} points/s, "
          f"{rec['tflops_algorithmic']:.2f} TFLOP/s", file=sys.stderr, flush=True)
    return rec


# the paper's own timings (Tables 1-2): wall seconds for 100 consecutive consolidated Euler-Newton
# steps in FP64 by number of points, V100 column (another machine: context only)
PAPER_V100_S = {"ps14": {10: 0.0222, 50: 0.0274, 250: 0.0296, 500: 0.0313, 1000: 0.0355},
                "ps24": {250: 0.0728, 500: 0.0757, 1000: 0.0852}}


def run_paper_shapes(hom, torch, steps=100):
    """100 consecutive consolidated steps (one hom_step, then z <- z + ds dE + dN, s <- s + ds) in
    FP64 on systems of the sizes of the paper's timing systems (n = 14 with 184 monomials, n = 24
    with 324; random, not the systems) at the paper's point counts: wall seconds on the host clock
    around the 100 steps (as the paper times them, launches included) and point-steps/s, beside
    the paper's V100 figures."""
    import numpy as np

    import workloads as W
    out = {}
    for name in ("ps14", "ps24"):
        sys_, z, s = W.config_system(name, P=1000)
        h = hom.System.from_workload(sys_)
        c = torch.tensor(sys_.c, dtype=torch.complex128, device="cuda")
        rec = {}
        for P in (10, 50, 250, 500, 1000):
            z0 = torch.tensor(z[:P], dtype=torch.complex128, device="cuda")
            s0 = torch.tensor(s[:P], dtype=torch.float64, device="cuda")
            ds = 1e-3

            def run(k):
                zt, st = z0, s0
                for _ in range(k):
                    dE, dN, _ = hom.step(h, c, zt, st)
                    zt = zt + ds * dE + dN
                    st = st + ds
                return zt

            run(3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run(steps)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) * 100 / steps
            rec[str(P)] = {"s_per_100_steps": sec, "point_steps_per_s": P * 100 / sec,
                           "paper_v100_s_per_100_steps": PAPER_V100_S[name].get(P)}
        out[name] = {"n": sys_.n, "monomials": int(np.sum(sys_.m)), "by_points": rec}
        print(f"# paper shape {name} (n={sys_.n}, M={int(np.sum(sys_.m))}), s per 100 steps by P: "
              + ", ".join(f"{k}: {v['s_per_100_steps']:.4f} (V100 {v['paper_v100_s_per_100_steps']})"
                          for k, v in rec.items()), file=sys.stderr, flush=True)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(csys, z0, target_s=15.0):
    """The oracle (unchanged) tracking a bounded sample of the same paths on the host cores."""
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    n0 = 256
    t = time.perf_counter()
    _, _, _, _, cnt = oracle.track(csys, csys.c, z0[:n0], -32.0, threads=threads)
    dt = time.perf_counter() - t
    n1 = int(min(len(z0), max(n0, n0 * target_s / max(dt, 1e-3))))
    t = time.perf_counter()
    ze, _, _, st, cnt = oracle.track(csys, csys.c, z0[:n1], -32.0, threads=threads)
    dt = time.perf_counter() - t
    # one thread on a smaller sample (about 5 s)
    n2 = max(16, int(n1 * 5.0 / max(dt * threads, 1e-3)))
    t = time.perf_counter()
    _, _, _, _, cnt1 = oracle.track(csys, csys.c, z0[:n2], -32.0, threads=1)
    dt1 = time.perf_counter() - t
    return {"value": float(cnt[:, 3].sum()) / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"first {n1} of the {len(z0)} paths, tracked s=-32..0 in FP64 "
                      f"({dt:.1f} s, {float(np.mean(st == 0)):.4f} ok)",
            "single_thread_value": float(cnt1[:, 3].sum()) / dt1,
            "single_thread_sample": f"first {n2} paths, {dt1:.1f} s",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}, ze, st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--paths", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense-support (n=32, m=128) eval/step leg")
    ap.add_argument("--dense-points", type=int, default=262144)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched (256 systems) leg")
    ap.add_argument("--no-grad", action="store_true", help="skip the differentiation leg")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also write and then read one 512 MiB buffer (scales the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for "
              f"--gpus {args.gpus}); paths shard across GPUs with no exchange, see DESIGN.md",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2111_14317_amd as hom
    csys, z0 = _workload(args.paths)
    h = hom.System.from_workload(csys)
    if args.copy_calib:  # known traffic for scaling the HBM counters: write 512 MiB, read 512 MiB
        buf = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
        buf.fill_(1.0)  # writes 512 MiB
        torch.cuda.synchronize()
        total = float(torch.sum(buf))  # reads 512 MiB
        torch.cuda.synchronize()
        assert total > 0
        del buf
    res = {}
    # the plain FP64 form, the mixed form, and an FP64 control at the mixed form's corrector
    # tolerance (separates the effect of the precision from that of the tolerance)
    legs = (("fp64", hom.FP64, {}), ("mixed", hom.MIXED, {}),
            ("fp64_tol_track_1e-5", hom.FP64, {"tol_track": 1e-5}),
            ("mixed_hermite", hom.MIXED, {"predictor": hom.PREDICT_HERMITE}),
            ("fp64_hermite", hom.FP64, {"predictor": hom.PREDICT_HERMITE}),
            ("mixed_rk4", hom.MIXED, {"predictor": hom.PREDICT_RK4}))
    for name, prec, kw in legs:
        res[name] = run_form(hom, torch, h, csys, z0, prec, args.steps, args.warmup, **kw)
        print(f"# {name}: {res[name]['rate']:.4e} {UNIT}, {res[name]['ms_per_step']:.2f} ms/step, "
              f"ok {res[name]['ok_frac']:.5f}, {res[name]['evals_per_path']:.1f} evals/path, "
              f"kernels {res[name]['kernels']}", file=sys.stderr, flush=True)
    mixed = res["mixed"]
    dom = f"k_track<{N_EQ},mixed>"
    roof = None
    if dom in mixed["kernels"]:
        dom_ms, dom_units = mixed["kernels"][dom], mixed["units"][dom]
        achieved = dom_units * FLOPS_PER_UNIT / (dom_ms * 1e-3)
        peak = _peak_mixed()
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": measured_traffic(), "kernel": dom, "kernel_ms": dom_ms,
                "kernel_units": dom_units, "flops_per_unit": FLOPS_PER_UNIT}

    def form_rec(r):
        f64_dom = f"k_track<{N_EQ},fp64>"
        frac = None
        if f64_dom in r["kernels"]:
            frac = r["units"][f64_dom] * FLOPS_PER_UNIT / (r["kernels"][f64_dom] * 1e-3) / PEAK_FP64
        return {"value": r["rate"], "ms_per_step": r["ms_per_step"], "ok_frac": r["ok_frac"],
                "statuses_last_step": status_hist(r["status"]),
                "evals_per_path": r["evals_per_path"], "paths_per_s": r["paths_per_s"],
                "kernels_ms": r["kernels"], "kernel_units": r["units"],
                "roofline_frac_fp64_peak": frac}

    out = {
        "metric": METRIC, "value": mixed["rate"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"track {args.paths} planted-cell paths of a random n=10 Laurent "
                               "system (12 monomials/eq, exponents U[-3,3], unit-circle coeffs, "
                               "lifting {0,0,U{1..63}}) from s=-32 to 0, FP64 endgame",
                   "paths": args.paths, "n": N_EQ, "monomials_per_eq": M_EQ},
        "fp64": form_rec(res["fp64"]),
        "mixed": form_rec(mixed),
        "fp64_tol_track_1e-5": form_rec(res["fp64_tol_track_1e-5"]),
        "mixed_hermite": form_rec(res["mixed_hermite"]),
        "fp64_hermite": form_rec(res["fp64_hermite"]),
        "mixed_rk4": form_rec(res["mixed_rk4"]),
        "endpoints_mixed_hermite_vs_fp64": compare_endpoints(res["mixed_hermite"], res["fp64"]),
        "endpoints_mixed_rk4_vs_fp64": compare_endpoints(res["mixed_rk4"], res["fp64"]),
        "endpoints_mixed_vs_fp64": compare_endpoints(mixed, res["fp64"]),
        "endpoints_fp64_tol_track_1e-5_vs_fp64": compare_endpoints(res["fp64_tol_track_1e-5"],
                                                                   res["fp64"]),
        "roofline": roof,
    }
    out["mixed"].pop("roofline_frac_fp64_peak")
    out["mixed_hermite"].pop("roofline_frac_fp64_peak")
    out["mixed_rk4"].pop("roofline_frac_fp64_peak")
    if not args.no_dense:
        out["eval_step_n10_65536_points"] = run_eval_n10(hom, torch, P=65536)
        out["eval_step_n10_1M_points"] = run_eval_n10(hom, torch, P=1 << 20)
        out["dense_n32_m128"] = run_dense(hom, torch, args.dense_points)
        out["common_support_n32_m128"] = run_union(hom, torch, args.dense_points)
        out["start_points_n10_cell"] = run_starts(hom, torch)
        out["step_proj_n10_65536_points"] = run_step_proj(hom, torch)
        out["paper_shapes_100_steps_fp64"] = run_paper_shapes(hom, torch)
    # the units' rates measured on this device (the published peaks stay the roofline denominators)
    peaks = hom.peak_probes()
    out["measured_peaks"] = peaks
    if out.get("roofline"):
        t = (FP64_SHARE / (peaks["fp64_fma_tflops"] * 1e12) +
             (FLOPS_PER_UNIT - FP64_SHARE) / (peaks["fp32_fma_tflops"] * 1e12))
        m_peak = FLOPS_PER_UNIT / t / 1e12
        out["roofline"]["measured_peak"] = m_peak
        out["roofline"]["frac_of_measured_peak"] = out["roofline"]["achieved"] / m_peak
    print(f"# measured peaks: {peaks}", file=sys.stderr, flush=True)
    if not args.no_batch:
        out["batch_c4"] = run_c4(hom, torch)
    c5 = None
    if not args.no_grad:
        c5 = out["grad_c5"] = run_c5(hom, torch)
    if not args.no_cpu:
        out["cpu_baseline"], ora_z, ora_st = cpu_baseline(csys, z0)
        out["mixed_error_vs_oracle"] = error_table(hom, torch, csys, mixed, res["fp64"], ora_z,
                                                   ora_st, c5)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
