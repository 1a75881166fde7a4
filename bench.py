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


def run_form(hom, torch, h, csys, z0, precision, steps, warmup):
    """Returns dict with rate, ms/step, ok fraction, mean evals/path and kernel timings."""
    dev = "cuda"
    P = z0.shape[0]
    c = torch.tensor(csys.c, dtype=torch.complex128, device=dev)
    z_init = torch.tensor(z0, dtype=torch.complex128, device=dev)
    params = hom.default_params(precision)
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
    return dict(rate=evals / sec, ms_per_step=1e3 * sec / steps, ok_frac=min(ok),
                evals_per_path=sum(evals_per_path) / len(evals_per_path),
                evals_per_step=evals / steps, kernels=kern, units=units,
                launches={k: v / steps for k, v in launches.items()}, paths_per_s=P * steps / sec)


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
    _, _, _, st, cnt = oracle.track(csys, csys.c, z0[:n1], -32.0, threads=threads)
    dt = time.perf_counter() - t
    return {"value": float(cnt[:, 3].sum()) / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"first {n1} of the {len(z0)} paths, tracked s=-32..0 in FP64 "
                      f"({dt:.1f} s, {float(np.mean(st == 0)):.4f} ok)"}


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
    for name, prec in (("fp64", hom.FP64), ("mixed", hom.MIXED)):
        res[name] = run_form(hom, torch, h, csys, z0, prec, args.steps, args.warmup)
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
    f64 = res["fp64"]
    f64_dom = f"k_track<{N_EQ},fp64>"
    f64_frac = None
    if f64_dom in f64["kernels"]:
        f64_frac = f64["units"][f64_dom] * FLOPS_PER_UNIT / (f64["kernels"][f64_dom] * 1e-3) / PEAK_FP64
    out = {
        "metric": METRIC, "value": mixed["rate"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"track {args.paths} planted-cell paths of a random n=10 Laurent "
                               "system (12 monomials/eq, exponents U[-3,3], unit-circle coeffs, "
                               "lifting {0,0,U{1..63}}) from s=-32 to 0, FP64 endgame",
                   "paths": args.paths, "n": N_EQ, "monomials_per_eq": M_EQ},
        "fp64": {"value": res["fp64"]["rate"], "ms_per_step": res["fp64"]["ms_per_step"],
                 "ok_frac": res["fp64"]["ok_frac"], "evals_per_path": res["fp64"]["evals_per_path"],
                 "paths_per_s": res["fp64"]["paths_per_s"], "kernels_ms": res["fp64"]["kernels"],
                 "kernel_units": res["fp64"]["units"], "roofline_frac_fp64_peak": f64_frac},
        "mixed": {"value": mixed["rate"], "ms_per_step": mixed["ms_per_step"],
                  "ok_frac": mixed["ok_frac"], "evals_per_path": mixed["evals_per_path"],
                  "paths_per_s": mixed["paths_per_s"], "kernels_ms": mixed["kernels"],
                  "kernel_units": mixed["units"]},
        "roofline": roof,
    }
    if not args.no_dense:
        out["eval_step_n10_65536_points"] = run_eval_n10(hom, torch, P=65536)
        out["eval_step_n10_1M_points"] = run_eval_n10(hom, torch, P=1 << 20)
        out["dense_n32_m128"] = run_dense(hom, torch, args.dense_points)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(csys, z0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
