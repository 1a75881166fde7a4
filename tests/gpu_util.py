"""Helpers of the GPU parity tests (no library arithmetic)."""
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def eval_err(G_gpu, L_gpu, G_ora, L_ora, den):
    """componentwise scaled error |G_gpu e^{L_gpu - L_ora} - G_ora| / den (den = sum |terms| |C|)"""
    Gg = G_gpu * np.exp(L_gpu - L_ora)[:, :, None]
    diff = np.abs(Gg - G_ora)
    return np.where(den > 0, diff / np.where(den > 0, den, 1.0), diff)


def eval_err_fp32(G_gpu, L_gpu, G_ora, L_ora, den, floor=1e-30):
    """Error metric of the FP32 evaluation: as eval_err, with each column's scale floored at
    `floor` times the row's total term mass sum_a |V_a| (the last column of den).  FP32 cannot
    hold terms below ~1e-38 of a row's largest one, so columns whose whole mass lies there are
    flushed; they are irrelevant at FP32 precision."""
    Gg = G_gpu * np.exp(L_gpu - L_ora)[:, :, None]
    scale = np.maximum(den, floor * den[:, :, -1:])
    return np.abs(Gg - G_ora) / np.where(scale > 0, scale, 1.0)


def cond_inf(sys, c, z, s):
    G, _ = oracle.eval(sys, c, z, s)
    J = G[:, :, :sys.n]
    return np.linalg.cond(J, p=np.inf)


def torch_params(hom, p_oracle, precision):
    """library params with the oracle's constants"""
    kw = {f: getattr(p_oracle, f) for f in ("ds0", "ds_max", "ds_min", "tol_polish", "tol_track",
                                            "tol_end", "res_tol", "div_re", "sing_ratio", "max_polish",
                                            "max_newton", "max_end", "max_steps", "max_iters")}
    return hom.default_params(precision, **kw)


def mod2pi_dist(a, b):
    """max-modulus distance of log points modulo 2 pi i"""
    dre = np.abs(a.real - b.real)
    dim = np.abs(np.angle(np.exp(1j * (a.imag - b.imag))))
    return np.maximum(dre, dim).max(axis=-1)
