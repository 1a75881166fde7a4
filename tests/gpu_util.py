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
                                            "tol_end", "res_tol", "div_re", "sing_ratio", "tol_predict", "predictor", "max_polish",
                                            "max_newton", "max_end", "max_steps", "max_iters")}
    return hom.default_params(precision, **kw)


def mod2pi_dist(a, b):
    """max-modulus distance of log points modulo 2 pi i"""
    dre = np.abs(a.real - b.real)
    dim = np.abs(np.angle(np.exp(1j * (a.imag - b.imag))))
    return np.maximum(dre, dim).max(axis=-1)


def _projection(z, seed=20211129):
    """A fixed random positive combination of Re z_j, cos Im z_j and sin Im z_j per point, and the
    sum of its weights W: two points within d of each other (max modulus, modulo 2 pi i) project
    to within W d, since cos and sin are 1-Lipschitz."""
    rng = np.random.default_rng(seed)
    n = z.shape[1]
    wr, wc, ws = (rng.uniform(0.5, 1.0, n) for _ in range(3))
    return z.real @ wr + np.cos(z.imag) @ wc + np.sin(z.imag) @ ws, wr.sum() + wc.sum() + ws.sum()


def _window_pairs(pa, pb_sorted, radius):
    """For each value of pa, the index range [lo, hi) of pb_sorted within radius."""
    lo = np.searchsorted(pb_sorted, pa - radius, side="left")
    hi = np.searchsorted(pb_sorted, pa + radius, side="right")
    return lo, hi


def nearest_mod2pi(a, b, radius=1e-6):
    """For each row of a: the smallest mod2pi_dist to a row of b among the rows within `radius`
    (inf when there is none) and that row's index (-1).  Candidates come from a 1-D projection
    (sorted, windowed), then the exact distance is taken."""
    a = np.asarray(a)
    b = np.asarray(b)
    d_out = np.full(len(a), np.inf)
    j_out = np.full(len(a), -1, np.int64)
    if len(a) == 0 or len(b) == 0:
        return d_out, j_out
    pa, W = _projection(a)
    pb, _ = _projection(b)
    order = np.argsort(pb)
    pbs = pb[order]
    lo, hi = _window_pairs(pa, pbs, radius * W)
    width = hi - lo
    for k in range(int(width.max(initial=0))):
        has = width > k
        idx = np.nonzero(has)[0]
        cand = order[lo[idx] + k]
        d = mod2pi_dist(a[idx], b[cand])
        better = d < d_out[idx]
        d_out[idx[better]] = d[better]
        j_out[idx[better]] = cand[better]
    return d_out, j_out


def distinct_count(z, tol=1e-8):
    """number of endpoints that are pairwise more than tol apart modulo 2 pi i (a point is a
    duplicate when an earlier point lies within tol)"""
    z = np.asarray(z)
    if len(z) == 0:
        return 0
    p, W = _projection(z)
    order = np.argsort(p)
    ps = p[order]
    dup = np.zeros(len(z), bool)
    k = 1
    while True:
        near = ps[k:] - ps[:-k] <= tol * W if k < len(ps) else np.zeros(0, bool)
        if not near.any():
            break
        i, j = order[:-k][near], order[k:][near]
        close = mod2pi_dist(z[i], z[j]) <= tol
        later = np.maximum(i, j)[close]
        dup[later] = True
        k += 1
    return int((~dup).sum())


def status_hist(st):
    u, c = np.unique(np.asarray(st), return_counts=True)
    return {int(a): int(b) for a, b in zip(u, c)}


def _kappa_end(sys_, z):
    """condition number of J_z at endpoints (t = 1), from the oracle's evaluation"""
    G, _ = oracle.eval(sys_, sys_.c, z, np.zeros(len(z)))
    return np.abs(np.linalg.cond(G[:, :, :sys_.n], p=np.inf))


def check_fp64_per_path(sys_, zg, sg, zo, so, label, max_excluded=0.0):
    """FP64 tracker against the oracle's tracker, path by path: the same status on every path, and
    endpoints within 1e-12 (max modulus, modulo 2 pi i) on every path that ends OK with a
    well-conditioned endpoint (kappa <= 1e4; the excluded count is asserted small)."""
    assert np.array_equal(sg, so), (label, status_hist(sg), status_hist(so))
    ok = sg == 0
    kap = _kappa_end(sys_, zo)
    keep = ok & (kap <= 1e4)
    d = mod2pi_dist(zg, zo)
    say(f"  {label}: statuses {status_hist(sg)}, kappa > 1e4 at {int((ok & ~keep).sum())} OK endpoints, "
        f"max d {d[keep].max() if keep.any() else 0:.2e}")
    assert (ok & ~keep).sum() <= max_excluded * len(sg)
    assert d[keep].max(initial=0.0) <= 1e-12
    return d


def check_mixed_set(sys_, zg, sg, zo, so, label, min_ok=0.999, max_swaps=0.0):
    """Mixed tracker against the oracle's FP64 tracker: at least `min_ok` of the paths end OK,
    every OK endpoint is a root (residual <= 1e-10), the OK endpoints are pairwise distinct, and
    each lies within 1e-10 (modulo 2 pi i) of an OK oracle endpoint with kappa <= 1e4 (endpoints
    are compared as sets: a path that ends on another path's root is counted as a swap).  Returns
    the number of swaps."""
    ok = sg == 0
    say(f"  {label}: statuses {status_hist(sg)} (oracle {status_hist(so)})")
    assert ok.mean() >= min_ok, status_hist(sg)
    assert oracle.residual(sys_, sys_.c, zg[ok]).max(initial=0.0) <= 1e-10
    zgo = zg[ok]
    assert distinct_count(zgo) == len(zgo)
    ref_ok = so == 0
    kap = _kappa_end(sys_, zo[ref_ok])
    d, j = nearest_mod2pi(zgo, zo[ref_ok])
    assert (j >= 0).all(), "an OK endpoint with no oracle endpoint near it"
    well = kap[j] <= 1e4
    say(f"    set match: max d {d[well].max() if well.any() else 0:.2e} over {int(well.sum())} "
        f"(kappa > 1e4: {int((~well).sum())})")
    assert (~well).sum() <= 1e-3 * len(sg) + 1
    assert d[well].max(initial=0.0) <= 1e-10
    swaps = int((mod2pi_dist(zgo, zo[ok]) > 1e-10).sum())
    say(f"    paths ending on another path's root: {swaps}")
    assert swaps <= max_swaps * len(sg)
    return swaps


def dir_bound(kappa, n, unit_roundoff, floor):
    """Forward-error bound of directions from one LU with partial pivoting at every point:
    max(floor, 16 n u kappa), the backward error of the elimination (n u times a growth factor)
    together with the evaluation's rounding, amplified by the condition number (16 covers the
    growth factor and the evaluation)."""
    return np.maximum(floor, 16.0 * n * unit_roundoff * np.abs(np.asarray(kappa)))


def proj_kappa(sys_, y, s):
    """kappa_inf of the row-equilibrated projective system [dH~/dy; y^*] at points y [P][n+1]:
    dH~/dy at y = y_n (x, 1) from the affine evaluation (columns J_z / x, and the homogenising
    column from Euler's identity d_k h_k - sum_j (J_z)_kj), rows normalised."""
    n = sys_.n
    x = y[:, :n] / y[:, n:]
    z = np.log(x)
    G, _ = oracle.eval(sys_, sys_.c, z, np.broadcast_to(s, (len(y),)))
    Jz, H = G[:, :, :n], G[:, :, n + 1]
    d = np.array([int(sys_.A[sys_.equation(k)].astype(int).sum(1).max()) for k in range(n)])
    J = np.zeros((len(y), n + 1, n + 1), complex)
    J[:, :n, :n] = Jz / x[:, None, :]
    J[:, :n, n] = d[None, :] * H - Jz.sum(2)
    J[:, n, :] = np.conj(np.concatenate([x, np.ones((len(y), 1))], axis=1))
    J /= np.abs(J).sum(2, keepdims=True)
    return np.linalg.cond(J, p=np.inf)


def dir_err(a, b):
    """per-point max-norm relative error of directions"""
    return np.abs(a - b).max(1) / np.maximum(np.abs(b).max(1), 1e-300)


def check_dirs(dE, dN, oE, oN, ost, kappa, mixed, n, label="", min_well=0):
    """Every nonsingular point within the LU's forward-error bound dir_bound (kappa times 16 n u,
    u the unit roundoff of the solve's precision; points whose FP32 pivot ratio is below 1e-4 are
    redone in FP64 by the mixed form), and the well-conditioned ones (kappa <= 1e3 in FP64, 1e2
    mixed) within 1e-12 / 1e-5; at least `min_well` of them.  Dense n >= 20 Jacobians at random
    points rarely have kappa <= 1e2."""
    kappa = np.abs(np.asarray(kappa))
    fin = (ost == 0) & np.isfinite(kappa)
    e = np.maximum(dir_err(dE, oE), dir_err(dN, oN))
    tol, kmax, u = (1e-5, 1e2, 2.0 ** -24) if mixed else (1e-12, 1e3, 2.0 ** -53)
    well = (kappa <= kmax) & fin
    bound = dir_bound(kappa, n, u, tol)
    say(f"  {label} kappa<={kmax:g}: {well.sum()}/{len(e)} max err {e[well].max(initial=0):.3e}; "
        f"all {fin.sum()}: max err/bound {(e / bound)[fin].max(initial=0):.2e}, "
        f"max err/kappa {(e / np.maximum(kappa, 1))[fin].max(initial=0):.2e}")
    assert well.sum() >= min_well
    assert e[well].max(initial=0.0) <= tol
    assert (e[fin] <= bound[fin]).all()
