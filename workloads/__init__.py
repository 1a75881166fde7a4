"""Seeded synthetic inputs for the polyhedral-homotopy hot path.

This module builds the *inputs* of the hot path and nothing else: random Laurent systems shaped
like the workloads the library is measured on, random evaluation points, planted mixed cells and
the start points of a polyhedral homotopy (roots of the binomial start system, which the paper
treats as given input, Sec. 2 after eq. (1)).  It holds none of the method's arithmetic: no
evaluation of H or its derivatives, no linear solve, no path tracking.  Both the HIP path's tests
and benchmark and the oracle's tests draw their inputs from here.

Conventions (Sec. 2, eq. (1)-(2); Sec. 5.1):
  * a system has n equations in n unknowns; equation k has m_k monomials; M = sum_k m_k;
  * A   int8   [M][n]  exponent vectors, equation-major (equation 0's rows first);
  * w   float64 [M]    lifting values omega_k(a) (non-negative, rational allowed);
  * c   complex128 [M] coefficients;
  * a point is (z, s): z = log x in C^n (any branch), s = log t real, t = 1 <=> s = 0.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from fractions import Fraction

import numpy as np

BASE_SEED = 211114317


# --------------------------------------------------------------------------------------------
# systems
# --------------------------------------------------------------------------------------------
@dataclasses.dataclass
class System:
    """A lifted Laurent system H(x,t) = sum_a c_a x^a t^{w(a)} per equation (eq. (1))."""

    n: int
    m: np.ndarray  # int32 [n]
    A: np.ndarray  # int8 [M][n]
    w: np.ndarray  # float64 [M]
    c: np.ndarray  # complex128 [M]

    def __post_init__(self):
        self.m = np.ascontiguousarray(self.m, dtype=np.int32)
        self.A = np.ascontiguousarray(self.A, dtype=np.int8)
        self.w = np.ascontiguousarray(self.w, dtype=np.float64)
        self.c = np.ascontiguousarray(self.c, dtype=np.complex128)
        assert self.m.shape == (self.n,)
        assert self.A.shape == (self.M, self.n)
        assert self.w.shape == (self.M,) and self.c.shape == (self.M,)

    @property
    def M(self) -> int:
        return int(self.m.sum())

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.m)]).astype(np.int64)

    def equation(self, k: int) -> slice:
        off = self.offsets
        return slice(int(off[k]), int(off[k + 1]))

    def with_lifting(self, w) -> "System":
        return System(self.n, self.m.copy(), self.A.copy(), np.asarray(w, np.float64), self.c.copy())

    def with_coefficients(self, c) -> "System":
        return System(self.n, self.m.copy(), self.A.copy(), self.w.copy(), np.asarray(c, np.complex128))


def _distinct_rows(rng, m, n, draw):
    """m distinct exponent vectors (sampling without replacement)."""
    rows, seen = [], set()
    while len(rows) < m:
        r = tuple(int(v) for v in draw(rng, n))
        if r not in seen:
            seen.add(r)
            rows.append(r)
    return rows


def _uniform_exps(lo, hi):
    return lambda rng, n: rng.integers(lo, hi + 1, size=n)


def _sparse_exps(bound, zero_frac):
    nz = np.array([v for v in range(-bound, bound + 1) if v != 0])

    def draw(rng, n):
        v = rng.choice(nz, size=n)
        v[rng.random(n) < zero_frac] = 0
        return v

    return draw


def _coefficients(rng, M, kind):
    if kind == "unit":
        return np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, size=M))
    if kind == "gauss":  # complex Gaussian with E|c|^2 = 1
        return (rng.normal(0.0, math.sqrt(0.5), M) + 1j * rng.normal(0.0, math.sqrt(0.5), M))
    raise ValueError(kind)


def random_system(n, m, draw_exps, coef_kind, lift_hi, rng_sup, rng_coef, rng_lift) -> System:
    m = np.full(n, m, dtype=np.int32) if np.isscalar(m) else np.asarray(m, np.int32)
    rows = []
    for k in range(n):
        rows += _distinct_rows(rng_sup, int(m[k]), n, draw_exps)
    A = np.array(rows, dtype=np.int8).reshape(-1, n)
    M = A.shape[0]
    c = _coefficients(rng_coef, M, coef_kind)
    w = rng_lift.integers(0, lift_hi + 1, size=M).astype(np.float64)
    return System(n, m, A, w, c)


def union_system(n, m, draw_exps, coef_kind, lift_hi, rng_sup, rng_coef, rng_lift) -> System:
    """A system with one common support (the unmixed case of Sec. 5.1): m distinct exponent
    vectors and their liftings shared by every equation (listed in the same order), and an
    independent coefficient for every (equation, monomial)."""
    rows = _distinct_rows(rng_sup, m, n, draw_exps)
    S = np.array(rows, dtype=np.int8).reshape(m, n)
    w = rng_lift.integers(0, lift_hi + 1, size=m).astype(np.float64)
    A = np.tile(S, (n, 1))
    c = _coefficients(rng_coef, n * m, coef_kind)
    return System(n, np.full(n, m, np.int32), A, np.tile(w, n), c)


def union_config(P: int | None = None, n: int = 32, m: int = 128):
    """The dense configuration's shapes (exponents in [-4, 4] with 30% zeros, complex Gaussian
    coefficients, liftings U{0..255}, points as the other configurations) with one support common
    to all equations; P = 262144 by default."""
    r_sup, r_coef, r_lift, r_pts, _, _ = streams("c3")
    r_sup = np.random.default_rng(r_sup.integers(2 ** 63))  # a stream of its own
    sys = union_system(n, m, _sparse_exps(4, 0.3), "gauss", 255, r_sup, r_coef, r_lift)
    z, s = random_points(n, 262144 if P is None else P, r_pts)
    return sys, z, s


def random_points(n, P, rng, s_lo=-8.0, s_hi=0.0):
    """Re z ~ N(0, 0.5), Im z ~ U[0, 2 pi), s ~ U[s_lo, s_hi]."""
    z = rng.normal(0.0, 0.5, size=(P, n)) + 1j * rng.uniform(0.0, 2.0 * np.pi, size=(P, n))
    s = rng.uniform(s_lo, s_hi, size=P)
    return np.ascontiguousarray(z), np.ascontiguousarray(s)


# --------------------------------------------------------------------------------------------
# the five workload configurations (small tiny case first)
# --------------------------------------------------------------------------------------------
CONFIGS = {
    "c1": dict(n=3, m=4, exps=("u", -2, 2), coef="unit", lift=31, P=4096),
    "c2": dict(n=10, m=12, exps=("u", -3, 3), coef="unit", lift=63, P=65536),
    "c3": dict(n=32, m=128, exps=("z", 4, 0.3), coef="gauss", lift=255, P=262144),
    "c5": dict(n=8, m=16, exps=("u", -2, 2), coef="unit", lift=31, P=16384),
    # the sizes of the paper's timing systems (Tables 1-2: n = 14 with 184 monomials, n = 24 with
    # 324), not the systems: monomials split as evenly as possible over the equations, 0/1
    # exponents (each entry 1 with probability 0.3), up to 1000 points
    "ps14": dict(n=14, m=[14] * 2 + [13] * 12, exps=("b", 0.3), coef="unit", lift=31, P=1000),
    "ps24": dict(n=24, m=[14] * 12 + [13] * 12, exps=("b", 0.3), coef="unit", lift=31, P=1000),
}
CONFIG_INDEX = {"c1": 0, "c2": 1, "c3": 2, "c4": 3, "c5": 4, "ps14": 5, "ps24": 6}


def streams(cfg: str):
    """Six independent streams: supports, coefficients, lifting, points, start subset, spare."""
    ss = np.random.SeedSequence(BASE_SEED + CONFIG_INDEX[cfg]).spawn(6)
    return [np.random.default_rng(s) for s in ss]


def _draw_for(spec):
    kind = spec[0]
    if kind == "u":
        return _uniform_exps(spec[1], spec[2])
    if kind == "b":  # 0/1 entries, 1 with probability spec[1]
        return lambda rng, n: (rng.random(n) < spec[1]).astype(np.int64)
    return _sparse_exps(spec[1], spec[2])


def config_system(cfg: str, P: int | None = None):
    """System and random evaluation points of configuration `cfg` ('c1', 'c2', 'c3', 'c5', 'ps14',
    'ps24')."""
    spec = CONFIGS[cfg]
    r_sup, r_coef, r_lift, r_pts, _, _ = streams(cfg)
    sys = random_system(spec["n"], spec["m"], _draw_for(spec["exps"]), spec["coef"], spec["lift"],
                        r_sup, r_coef, r_lift)
    z, s = random_points(sys.n, spec["P"] if P is None else P, r_pts)
    return sys, z, s


def c4_systems(num_sys=256, P_lo=512, P_hi=4096, W=63, min_det=None):
    """Batched uneven instances: n ~ U{6..24}, m ~ U{8..64} per system, exponents U{-3..3},
    unit-circle coefficients, one planted cell per system (lifting {0,0,U{1..W}})."""
    r_sup, r_coef, r_lift, r_pts, r_sub, r_spare = streams("c4")
    out = []
    for _ in range(num_sys):
        n = int(r_spare.integers(6, 25))
        m = int(r_spare.integers(8, 65))
        P = int(r_spare.integers(P_lo, P_hi + 1))
        sys = random_system(n, m, _uniform_exps(-3, 3), "unit", W, r_sup, r_coef, r_lift)
        cell_sys, cell = plant_cell(sys, W, r_lift, min_det=P if min_det is None else min_det)
        z0 = binomial_start_points(cell_sys, cell, P, r_sub)
        out.append((cell_sys, cell, z0))
    return out


def stack_batch(systems, starts):
    """The arrays of a batched call: start points zero padded to the largest n (z [P][n_max]),
    each path's system index (non-decreasing) and the concatenated coefficients."""
    n_max = max(s.n for s in systems)
    P = sum(len(z0) for z0 in starts)
    z = np.zeros((P, n_max), np.complex128)
    idx = np.concatenate([np.full(len(z0), q, np.int32) for q, z0 in enumerate(starts)])
    row = 0
    for z0 in starts:
        z[row:row + len(z0), :z0.shape[1]] = z0
        row += len(z0)
    c = np.concatenate([s.c for s in systems])
    return z, idx, c


# --------------------------------------------------------------------------------------------
# integer Smith normal form  U D V = diag(sigma), U, V unimodular
# --------------------------------------------------------------------------------------------
def smith_normal_form(D):
    """Integer Smith normal form by elementary row/column operations (Python ints, exact)."""
    D = [[int(v) for v in row] for row in np.asarray(D)]
    n = len(D)
    U = [[int(i == j) for j in range(n)] for i in range(n)]
    V = [[int(i == j) for j in range(n)] for i in range(n)]

    def swap_rows(X, i, j):
        X[i], X[j] = X[j], X[i]

    def swap_cols(X, i, j):
        for row in X:
            row[i], row[j] = row[j], row[i]

    def add_row(X, dst, src, f):  # row dst += f * row src
        X[dst] = [a + f * b for a, b in zip(X[dst], X[src])]

    def add_col(X, dst, src, f):  # col dst += f * col src
        for row in X:
            row[dst] += f * row[src]

    for t in range(n):
        while True:
            # pivot = smallest nonzero |entry| in the trailing block
            best = None
            for i in range(t, n):
                for j in range(t, n):
                    if D[i][j] != 0 and (best is None or abs(D[i][j]) < abs(D[best[0]][best[1]])):
                        best = (i, j)
            if best is None:
                raise ValueError("singular matrix")
            i, j = best
            swap_rows(D, t, i); swap_rows(U, t, i)
            swap_cols(D, t, j); swap_cols(V, t, j)
            done = True
            for i in range(t + 1, n):
                q = D[i][t] // D[t][t]
                if q:
                    add_row(D, i, t, -q); add_row(U, i, t, -q)
                if D[i][t] != 0:
                    done = False
            for j in range(t + 1, n):
                q = D[t][j] // D[t][t]
                if q:
                    add_col(D, j, t, -q); add_col(V, j, t, -q)
                if D[t][j] != 0:
                    done = False
            if not done:
                continue
            # divisibility: pivot must divide the whole trailing block
            bad = None
            for i in range(t + 1, n):
                for j in range(t + 1, n):
                    if D[i][j] % D[t][t] != 0:
                        bad = i
                        break
                if bad is not None:
                    break
            if bad is None:
                break
            add_row(D, t, bad, 1); add_row(U, t, bad, 1)
        if D[t][t] < 0:
            D[t] = [-v for v in D[t]]
            U[t] = [-v for v in U[t]]
    sigma = [D[i][i] for i in range(n)]
    return U, sigma, V


# --------------------------------------------------------------------------------------------
# binomial start systems
# --------------------------------------------------------------------------------------------
def _randbelow(rng, bound):
    """Seeded integer in [0, bound) for Python-int bounds of any size."""
    if bound <= 2 ** 62:
        return int(rng.integers(0, bound))
    v, span = 0, 1
    while span < bound * 2 ** 32:
        v = v * 2 ** 62 + int(rng.integers(0, 2 ** 62))
        span *= 2 ** 62
    return v % bound


def binomial_roots(Dmat, beta, count, rng):
    """`count` distinct roots of x^{d_k} = beta_k (rows d_k of Dmat), as z = log x.

    With U D V = S = diag(sigma): D z = log(beta) + 2 pi i k, and the |det D| distinct roots are
    z = V w,  w_j = ((U b)_j + 2 pi i j_j) / sigma_j,  j_j in [0, sigma_j),  b = log(beta).
    Imaginary parts are reduced into [-pi, pi).  Roots are chosen in a seeded order.
    """
    U, sigma, V = smith_normal_form(Dmat)
    n = len(sigma)
    total = 1
    for v in sigma:
        total *= v
    if count > total:
        raise ValueError(f"only {total} roots, {count} requested")
    if total <= 4 * count:
        idx = [int(v) for v in rng.permutation(total)[:count]]
        ks = []
        for q in idx:
            k = []
            for sg in sigma:
                k.append(q % sg)
                q //= sg
            ks.append(tuple(k))
    else:
        seen, ks = set(), []
        while len(ks) < count:
            k = tuple(_randbelow(rng, sg) if sg > 1 else 0 for sg in sigma)
            if k not in seen:
                seen.add(k)
                ks.append(k)
    # U and V can hold huge entries, so they never touch floating point: one root comes from a
    # float solve with the principal log, and the others differ from it by 2 pi i V S^{-1} j,
    # whose fractional part is formed exactly in integers (every sigma_l divides sigma_{n-1}).
    b = np.log(np.asarray(beta, np.complex128))
    z_base = np.linalg.solve(np.asarray(Dmat, np.float64), b)
    L = sigma[-1]
    # only coordinates with sigma_l > 1 take nonzero k_l; fold V's columns for them mod L once
    live = [l for l in range(n) if sigma[l] > 1]
    cols = {l: [(V[i][l] * (L // sigma[l])) % L for i in range(n)] for l in live}
    z = np.empty((len(ks), n), dtype=np.complex128)
    for q, k in enumerate(ks):
        num = [0] * n
        for l in live:
            if k[l]:
                col = cols[l]
                num = [a + k[l] * b for a, b in zip(num, col)]
        z[q] = z_base + 2j * np.pi * np.array([(v % L) / L for v in num])
    z = z.real + 1j * (np.mod(z.imag + np.pi, 2.0 * np.pi) - np.pi)
    return np.ascontiguousarray(z)


def cell_binomial(sys: System, cell):
    """The binomial start system of a mixed cell: rows d_k = a_{k,j1} - a_{k,j0} and
    beta_k = -c_{k,j0} / c_{k,j1}; cell = [(j0, j1)] per equation (indices within equation k)."""
    off = sys.offsets
    D = np.zeros((sys.n, sys.n), dtype=np.int64)
    beta = np.zeros(sys.n, dtype=np.complex128)
    for k, (j0, j1) in enumerate(cell):
        i0, i1 = off[k] + j0, off[k] + j1
        D[k] = sys.A[i1].astype(np.int64) - sys.A[i0].astype(np.int64)
        beta[k] = -sys.c[i0] / sys.c[i1]
    return D, beta


def binomial_start_points(sys: System, cell, count, rng):
    D, beta = cell_binomial(sys, cell)
    return binomial_roots(D, beta, count, rng)


def int_det(D) -> int:
    """Exact integer determinant (fraction-free Bareiss elimination)."""
    M = [[int(v) for v in row] for row in np.asarray(D)]
    n = len(M)
    sign, prev = 1, 1
    for k in range(n - 1):
        if M[k][k] == 0:
            for i in range(k + 1, n):
                if M[i][k] != 0:
                    M[k], M[i] = M[i], M[k]
                    sign = -sign
                    break
            else:
                return 0
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                M[i][j] = (M[i][j] * M[k][k] - M[i][k] * M[k][j]) // prev
        prev = M[k][k]
    return sign * M[n - 1][n - 1]


def plant_cell(sys: System, W: int, rng, min_det: int = 1, max_tries: int = 10000):
    """Planted mixed cell: per equation a pair gets lifting 0 and the other monomials U{1..W}.

    The pair is then a mixed cell with inner normal (0, 1): <a, 0> + w(a) = w(a) > 0 = beta_k for
    every other a.  Pairs are redrawn until |det D| >= min_det.
    Returns (system with the planted lifting, cell) with cell[k] = (j0, j1) within equation k.
    """
    for _ in range(max_tries):
        cell = []
        for k in range(sys.n):
            j0, j1 = sorted(int(v) for v in rng.choice(int(sys.m[k]), size=2, replace=False))
            cell.append((j0, j1))
        D, _ = cell_binomial(sys, cell)
        if abs(int_det(D)) >= min_det:
            break
    else:
        raise RuntimeError("no planted cell with large enough |det D|")
    w = rng.integers(1, W + 1, size=sys.M).astype(np.float64)
    off = sys.offsets
    for k, (j0, j1) in enumerate(cell):
        w[off[k] + j0] = 0.0
        w[off[k] + j1] = 0.0
    return sys.with_lifting(w), cell


# --------------------------------------------------------------------------------------------
# brute-force mixed cells (tiny systems) and per-cell homotopies
# --------------------------------------------------------------------------------------------
class NonGenericLifting(Exception):
    pass


def _solve_rational(D, rhs):
    n = len(rhs)
    M = [[Fraction(int(D[i][j])) for j in range(n)] + [Fraction(rhs[i])] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def mixed_cells_bruteforce(sys: System):
    """All fine mixed cells of the lifted supports, by enumerating one pair per equation.

    A choice of pairs is a cell when the inner normal alpha solving
    <a_{k,1} - a_{k,0}, alpha> = w_{k,0} - w_{k,1} makes the pair the unique minimisers of
    <a, alpha> + w_k(a) over S_k.  Ties mean the lifting is not generic (raises).
    Liftings must be integers.  Returns a list of dicts (cell, alpha, beta, det).
    """
    n = sys.n
    off = sys.offsets
    wq = [Fraction(int(v)) for v in sys.w]
    pairs = [list(itertools.combinations(range(int(sys.m[k])), 2)) for k in range(n)]
    cells = []
    for choice in itertools.product(*pairs):
        D, _ = cell_binomial(sys, choice)
        det = int_det(D)
        if det == 0:
            continue
        rhs = [wq[off[k] + j0] - wq[off[k] + j1] for k, (j0, j1) in enumerate(choice)]
        alpha = _solve_rational(D, rhs)
        ok = True
        betas = []
        for k, (j0, j1) in enumerate(choice):
            sl = range(int(off[k]), int(off[k + 1]))
            vals = {i: sum(alpha[j] * int(sys.A[i][j]) for j in range(n)) + wq[i] for i in sl}
            beta = vals[off[k] + j0]
            assert beta == vals[off[k] + j1]
            for i in sl:
                if i in (off[k] + j0, off[k] + j1):
                    continue
                if vals[i] < beta:
                    ok = False
                    break
                if vals[i] == beta:
                    raise NonGenericLifting(f"tie in equation {k}")
            if not ok:
                break
            betas.append(beta)
        if ok:
            cells.append(dict(cell=list(choice), alpha=alpha, beta=betas, det=abs(det)))
    return cells


def generic_lifting_cells(sys: System, rng_lift, lift_hi, max_redraws=100):
    """Redraw integer liftings U{0..lift_hi} until the brute-force enumeration has no ties."""
    cur = sys
    for _ in range(max_redraws):
        try:
            return cur, mixed_cells_bruteforce(cur)
        except NonGenericLifting:
            cur = sys.with_lifting(rng_lift.integers(0, lift_hi + 1, size=sys.M).astype(np.float64))
    raise RuntimeError("no generic lifting found")


def cell_homotopy(sys: System, cell_info):
    """Per-cell lifting w'_k(a) = <a, alpha> + w_k(a) - beta_k (>= 0, zero on the pair), scaled
    so the smallest positive value is 1.  x = y t^alpha maps the paths of the cell's homotopy to
    those of eq. (1); at t = 1 both coordinates agree."""
    alpha, betas = cell_info["alpha"], cell_info["beta"]
    off = sys.offsets
    wq = []
    for k in range(sys.n):
        for i in range(int(off[k]), int(off[k + 1])):
            v = sum(alpha[j] * int(sys.A[i][j]) for j in range(sys.n)) + Fraction(int(sys.w[i])) - betas[k]
            assert v >= 0
            wq.append(v)
    pos = min(v for v in wq if v > 0)
    w = np.array([float(v / pos) for v in wq], dtype=np.float64)
    return sys.with_lifting(w)


def c1_cells():
    """Configuration c1 with a generic lifting, its mixed cells and every cell's start points.
    Returns (system, [(cell_system, cell_info, z_start)])."""
    r_sup, r_coef, r_lift, r_pts, r_sub, _ = streams("c1")
    spec = CONFIGS["c1"]
    sys = random_system(spec["n"], spec["m"], _draw_for(spec["exps"]), spec["coef"], spec["lift"],
                        r_sup, r_coef, r_lift)
    sys, cells = generic_lifting_cells(sys, r_lift, spec["lift"])
    out = []
    for info in cells:
        csys = cell_homotopy(sys, info)
        z0 = binomial_start_points(csys, info["cell"], info["det"], r_sub)
        out.append((csys, info, z0))
    return sys, out


def planted_config(cfg: str, P: int | None = None, W: int | None = None):
    """Tracking workload of `cfg`: the configuration's system with a planted cell and P start
    points (roots of the cell's binomial system)."""
    spec = CONFIGS[cfg]
    r_sup, r_coef, r_lift, r_pts, r_sub, _ = streams(cfg)
    sys = random_system(spec["n"], spec["m"], _draw_for(spec["exps"]), spec["coef"], spec["lift"],
                        r_sup, r_coef, r_lift)
    P = spec["P"] if P is None else P
    W = spec["lift"] if W is None else W
    csys, cell = plant_cell(sys, W, r_lift, min_det=P)
    z0 = binomial_start_points(csys, cell, P, r_sub)
    return csys, cell, z0
