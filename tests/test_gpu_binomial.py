"""GPU start points (Sec. 2: the roots of each mixed cell's binomial system) against the oracle:
the whole root set of every cell, compared as sets (the two enumerate the roots in different
orders), and at full size through properties that hold at any size."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hom():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    import paper_2111_14317_amd as hom
    return hom


def _residual(D, beta, z):
    return (np.abs(np.exp(z @ np.asarray(D, np.float64).T) - beta[None, :]) / np.abs(beta)).max(1)


def _match(a, b, tol):
    """every row of a within tol of a row of b (Im mod 2 pi), one to one"""
    assert a.shape == b.shape
    key = lambda z: np.round(np.concatenate([z.real, np.mod(z.imag, 2 * np.pi)], 1) * 1e6)
    ib = {tuple(r): k for k, r in enumerate(key(b))}
    used = np.zeros(len(b), bool)
    worst = 0.0
    for k, r in enumerate(key(a)):
        j = ib.get(tuple(r))
        if j is None:  # rounding at a key boundary: nearest by search
            d = np.maximum(np.abs(b.real - a[k].real), np.abs(np.angle(np.exp(1j * (b.imag - a[k].imag))))).max(1)
            j = int(d.argmin())
        d = max(np.abs(b[j].real - a[k].real).max(), np.abs(np.angle(np.exp(1j * (b[j].imag - a[k].imag)))).max())
        worst = max(worst, d)
        assert not used[j], "two roots match one oracle root"
        used[j] = True
    assert worst <= tol, worst
    return worst


def _cell(rng, n, max_det):
    """A nonsingular integer D with 1 < |det D| <= max_det and its beta: rejection sampling of
    entries in [-3, 3] for n <= 4; above, D = L U with L unit lower triangular and U upper
    triangular (off the diagonals, entries in [-1, 1] with density 2 / n, so that D stays well
    conditioned; U's diagonal from {1, 2, 3}), rows and columns permuted."""
    beta = rng.normal(size=n) + 1j * rng.normal(size=n)
    if n <= 4:
        while True:
            D = rng.integers(-3, 4, size=(n, n))
            d = round(abs(np.linalg.det(D)))
            if 1 < d <= max_det:
                return D, beta
    while True:
        diag = rng.choice([1, 1, 2, 3], size=n)
        if 1 < np.prod(diag) <= max_det:
            break
    sparse = lambda: rng.integers(-1, 2, size=(n, n)) * (rng.random((n, n)) < 2.0 / n)
    Lo = np.tril(sparse(), -1) + np.eye(n, dtype=np.int64)
    Up = np.triu(sparse(), 1) + np.diag(diag)
    D = (Lo @ Up)[rng.permutation(n)][:, rng.permutation(n)]
    return D, beta


@pytest.mark.parametrize("n,seed,max_det", [(1, 0, 40), (2, 1, 300), (3, 2, 300), (4, 3, 300),
                                            (6, 4, 300), (10, 5, 200), (16, 6, 64), (32, 7, 48)])
def test_cell_roots_equal_oracle_set(hom, n, seed, max_det):
    """Every root of one cell; the set equals the oracle's to 1e-12 (Im mod 2 pi)."""
    rng = np.random.default_rng(seed)
    D, beta = _cell(rng, n, max_det)
    ref = oracle.binomial_roots(D, beta)
    say(f"[binomial] n={n} det={len(ref)}")
    z, num = hom.binomial_starts(D, beta)
    z = z.cpu().numpy()
    assert num[0] == len(ref) == len(z)
    w = _match(z, ref, 1e-12)
    assert (z.imag >= -np.pi).all() and (z.imag < np.pi).all()
    say(f"  max |dz| {w:.2e}")


def test_many_cells_one_call_and_ranges(hom):
    """200 cells of n = 5 in one launch, each cell's block against the oracle; sub-ranges equal
    the matching rows of the full call; an empty range writes nothing."""
    rng = np.random.default_rng(11)
    cells = [_cell(rng, 5, 60) for _ in range(200)]
    D = np.stack([c[0] for c in cells])
    beta = np.stack([c[1] for c in cells])
    say("[binomial] 200 cells n=5")
    z, num = hom.binomial_starts(D, beta)
    z = z.cpu().numpy()
    assert len(z) == num.sum()
    off = np.concatenate([[0], np.cumsum(num)])
    for k in range(0, 200, 7):
        _match(z[off[k]:off[k + 1]], oracle.binomial_roots(D[k], beta[k]), 1e-12)
    first = np.minimum(num // 3, num - 1)
    count = np.where(np.arange(200) % 5 == 0, 0, num - first)
    zr, _ = hom.binomial_starts(D, beta, first=first, count=count)
    zr = zr.cpu().numpy()
    ro = np.concatenate([[0], np.cumsum(count)])
    for k in range(200):
        assert np.array_equal(zr[ro[k]:ro[k + 1]], z[off[k] + first[k]:off[k] + first[k] + count[k]])


def test_planted_cell_roots_and_tracking(hom):
    """The n = 8 planted cell (4820 roots): the GPU set equals the oracle's; all 4820 paths tracked
    in FP64 from each side's own start points end on the same endpoint set."""
    import torch
    csys, cell, _ = W.planted_config("c5", P=4)
    D, beta = W.cell_binomial(csys, cell)
    ref = oracle.binomial_roots(D, beta)
    say(f"[binomial] planted n=8 cell, {len(ref)} roots")
    z, num = hom.binomial_starts(D, beta)
    _match(z.cpu().numpy(), ref, 1e-12)
    h = hom.System.from_workload(csys)
    st = hom.track(h, csys.c, z, -32.0, hom.default_params(hom.FP64))
    ze = st.z.cpu().numpy()
    assert (st.status.cpu().numpy() == 0).all()
    zo, _, _, sto, _ = oracle.track(csys, csys.c, ref, -32.0, oracle.TrackParams())
    assert (sto == 0).all()
    _match(ze, zo, 1e-10)


def test_full_size_cell_properties(hom):
    """All 3,881,632 roots of the n = 10 planted cell (the tracking benchmark's start system):
    sampled roots satisfy the system (relative 1e-12 from the definition), and the roots are
    pairwise distinct (their lattice points 2 pi Im(z - z_0) L are distinct integer vectors)."""
    import torch
    csys, cell, _ = W.planted_config("c2", P=4)
    D, beta = W.cell_binomial(csys, cell)
    say("[binomial] n=10 cell, all roots")
    z, num = hom.binomial_starts(D, beta)
    assert len(z) == num[0] == 3881632
    idx = np.random.default_rng(3).choice(len(z), 4096, replace=False)
    zs = z[torch.as_tensor(idx, device=z.device)].cpu().numpy()
    assert _residual(D, beta, zs).max() <= 1e-12
    zn = z.cpu().numpy()
    del z
    torch.cuda.empty_cache()
    assert (zn.imag >= -np.pi).all() and (zn.imag < np.pi).all()
    assert np.abs(zn.real - zn[:1].real).max() <= 1e-12  # Re z is the same for every root
    U, sig, V = W.smith_normal_form(D)
    L = int(sig[-1])
    lat = np.mod(np.rint((zn.imag - zn[:1].imag) / (2 * np.pi) * L).astype(np.int64), L)
    assert len(np.unique(lat, axis=0)) == len(zn)


@pytest.mark.parametrize("factors", [(1, 1, 540000), (1, 600, 1200)])
def test_large_cells_sub_ranges(hom, factors):
    """Cells of 540,000 roots (one invariant factor above one: each thread's later roots come from
    fixed increments) and 720,000 roots (two factors: every digit computed): a sub-range call
    returns bitwise the same roots as the matching slice of the whole cell; sampled roots satisfy
    the system to within the rounding of z times the exponents; all roots are pairwise distinct."""
    import torch
    U = np.array([[1, 2, 0], [0, 1, 0], [3, 0, 1]])  # unimodular
    V = np.array([[1, 0, 0], [1, 1, 0], [2, 5, 1]])
    D = U @ np.diag(factors) @ V
    det = int(np.prod(factors))
    assert round(abs(np.linalg.det(D.astype(float)))) == det
    beta = np.array([0.7 + 0.2j, -1.3 + 0.4j, 0.1 - 2.0j])
    say(f"[binomial] n=3 cell with factors {factors}, {det} roots")
    z, num = hom.binomial_starts(D, beta)
    assert num[0] == det and len(z) == det
    first, count = 12345, 200000
    zs, _ = hom.binomial_starts(D, beta, first=[first], count=[count])
    assert torch.equal(zs, z[first:first + count])
    idx = np.random.default_rng(7).choice(det, 4096, replace=False)
    samp = z[torch.as_tensor(idx, device=z.device)].cpu().numpy()
    # exponents up to 2.7e6: rounding z to doubles alone moves D z by about eps sum_j |D_kj| |z_j|
    scale = (np.abs(samp) @ np.abs(D).T.astype(np.float64)).max(1)
    assert (_residual(D, beta, samp) <= 1e-12 + 16 * 2.0 ** -52 * scale).all()
    zn = z.cpu().numpy()
    L = int(factors[-1])
    lat = np.mod(np.rint((zn.imag - zn[:1].imag) / (2 * np.pi) * L).astype(np.int64), L)
    assert len(np.unique(lat, axis=0)) == det


def test_plan_counts_and_errors(hom):
    """The GPU plan's root counts equal |det D| (numpy) and the oracle's; singular D, zero beta,
    a range outside a cell's roots and too few output rows are refused (HOM_EINVAL); a largest
    invariant factor beyond 2^31 and a Smith form beyond int64 are HOM_EUNSUPPORTED."""
    import ctypes
    import torch
    lib = hom.lib
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
    rng = np.random.default_rng(12)
    for n in (1, 2, 3, 4, 6):
        D, beta = _cell(rng, n, 200)
        D = np.ascontiguousarray(D, np.int32)
        beta = np.ascontiguousarray(beta)
        num = np.zeros(1, np.int64)
        assert lib.hom_binomial_starts(n, 1, P(D), P(beta), None, None, P(num), None, 0,
                                       None) == hom.HOM_OK
        assert num[0] == round(abs(np.linalg.det(D))) == len(oracle.binomial_roots(D, beta))
    D = np.stack([np.diag([2, 3]), np.array([[1, 2], [3, 4]]), np.array([[4, 0], [0, -1]])]).astype(np.int32)
    beta = np.ones((3, 2), np.complex128)
    num = np.zeros(3, np.int64)
    assert lib.hom_binomial_starts(2, 3, P(D), P(beta), None, None, P(num), None, 0, None) == 0
    assert list(num) == [6, 2, 4]
    E = hom.HOM_EINVAL
    sing = np.array([[[1, 2], [2, 4]]], np.int32)
    assert lib.hom_binomial_starts(2, 1, P(sing), P(beta[:1]), None, None, P(num), None, 0, None) == E
    assert b"singular" in lib.hom_last_error()
    zero = np.array([[1.0, 0.0]], np.complex128)
    assert lib.hom_binomial_starts(2, 1, P(D[:1]), P(zero), None, None, P(num), None, 0, None) == E
    assert b"beta" in lib.hom_last_error()
    f, c = np.array([0], np.int64), np.array([7], np.int64)  # 7 > 6 roots
    assert lib.hom_binomial_starts(2, 1, P(D[:1]), P(beta), P(f), P(c), P(num), None, 0, None) == E
    z = torch.zeros((5, 2), dtype=torch.complex128, device="cuda")  # 6 roots, 5 rows
    zp = ctypes.c_void_p(z.data_ptr())
    assert lib.hom_binomial_starts(2, 1, P(D[:1]), P(beta), None, None, P(num), zp, 5, None) == E
    assert b"z_rows" in lib.hom_last_error()
    big = np.array([[[65536, 0], [0, 32769]]], np.int32)  # invariant factors 1, 65536 * 32769
    assert lib.hom_binomial_starts(2, 1, P(big), P(beta), None, None, P(num), None, 0,
                                   None) == hom.HOM_EUNSUPPORTED
    # entries near 2^31: the elimination's products leave int64 before the factors are known
    ovf = np.array([[[-806518787, 643041142, 2119013548], [1405629503, 160003470, -1861309367],
                     [2123086262, -1491957382, -1356837216]]], np.int32)
    b3 = np.ones((1, 3), np.complex128)
    assert lib.hom_binomial_starts(3, 1, P(ovf), P(b3), None, None, P(num), None, 0,
                                   None) == hom.HOM_EUNSUPPORTED
    assert b"int64" in lib.hom_last_error()
