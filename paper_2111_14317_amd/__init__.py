"""Python binding of libhom (include/hom.h): the MI355X polyhedral-homotopy hot path.

Argument marshalling only: every step of the evaluation, solve, tracking and adjoint runs in the
HIP kernels of libhom.so.  Tensors are torch tensors on the current HIP device; complex arrays
are complex128 (interleaved), contiguous.  Calls are enqueued on torch's current stream.
The library must be built (``python -m paper_2111_14317_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

# torch owns the device memory and streams handed to the library, and it bundles its own HIP
# runtime (SONAME libamdhip64.so.7).  Importing it first makes the dynamic loader resolve
# libhom.so's libamdhip64.so.7 to that same runtime instead of loading a second one.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# HOM_LIBRARY selects another build of the library (e.g. one compiled with different options)
LIB_PATH = os.environ.get("HOM_LIBRARY") or os.path.join(_HERE, "libhom.so")

HOM_OK, HOM_EINVAL, HOM_ENOMEM, HOM_EDEVICE, HOM_EUNSUPPORTED = 0, -1, -2, -3, -4
FP64, MIXED = 0, 1
UNSCALED, AFFINE, EVAL_FP32, EVAL_VALU = 1, 2, 4, 8
CREATE_VALU, CREATE_PROJECTIVE, CREATE_PER_EQUATION = 1, 2, 4
PATH_OK, PATH_START, PATH_RUNNING = 0, 1, 2
PATH_SINGULAR, PATH_STEP_MIN, PATH_DIVERGED, PATH_NONFINITE = -1, -2, -3, -4
PATH_POLISH_FAIL, PATH_ENDGAME_FAIL, PATH_MAX_ITERS = -5, -6, -7
TRACK_EXACT_SHIFT, TRACK_SERIAL, TRACK_SIDE_NOWAIT = 1, 2, 4
PREDICT_EULER, PREDICT_HERMITE, PREDICT_RK4 = 0, 1, 2

EXPORTED = ["hom_create", "hom_create_batch", "hom_destroy", "hom_system_info", "hom_eval", "hom_step",
            "hom_step_proj", "hom_track_params_default", "hom_track", "hom_track_noalloc",
            "hom_endpoint_grad", "hom_binomial_starts", "hom_peak_probe", "hom_set_profiling",
            "hom_profile_read", "hom_last_error"]


class HomError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libhom error {code}: {msg}")
        self.code = code


class TrackParams(ctypes.Structure):
    _fields_ = [("ds0", ctypes.c_double), ("ds_max", ctypes.c_double), ("ds_min", ctypes.c_double),
                ("tol_polish", ctypes.c_double), ("tol_track", ctypes.c_double),
                ("tol_end", ctypes.c_double), ("res_tol", ctypes.c_double),
                ("div_re", ctypes.c_double), ("sing_ratio", ctypes.c_double),
                ("tol_predict", ctypes.c_double), ("max_polish", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("max_end", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("predictor", ctypes.c_int32)]


class SysDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_void_p), ("A", ctypes.c_void_p),
                ("w", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -m paper_2111_14317_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.hom_create.argtypes = [i32, P, P, P, i32, ctypes.POINTER(ctypes.c_void_p)]
    lib.hom_create_batch.argtypes = [i32, P, i32, ctypes.POINTER(ctypes.c_void_p)]
    lib.hom_destroy.argtypes = [P]
    lib.hom_system_info.argtypes = [P, P, P, P, P]
    lib.hom_eval.argtypes = [P, P, i64, P, P, P, P, i32, P]
    lib.hom_step.argtypes = [P, P, i64, P, P, P, P, P, i32, P]
    lib.hom_step_proj.argtypes = [P, P, i64, P, P, P, P, P, P]
    lib.hom_track_params_default.argtypes = [ctypes.POINTER(TrackParams), i32]
    lib.hom_track.argtypes = [P, P, i64, P, P, P, P, ctypes.POINTER(TrackParams), P, P, P]
    lib.hom_track_noalloc.argtypes = [P, P, i64, P, P, P, ctypes.POINTER(TrackParams), P, P, P]
    lib.hom_endpoint_grad.argtypes = [P, P, i64, P, P, P, i32, P]
    lib.hom_binomial_starts.argtypes = [i32, i32, P, P, P, P, P, P, i64, P]
    lib.hom_peak_probe.argtypes = [i32, P, P]
    lib.hom_set_profiling.argtypes = [i32]
    lib.hom_profile_read.argtypes = [P, P, P, i32]
    lib.hom_last_error.restype = ctypes.c_char_p
    for name in EXPORTED[:-1]:
        getattr(lib, name).restype = i32
    return lib


lib = _load()


def _check(code):
    if code != HOM_OK:
        raise HomError(code, lib.hom_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_contiguous(), "tensor must be contiguous"
    return ctypes.c_void_p(t.data_ptr())


def default_params(precision=FP64, **overrides) -> TrackParams:
    p = TrackParams()
    _check(lib.hom_track_params_default(ctypes.byref(p), precision))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


class System:
    """A system handle (Alg. 1): exponents A int8 [M][n] equation-major, liftings w [M].
    With the largest m_k >= 32 the handle also carries matrix-core tables (dense supports), and
    eval / step run the MFMA engines unless `valu` is set (or eval gets EVAL_VALU)."""

    num_sys = 1

    def __init__(self, n, m, A, w, valu=False, projective=False, per_equation=False):
        m = np.ascontiguousarray(m, np.int32)
        A = np.ascontiguousarray(A, np.int8)
        w = np.ascontiguousarray(w, np.float64)
        h = ctypes.c_void_p()
        flags = ((CREATE_VALU if valu else 0) | (CREATE_PROJECTIVE if projective else 0) |
                 (CREATE_PER_EQUATION if per_equation else 0))
        _check(lib.hom_create(int(n), m.ctypes.data_as(ctypes.c_void_p),
                              A.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
                              flags, ctypes.byref(h)))
        self.handle = h
        self.n = int(n)
        self.M = int(m.sum())
        self.projective = bool(projective)

    @classmethod
    def from_workload(cls, sys, valu=False, projective=False, per_equation=False):
        return cls(sys.n, sys.m, sys.A, sys.w, valu=valu, projective=projective,
                   per_equation=per_equation)

    def close(self):
        if self.handle:
            lib.hom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch(System):
    """A handle over several systems of uneven n and supports (the batched form): only `track`
    accepts it, with paths grouped by system (see `track`)."""

    def __init__(self, systems):
        keep, descs = [], (SysDesc * len(systems))()
        ns = []
        for q, sy in enumerate(systems):
            m = np.ascontiguousarray(sy.m, np.int32)
            A = np.ascontiguousarray(sy.A, np.int8)
            w = np.ascontiguousarray(sy.w, np.float64)
            keep += [m, A, w]
            descs[q] = SysDesc(int(sy.n), m.ctypes.data, A.ctypes.data, w.ctypes.data)
            ns.append(int(sy.n))
        h = ctypes.c_void_p()
        _check(lib.hom_create_batch(len(systems), descs, 0, ctypes.byref(h)))
        del keep
        self.handle = h
        self.n = max(ns)
        self.ns = ns
        self.mmax = [int(np.max(sy.m)) for sy in systems]
        self.num_sys = len(systems)
        self.M = int(sum(int(np.sum(sy.m)) for sy in systems))


def _dev_like(x, dtype, device):
    import torch
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.asarray(x), dtype=dtype, device=device).contiguous()


def eval(sys: System, c, z, s, flags=0, device="cuda"):
    """G [P][n][n+2] = [J_z | H_s | H] (rows scaled by e^{-logscale}) and logscale [P][n]."""
    import torch
    c = _dev_like(c, torch.complex128, device)
    z = _dev_like(z, torch.complex128, device).reshape(-1, sys.n)
    s = _dev_like(s, torch.float64, device).reshape(-1)
    P = z.shape[0]
    G = torch.empty((P, sys.n, sys.n + 2), dtype=torch.complex128, device=device)
    L = torch.empty((P, sys.n), dtype=torch.float64, device=device)
    _check(lib.hom_eval(sys.handle, _ptr(c), P, _ptr(z), _ptr(s), _ptr(G), _ptr(L), flags,
                        _stream()))
    return G, L


def step(sys: System, c, z, s, precision=FP64, device="cuda"):
    """Euler dz/ds = -J_z^{-1} H_s and Newton -J_z^{-1} H at every point, and status."""
    import torch
    c = _dev_like(c, torch.complex128, device)
    z = _dev_like(z, torch.complex128, device).reshape(-1, sys.n)
    s = _dev_like(s, torch.float64, device).reshape(-1)
    P = z.shape[0]
    dE = torch.empty((P, sys.n), dtype=torch.complex128, device=device)
    dN = torch.empty((P, sys.n), dtype=torch.complex128, device=device)
    st = torch.empty(P, dtype=torch.int32, device=device)
    _check(lib.hom_step(sys.handle, _ptr(c), P, _ptr(z), _ptr(s), _ptr(dE), _ptr(dN), _ptr(st),
                        precision, _stream()))
    return dE, dN, st


def step_proj(sys: System, c, y, s, device="cuda"):
    """Euler and Newton directions in homogeneous coordinates at points y [P][n+1] (a handle
    created with projective=True): [dH~/dy; y^*] dE = [-dH~/ds; 0], [dH~/dy; y^*] dN = [-H~; 0],
    from the null space of the unified system by Householder reflections.  Returns (dE, dN,
    status)."""
    import torch
    c = _dev_like(c, torch.complex128, device)
    y = _dev_like(y, torch.complex128, device).reshape(-1, sys.n + 1)
    P = y.shape[0]
    s = _dev_like(s, torch.float64, device).reshape(-1).expand(P).contiguous()
    dE = torch.empty((P, sys.n + 1), dtype=torch.complex128, device=device)
    dN = torch.empty((P, sys.n + 1), dtype=torch.complex128, device=device)
    st = torch.empty(P, dtype=torch.int32, device=device)
    _check(lib.hom_step_proj(sys.handle, _ptr(c), P, _ptr(y), _ptr(s), _ptr(dE), _ptr(dN),
                             _ptr(st), _stream()))
    return dE, dN, st


def binomial_starts(D, beta, first=None, count=None, device="cuda"):
    """Roots of binomial start systems x^{d_k} = beta_k (Sec. 2), one system per cell:
    D int [cells][n][n] (or [n][n]), beta complex [cells][n] (or [n]).  With first/count
    ([cells] each) only roots first .. first + count - 1 of each cell.  Returns (z, num_roots):
    z complex128 [rows][n] on the device (log coordinates, the cells' roots one after the
    other), num_roots int64 [cells] = |det D| per cell."""
    import torch
    D = np.ascontiguousarray(D, np.int32)
    if D.ndim == 2:
        D = D[None]
    cells, n = D.shape[0], D.shape[1]
    if D.shape != (cells, n, n):
        raise ValueError("D must be [cells][n][n]")
    beta = np.ascontiguousarray(np.asarray(beta, np.complex128).reshape(cells, n))
    if (first is None) != (count is None):
        raise ValueError("first and count go together")
    f = c = None
    if first is not None:
        f = np.ascontiguousarray(np.broadcast_to(np.asarray(first, np.int64), (cells,)))
        c = np.ascontiguousarray(np.broadcast_to(np.asarray(count, np.int64), (cells,)))
    num = np.zeros(cells, np.int64)
    args = (n, cells, D.ctypes.data_as(ctypes.c_void_p), beta.ctypes.data_as(ctypes.c_void_p),
            f.ctypes.data_as(ctypes.c_void_p) if f is not None else None,
            c.ctypes.data_as(ctypes.c_void_p) if c is not None else None,
            num.ctypes.data_as(ctypes.c_void_p))
    _check(lib.hom_binomial_starts(*args, None, 0, _stream()))  # sizing: num_roots only
    rows = int(c.sum()) if c is not None else int(num.sum())
    z = torch.empty((rows, n), dtype=torch.complex128, device=device)
    if rows:
        _check(lib.hom_binomial_starts(*args, _ptr(z), rows, _stream()))
    return z, num


PEAK_KINDS = {"hbm_read_gb_s": 0, "hbm_write_gb_s": 1, "fp64_fma_tflops": 2, "fp32_fma_tflops": 3,
              "fp32_exp2_g_per_s": 4, "mfma_f64_tflops": 5, "mfma_bf16_tflops": 6,
              "exp_f64_g_per_s": 7, "sincos_f64_g_per_s": 8}


def peak_probes():
    """Measured rates of the device's units (hom_peak_probe), keyed as PEAK_KINDS."""
    out = {}
    for name, kind in PEAK_KINDS.items():
        v = ctypes.c_double()
        _check(lib.hom_peak_probe(kind, ctypes.byref(v), _stream()))
        out[name] = v.value
    return out


@dataclasses.dataclass
class TrackState:
    z: "torch.Tensor"
    s: "torch.Tensor"
    ds: "torch.Tensor"
    status: "torch.Tensor"
    counters: "torch.Tensor"


def track(sys: System, c, z0, s0, params: TrackParams | None = None, state: TrackState | None = None,
          device="cuda", sys_idx=None) -> TrackState:
    """Track paths to s = 0.  Pass `state` (from a previous call) to resume RUNNING paths.
    Batch handle: c is the concatenation of the systems' coefficients, z0 is [P][n_max] (each
    path uses the first n of its system), sys_idx [P] int32 non-decreasing."""
    import torch
    params = params or default_params()
    c = _dev_like(c, torch.complex128, device)
    if sys.num_sys > 1 or isinstance(sys, Batch):
        if sys_idx is None:
            raise ValueError("a batch handle needs sys_idx")
        sys_idx = _dev_like(sys_idx, torch.int32, device)
    elif sys_idx is not None:
        raise ValueError("sys_idx is only for batch handles")
    if state is None:
        z = _dev_like(z0, torch.complex128, device).reshape(-1, sys.n).clone()
        P = z.shape[0]
        s = torch.empty(P, dtype=torch.float64, device=device)
        s.copy_(_dev_like(s0, torch.float64, device).reshape(-1).expand(P))
        state = TrackState(z, s, torch.zeros(P, dtype=torch.float64, device=device),
                           torch.full((P,), PATH_START, dtype=torch.int32, device=device),
                           torch.zeros((P, 4), dtype=torch.int32, device=device))
    P = state.z.shape[0]
    _check(lib.hom_track(sys.handle, _ptr(c), P, _ptr(state.z), _ptr(state.s), _ptr(state.ds),
                         _ptr(sys_idx), ctypes.byref(params), _ptr(state.status),
                         _ptr(state.counters), _stream()))
    return state


def track_noalloc(sys: System, c, state: TrackState, params: TrackParams | None = None):
    """hom_track_noalloc on an existing state (z, s, ds, status, counters, updated in place): the
    tracker with the library's static device scratch instead of any allocation (single-system
    handles; the mixed form's launches in serial order)."""
    params = params or default_params()
    P = state.z.shape[0]
    _check(lib.hom_track_noalloc(sys.handle, _ptr(c), P, _ptr(state.z), _ptr(state.s),
                                 _ptr(state.ds), ctypes.byref(params), _ptr(state.status),
                                 _ptr(state.counters), _stream()))
    return state


def new_state(z0, s0, device="cuda") -> TrackState:
    """A fresh tracking state: start points z0 [P][n] at s0, every path HOM_PATH_START."""
    import torch
    z = torch.as_tensor(np.asarray(z0), dtype=torch.complex128, device=device).contiguous().clone()
    P = z.shape[0]
    s = torch.empty(P, dtype=torch.float64, device=device)
    s.copy_(_dev_like(s0, torch.float64, device).reshape(-1).expand(P))
    return TrackState(z, s, torch.zeros(P, dtype=torch.float64, device=device),
                      torch.full((P,), PATH_START, dtype=torch.int32, device=device),
                      torch.zeros((P, 4), dtype=torch.int32, device=device))


def endpoint_grad(sys: System, c, z_end, grad_x, precision=FP64, device="cuda"):
    """grad_c [M] of a loss on endpoints x = e^{z_end}, given grad_x = dL/dRe x + i dL/dIm x."""
    import torch
    c = _dev_like(c, torch.complex128, device)
    z = _dev_like(z_end, torch.complex128, device).reshape(-1, sys.n)
    g = _dev_like(grad_x, torch.complex128, device).reshape(-1, sys.n)
    out = torch.empty(sys.M, dtype=torch.complex128, device=device)
    _check(lib.hom_endpoint_grad(sys.handle, _ptr(c), z.shape[0], _ptr(z), _ptr(g), _ptr(out),
                                 precision, _stream()))
    return out


def set_profiling(on: bool):
    """Record hipEvents around every kernel launch of this thread's compute calls."""
    _check(lib.hom_set_profiling(1 if on else 0))


def profile_read(cap=4096):
    """[(kernel label, milliseconds, eval+solves or -1)] of the launches recorded since the last
    read (waits for them)."""
    names = ctypes.create_string_buffer(64 * cap)
    ms = (ctypes.c_double * cap)()
    units = (ctypes.c_int64 * cap)()
    n = lib.hom_profile_read(names, ms, units, cap)
    if n < 0:
        _check(n)
    raw = names.raw
    return [(raw[64 * i:64 * i + 64].split(b"\0", 1)[0].decode(), ms[i], units[i]) for i in range(n)]


def _make_autograd():
    import torch

    class HomTrack(torch.autograd.Function):
        """x* = track(c; sys, z0, s0) with gradient w.r.t. c through the adjoint kernel.

        forward(c, sys, z0, s0, params, precision) -> (x_end [P][n] complex128, status [P]);
        backward uses only the paths that ended OK."""

        @staticmethod
        def forward(ctx, c, sys, z0, s0, params=None, precision=FP64):
            st = track(sys, c.detach(), z0, s0, params or default_params(precision))
            ok = st.status == PATH_OK
            ctx.sys, ctx.precision = sys, precision
            ctx.save_for_backward(c.detach(), st.z, ok)
            x = torch.exp(st.z)
            ctx.mark_non_differentiable(st.status)
            return x, st.status

        @staticmethod
        def backward(ctx, grad_x, grad_status):
            c, z_end, ok = ctx.saved_tensors
            g = torch.where(ok[:, None], grad_x, torch.zeros_like(grad_x)).contiguous()
            gc = endpoint_grad(ctx.sys, c, z_end, g, ctx.precision)
            return gc, None, None, None, None, None

    return HomTrack


try:
    HomTrack = _make_autograd()
except ImportError:  # torch missing: the ctypes layer still loads
    HomTrack = None
