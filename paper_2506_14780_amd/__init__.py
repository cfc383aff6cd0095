"""Python binding of libsknr (C ABI in include/sknr.h).

Argument marshalling only: every computation runs in the HIP library.
Device arrays are torch tensors on the HIP device (torch supplies device
memory and streams); their data pointers cross the ABI.  The library is
built in-tree by ``paper_2506_14780_amd.build``; importing this module
fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

__all__ = [
    "lib", "Context", "Problem", "solve", "solve_noalloc", "c_transform_row", "c_transform_col",
    "projected_system", "newton_step", "newton_coef", "NEWTON_DIRECT", "NEWTON_CG", "NEWTON_SCHULZ",
    "spectral_basis", "evaluate", "coupling", "gradient",
    "entropic_ot_loss",
    "SknrError", "COST_STORED", "COST_SQEUCLID", "XTERM_AUTO", "XTERM_FP32",
    "XTERM_BF16", "XTERM_BF16X3", "XTERM_BF16X6", "WARM_SEQUENTIAL", "WARM_STATIC", "WARM_USER",
    "LIB_PATH", "MAX_STAGES", "MAX_ELL", "serve_config", "submit", "poll", "wait", "cancel",
    "serve_stats", "OK", "NOT_CONVERGED", "EINVAL", "ENOMEM", "EDEVICE", "EBUSY", "ECANCELED", "EINTERNAL",
]

# torch ships its own HIP runtime; importing it first makes libsknr bind to
# that same runtime (one HIP runtime per process).
import torch  # noqa: E402,F401

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsknr.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"libsknr.so not built ({LIB_PATH}); run `python -m paper_2506_14780_amd.build`")
lib = ctypes.CDLL(LIB_PATH)

MAX_STAGES = 32
MAX_ELL = 32
COST_STORED, COST_SQEUCLID = 0, 1
XTERM_AUTO, XTERM_FP32, XTERM_BF16, XTERM_BF16X3, XTERM_BF16X6 = 0, 1, 2, 3, 4
WARM_SEQUENTIAL, WARM_STATIC, WARM_USER = 0, 1, 2
OK, NOT_CONVERGED = 0, 1
EINVAL, ENOMEM, EDEVICE, EBUSY, ECANCELED, EINTERNAL = -1, -2, -3, -4, -5, -6

_p = ctypes.c_void_p
_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


class _Problem(ctypes.Structure):
    _fields_ = [("n", _i64), ("m", _i64), ("d", _i32), ("kind", _i32), ("xterm", _i32),
                ("on_host", _i32), ("C", _p), ("ldc", _i64), ("x", _p), ("y", _p),
                ("cost_scale", _d), ("a", _p), ("b", _p)]


class _Opts(ctypes.Structure):
    _fields_ = [("eps", ctypes.POINTER(_d)), ("n_eps", _i32), ("max_iter", _i32), ("tol", _d),
                ("ell", _i32), ("warm_mode", _i32), ("eps_prime", _d), ("eig_oversample", _i32),
                ("eig_max_iter", _i32), ("eig_tol", _d), ("check_every", _i32),
                ("first_stage_nr", _i32), ("f0", _p), ("V0", _p), ("seed", ctypes.c_uint64),
                ("stream", _p), ("nr_switch_iters", _i32), ("newton_solver", _i32),
                ("newton_max_iter", _i32), ("newton_rtol", _d), ("nr_min_gain", _d), ("g0", _p)]


class _Stage(ctypes.Structure):
    _fields_ = [("eps", _d), ("iters", _i32), ("newton_tried", _i32), ("newton_accepted", _i32),
                ("eig_iters", _i32), ("marginal_err", _d), ("seconds", _d), ("rate_gain", _d),
                ("nr_skipped", _i32), ("reserved0", _i32)]


class _Result(ctypes.Structure):
    _fields_ = [("status", _i32), ("n_stages", _i32), ("total_iters", _i32), ("transposed", _i32),
                ("stage", _Stage * MAX_STAGES), ("marginal_err", _d), ("row_err", _d),
                ("col_err", _d), ("transport_cost", _d), ("dual_value", _d),
                ("primal_value", _d), ("mass", _d), ("marginal_err_exact", _d),
                ("transport_cost_exact", _d), ("seconds", _d), ("queue_seconds", _d),
                ("latency_seconds", _d)]


class _Eval(ctypes.Structure):
    _fields_ = [("row_err", _d), ("col_err", _d), ("marginal_err", _d), ("transport_cost", _d),
                ("dual_value", _d), ("primal_value", _d), ("mass", _d), ("row_err_exact", _d),
                ("col_err_exact", _d), ("marginal_err_exact", _d), ("transport_cost_exact", _d)]


class _ServeInfo(ctypes.Structure):
    _fields_ = [("lanes", _i32), ("queued", _i32), ("running", _i32), ("reserved0", _i32),
                ("completed", _i64), ("pool_bytes", ctypes.c_uint64), ("pool_used", ctypes.c_uint64),
                ("pool_peak", ctypes.c_uint64), ("batches", _i64), ("batched_jobs", _i64),
                ("batched_launches", _i64)]


class _KProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", _i64), ("total_ms", _d), ("units", _d)]


def _sig(name, args):
    fn = getattr(lib, name)
    fn.argtypes = args
    fn.restype = ctypes.c_int
    return fn


_P = ctypes.POINTER
lib.sknr_status_str.restype = ctypes.c_char_p
lib.sknr_status_str.argtypes = [ctypes.c_int]
lib.sknr_last_error.restype = ctypes.c_char_p
lib.sknr_version.restype = ctypes.c_char_p
_sig("sknr_ctx_create", [ctypes.c_int, ctypes.c_uint64, _P(_p)])
_sig("sknr_ctx_destroy", [_p])
_sig("sknr_solve", [_p, _P(_Problem), _P(_Opts), _p, _p, _P(_Result)])
_sig("sknr_solve_noalloc", [_p, _P(_Problem), _P(_Opts), _p, _p, _P(_Result)])
_sig("sknr_c_transform_row", [_p, _P(_Problem), _d, _p, _p, _p])
_sig("sknr_c_transform_col", [_p, _P(_Problem), _d, _p, _p, _p, _P(_d), _P(_d), _p])
_sig("sknr_projected_system", [_p, _P(_Problem), _d, _p, _p, _i32, _P(_d), _P(_d), _P(_d), _p])
_sig("sknr_newton_step", [_p, _P(_Problem), _d, _p, _p, _i32, _P(_i32), _P(_d), _P(_d), _p])
_sig("sknr_newton_coef", [_p, _P(_Problem), _d, _p, _p, _i32, _i32, _i32, _d, _P(_d), _P(_i32), _P(_i32), _p])
_sig("sknr_spectral_basis", [_p, _P(_Problem), _d, _p, _i32, _i32, _i32, _d, ctypes.c_uint64, _p,
                             _P(_d), _P(_i32), _p])
_sig("sknr_get_subspace", [_p, _p, _i64, _i32, _P(_i32), _p])
_sig("sknr_evaluate", [_p, _P(_Problem), _d, _p, _p, _P(_Eval), _p])
_sig("sknr_coupling", [_p, _P(_Problem), _d, _p, _p, _p, _p])
_sig("sknr_gradient", [_p, _P(_Problem), _d, _p, _p, _p, _p, _p, _p, _p])
_sig("sknr_profile", [_p, _i32])
_sig("sknr_serve_config", [_p, _i32, ctypes.c_uint64])
_sig("sknr_serve_batching", [_p, _i32])
_sig("sknr_submit", [_p, _P(_Problem), _P(_Opts), _P(ctypes.c_uint64)])
_sig("sknr_poll", [_p, ctypes.c_uint64, _P(_i32)])
_sig("sknr_wait", [_p, ctypes.c_uint64, _p, _p, _P(_Result)])
_sig("sknr_cancel", [_p, ctypes.c_uint64])
_sig("sknr_serve_stats", [_p, _P(_ServeInfo)])
_sig("sknr_profile_read", [_p, _P(_KProf), _i32, _P(_i32)])


class SknrError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.sknr_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {status} ({lib.sknr_status_str(status).decode()}): {msg}")
        self.status = status


def _check(st: int, where: str, allow_not_converged: bool = True) -> int:
    if st < 0 or (st == NOT_CONVERGED and not allow_not_converged):
        raise SknrError(st, where)
    return st


def _ptr(t):
    """Address of a torch tensor's data, or of a numpy array's (host)."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(t.ctypes.data)


def _on_host(t) -> bool:
    """numpy arrays and CPU tensors are host memory."""
    if t is None:
        return False
    if hasattr(t, "is_cuda"):  # torch tensor
        return not t.is_cuda
    return True


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """A libsknr context on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        try:  # torch owns the device memory and streams: let it set up HIP first
            import torch
            torch.cuda.init()
        except ImportError:  # pragma: no cover
            pass
        h = ctypes.c_void_p()
        _check(lib.sknr_ctx_create(device, hbm_budget_bytes, ctypes.byref(h)), "sknr_ctx_create")
        self.handle = h
        self.device = device

    def profile(self, enable: bool = True):
        """Per-kernel timing with HIP events (resets the table)."""
        _check(lib.sknr_profile(self.handle, 1 if enable else 0), "sknr_profile")

    def profile_read(self) -> list:
        cnt = _i32()
        _check(lib.sknr_profile_read(self.handle, None, 0, ctypes.byref(cnt)), "sknr_profile_read")
        arr = (_KProf * max(1, cnt.value))()
        _check(lib.sknr_profile_read(self.handle, arr, cnt.value, ctypes.byref(cnt)), "sknr_profile_read")
        return [dict(name=arr[i].name.decode(), launches=arr[i].launches, total_ms=arr[i].total_ms,
                     units=arr[i].units) for i in range(cnt.value)]

    def close(self):
        if self.handle:
            _check(lib.sknr_ctx_destroy(self.handle), "sknr_ctx_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class Problem:
    """Problem arrays: a, b float64; either C (n x m float32, row stride
    ldc) or x (n x d), y (m x d) float32.  Device tensors, or host arrays
    (numpy, CPU tensors; contiguous rows) that each call copies to the
    device."""

    a: object
    b: object
    C: object = None
    x: object = None
    y: object = None
    cost_scale: float = 1.0
    xterm: int = XTERM_AUTO
    ldc: int | None = None

    def on_host(self) -> bool:
        """True for host arrays (numpy or CPU tensors): sknr_problem.on_host,
        the call copies them to the device first.  All arrays of a problem
        live on the same side."""
        arrs = [t for t in (self.a, self.b, self.C, self.x, self.y) if t is not None]
        side = {_on_host(t) for t in arrs}
        if len(side) != 1:
            raise ValueError("problem arrays must all be on the host or all on the device")
        return side.pop()

    def c_struct(self) -> _Problem:
        p = _Problem()
        p.on_host = 1 if self.on_host() else 0
        p.n = int(self.a.shape[0])
        p.m = int(self.b.shape[0])
        p.a = _ptr(self.a)
        p.b = _ptr(self.b)
        p.xterm = self.xterm
        if self.C is not None:
            p.kind = COST_STORED
            p.C = _ptr(self.C)
            if self.ldc is not None:
                p.ldc = self.ldc
            elif hasattr(self.C, "stride") and callable(self.C.stride):
                p.ldc = int(self.C.stride(0))
            else:  # numpy: strides in bytes
                p.ldc = int(self.C.strides[0] // self.C.itemsize)
            p.d = 0
        else:
            p.kind = COST_SQEUCLID
            p.x = _ptr(self.x)
            p.y = _ptr(self.y)
            p.d = int(self.x.shape[1])
            p.cost_scale = self.cost_scale
        return p


def _opts(eps, tol, max_iter, ell, warm_mode, V0, f0, eps_prime, check_every, first_stage_nr, eig_oversample,
          eig_max_iter, eig_tol, seed, stream, nr_switch_iters=0, newton_solver=0, newton_max_iter=0,
          newton_rtol=0.0, nr_min_gain=0.0, g0=None):
    earr = (_d * len(eps))(*eps)
    o = _Opts()
    o.eps = ctypes.cast(earr, _P(_d))
    o.n_eps = len(eps)
    o.max_iter = max_iter
    o.tol = tol
    o.ell = ell
    o.warm_mode = warm_mode
    o.eps_prime = eps_prime
    o.eig_oversample = eig_oversample
    o.eig_max_iter = eig_max_iter
    o.eig_tol = eig_tol
    o.check_every = check_every
    o.first_stage_nr = 1 if first_stage_nr else 0
    o.f0 = _ptr(f0)
    o.V0 = _ptr(V0)
    o.seed = seed
    o.stream = _stream(stream)
    o.nr_switch_iters = int(nr_switch_iters)
    o.newton_solver = int(newton_solver)
    o.newton_max_iter = int(newton_max_iter)
    o.newton_rtol = float(newton_rtol)
    o.nr_min_gain = float(nr_min_gain)
    o.g0 = _ptr(g0)
    return o, earr  # earr must outlive the call


def _result_dict(r):
    res = {k: getattr(r, k) for k, _ in _Result._fields_ if k != "stage"}
    res["stages"] = [{k: getattr(r.stage[i], k) for k, _ in _Stage._fields_} for i in range(r.n_stages)]
    return res


def solve(ctx: Context, prob: Problem, eps, tol: float = 1e-6, max_iter: int = 10000, ell: int = 0,
          warm_mode: int = WARM_USER, V0=None, f0=None, eps_prime: float = 0.0, check_every: int = 0,
          first_stage_nr: bool = False, eig_oversample: int = 0, eig_max_iter: int = 0,
          eig_tol: float = 0.0, seed: int = 0, stream=None, f_out=None, g_out=None, nr_switch_iters: int = 0,
          newton_solver: int = 0, newton_max_iter: int = 0, newton_rtol: float = 0.0, nr_min_gain: float = 0.0,
          g0=None):
    """sknr_solve.  Returns (f, g, result dict); f, g are float64 device
    tensors in the caller's orientation.  The problem may hold host arrays
    (numpy or CPU tensors: copied to the device by the call); f0, g0, V0
    and the outputs are device tensors."""
    import torch
    eps = [float(e) for e in (eps if hasattr(eps, "__len__") else [eps])]
    dev = torch.device("cuda", ctx.device) if prob.on_host() else prob.a.device
    n, m = int(prob.a.shape[0]), int(prob.b.shape[0])
    f = f_out if f_out is not None else torch.empty(n, dtype=torch.float64, device=dev)
    g = g_out if g_out is not None else torch.empty(m, dtype=torch.float64, device=dev)
    o, earr = _opts(eps, tol, max_iter, ell, warm_mode, V0, f0, eps_prime, check_every, first_stage_nr,
                    eig_oversample, eig_max_iter, eig_tol, seed, stream, nr_switch_iters, newton_solver,
                    newton_max_iter, newton_rtol, nr_min_gain, g0)
    r = _Result()
    ps = prob.c_struct()
    st = lib.sknr_solve(ctx.handle, ctypes.byref(ps), ctypes.byref(o), _ptr(f), _ptr(g), ctypes.byref(r))
    _check(st, "sknr_solve")
    return f, g, _result_dict(r)


def solve_noalloc(ctx: Context, prob: Problem, eps, f_out, g_out, tol: float = 1e-6, max_iter: int = 10000,
                  ell: int = 0, warm_mode: int = WARM_USER, V0=None, f0=None, eps_prime: float = 0.0,
                  check_every: int = 0, first_stage_nr: bool = False, eig_oversample: int = 0,
                  eig_max_iter: int = 0, eig_tol: float = 0.0, seed: int = 0, stream=None,
                  nr_switch_iters: int = 0, newton_solver: int = 0, newton_max_iter: int = 0,
                  newton_rtol: float = 0.0, nr_min_gain: float = 0.0) -> dict:
    """sknr_solve_noalloc: sknr_solve with the workspace in the library's
    static device array (no device allocation).  f_out (n) and g_out (m)
    are caller-provided float64 device tensors; returns the result dict."""
    eps = [float(e) for e in (eps if hasattr(eps, "__len__") else [eps])]
    o, earr = _opts(eps, tol, max_iter, ell, warm_mode, V0, f0, eps_prime, check_every, first_stage_nr,
                    eig_oversample, eig_max_iter, eig_tol, seed, stream, nr_switch_iters, newton_solver,
                    newton_max_iter, newton_rtol, nr_min_gain)
    r = _Result()
    ps = prob.c_struct()
    st = lib.sknr_solve_noalloc(ctx.handle, ctypes.byref(ps), ctypes.byref(o), _ptr(f_out), _ptr(g_out),
                                ctypes.byref(r))
    _check(st, "sknr_solve_noalloc")
    return _result_dict(r)


# ------------------------------------------------------------------ serving
def serve_config(ctx: Context, max_active: int = 0, pool_bytes: int = 0, batched: bool = False):
    """sknr_serve_config and sknr_serve_batching: lanes, pool size and
    batched execution, before the first submit."""
    _check(lib.sknr_serve_config(ctx.handle, max_active, pool_bytes), "sknr_serve_config")
    _check(lib.sknr_serve_batching(ctx.handle, 1 if batched else 0), "sknr_serve_batching")


def submit(ctx: Context, prob: Problem, eps, tol: float = 1e-6, max_iter: int = 10000, ell: int = 0,
           warm_mode: int = WARM_SEQUENTIAL, eps_prime: float = 0.0, check_every: int = 0,
           first_stage_nr: bool = False, eig_oversample: int = 0, eig_max_iter: int = 0,
           eig_tol: float = 0.0, seed: int = 0, stream=None, nr_switch_iters: int = 0, newton_solver: int = 0,
           newton_max_iter: int = 0, newton_rtol: float = 0.0, nr_min_gain: float = 0.0) -> int:
    """sknr_submit: queue a solve (inputs are copied before returning);
    returns the ticket."""
    eps = [float(e) for e in (eps if hasattr(eps, "__len__") else [eps])]
    o, earr = _opts(eps, tol, max_iter, ell, warm_mode, None, None, eps_prime, check_every, first_stage_nr,
                    eig_oversample, eig_max_iter, eig_tol, seed, stream, nr_switch_iters, newton_solver,
                    newton_max_iter, newton_rtol, nr_min_gain)
    ps = prob.c_struct()
    t = ctypes.c_uint64()
    _check(lib.sknr_submit(ctx.handle, ctypes.byref(ps), ctypes.byref(o), ctypes.byref(t)), "sknr_submit")
    return t.value


def poll(ctx: Context, ticket: int) -> bool:
    d = _i32()
    _check(lib.sknr_poll(ctx.handle, ticket, ctypes.byref(d)), "sknr_poll")
    return bool(d.value)


def wait(ctx: Context, ticket: int, n: int, m: int, device=None, raise_on_error: bool = True):
    """sknr_wait: (f, g, result dict); result["status"] carries
    NOT_CONVERGED / ECANCELED when raise_on_error is False."""
    import torch
    dev = device if device is not None else torch.device("cuda", ctx.device)
    f = torch.empty(n, dtype=torch.float64, device=dev)
    g = torch.empty(m, dtype=torch.float64, device=dev)
    r = _Result()
    st = lib.sknr_wait(ctx.handle, ticket, _ptr(f), _ptr(g), ctypes.byref(r))
    if raise_on_error:
        _check(st, "sknr_wait")
    res = _result_dict(r)
    res["status"] = st
    return f, g, res


def cancel(ctx: Context, ticket: int):
    _check(lib.sknr_cancel(ctx.handle, ticket), "sknr_cancel")


def serve_stats(ctx: Context) -> dict:
    i = _ServeInfo()
    _check(lib.sknr_serve_stats(ctx.handle, ctypes.byref(i)), "sknr_serve_stats")
    return {k: getattr(i, k) for k, _ in _ServeInfo._fields_ if k != "reserved0"}


def c_transform_row(ctx, prob: Problem, eps: float, g, stream=None):
    import torch
    f = torch.empty(int(prob.a.shape[0]), dtype=torch.float64, device=g.device)
    ps = prob.c_struct()
    _check(lib.sknr_c_transform_row(ctx.handle, ctypes.byref(ps), eps, _ptr(g), _ptr(f), _stream(stream)),
           "sknr_c_transform_row")
    return f


def c_transform_col(ctx, prob: Problem, eps: float, f, g_prev=None, stream=None):
    """Returns (g, err, <g,b>)."""
    import torch
    g = torch.empty(int(prob.b.shape[0]), dtype=torch.float64, device=f.device)
    err, gdot = _d(), _d()
    ps = prob.c_struct()
    _check(lib.sknr_c_transform_col(ctx.handle, ctypes.byref(ps), eps, _ptr(f), _ptr(g_prev), _ptr(g),
                                    ctypes.byref(err), ctypes.byref(gdot), _stream(stream)),
           "sknr_c_transform_col")
    return g, err.value, gdot.value


def projected_system(ctx, prob: Problem, eps: float, f, V, stream=None):
    """Returns (G, grad, qsemi) as numpy arrays / float."""
    import numpy as np
    ell = int(V.shape[1])
    G = (_d * (ell * ell))()
    gr = (_d * ell)()
    q = _d()
    ps = prob.c_struct()
    _check(lib.sknr_projected_system(ctx.handle, ctypes.byref(ps), eps, _ptr(f), _ptr(V), ell, G, gr,
                                     ctypes.byref(q), _stream(stream)), "sknr_projected_system")
    return np.array(G[:]).reshape(ell, ell), np.array(gr[:]), q.value


def newton_step(ctx, prob: Problem, eps: float, f, V, stream=None):
    """In-place on f; returns (accepted, q0, q1)."""
    acc = _i32()
    q0, q1 = _d(), _d()
    ps = prob.c_struct()
    _check(lib.sknr_newton_step(ctx.handle, ctypes.byref(ps), eps, _ptr(f), _ptr(V), int(V.shape[1]),
                                ctypes.byref(acc), ctypes.byref(q0), ctypes.byref(q1), _stream(stream)),
           "sknr_newton_step")
    return bool(acc.value), q0.value, q1.value


NEWTON_DIRECT, NEWTON_CG, NEWTON_SCHULZ = 0, 1, 2


def newton_coef(ctx, prob: Problem, eps: float, f, V, solver: int = NEWTON_DIRECT, max_iter: int = 0,
                rtol: float = 0.0, stream=None):
    """sknr_newton_coef: the coefficients c = eps G^-1 grad of the
    projected Newton step by the chosen solver.  Returns (c [ell] numpy,
    ok, iterations)."""
    import numpy as np
    ell = int(V.shape[1])
    c = (_d * ell)()
    ok, it = _i32(), _i32()
    ps = prob.c_struct()
    _check(lib.sknr_newton_coef(ctx.handle, ctypes.byref(ps), eps, _ptr(f), _ptr(V), ell, solver, max_iter, rtol,
                                c, ctypes.byref(ok), ctypes.byref(it), _stream(stream)), "sknr_newton_coef")
    return np.array(c[:]), bool(ok.value), it.value


def spectral_basis(ctx, prob: Problem, eps: float, f, ell: int, oversample: int = 8, max_iter: int = 200,
                   tol: float = 1e-7, seed: int = 0, stream=None):
    """Returns (V [n x ell float64 device], rho [ell+1], iters)."""
    import numpy as np
    import torch
    n = int(prob.a.shape[0])
    V = torch.empty((n, ell), dtype=torch.float64, device=f.device)
    rho = (_d * (ell + 1))()
    it = _i32()
    ps = prob.c_struct()
    _check(lib.sknr_spectral_basis(ctx.handle, ctypes.byref(ps), eps, _ptr(f), ell, oversample, max_iter, tol,
                                   seed, _ptr(V), rho, ctypes.byref(it), _stream(stream)), "sknr_spectral_basis")
    return V, np.array(rho[:]), it.value


def get_subspace(ctx, rows: int, ell: int, stream=None):
    """sknr_get_subspace: the basis V_l of the last solve on ctx (rows =
    min(n, m) of that solve).  Returns (V [rows x ell float64 device],
    side: 0 = x side, 1 = y side)."""
    import torch
    V = torch.empty((rows, ell), dtype=torch.float64, device=torch.device("cuda", ctx.device))
    side = _i32()
    _check(lib.sknr_get_subspace(ctx.handle, _ptr(V), rows, ell, ctypes.byref(side), _stream(stream)),
           "sknr_get_subspace")
    return V, side.value


def evaluate(ctx, prob: Problem, eps: float, f, g, stream=None) -> dict:
    e = _Eval()
    ps = prob.c_struct()
    _check(lib.sknr_evaluate(ctx.handle, ctypes.byref(ps), eps, _ptr(f), _ptr(g), ctypes.byref(e),
                             _stream(stream)), "sknr_evaluate")
    return {k: getattr(e, k) for k, _ in _Eval._fields_}


def gradient(ctx, prob: Problem, eps: float, f, g, x: bool = True, y: bool = True, a: bool = True,
             b: bool = True, stream=None) -> dict:
    """sknr_gradient: the gradients of W_eps with respect to the requested
    data at the potentials (f, g); float64 device tensors keyed "x", "y"
    (n x d, m x d; squared-Euclidean problems), "a", "b"."""
    import torch
    n, m = int(prob.a.shape[0]), int(prob.b.shape[0])
    d = int(prob.x.shape[1]) if prob.x is not None else 0
    dev = f.device
    out = {}
    if x:
        out["x"] = torch.empty((n, d), dtype=torch.float64, device=dev)
    if y:
        out["y"] = torch.empty((m, d), dtype=torch.float64, device=dev)
    if a:
        out["a"] = torch.empty(n, dtype=torch.float64, device=dev)
    if b:
        out["b"] = torch.empty(m, dtype=torch.float64, device=dev)
    ps = prob.c_struct()
    _check(lib.sknr_gradient(ctx.handle, ctypes.byref(ps), eps, _ptr(f), _ptr(g), _ptr(out.get("x")),
                             _ptr(out.get("y")), _ptr(out.get("a")), _ptr(out.get("b")), _stream(stream)),
           "sknr_gradient")
    return out


class _EntropicOTLoss(torch.autograd.Function):
    """W_eps(a, b, x, y) by a solve; its gradients by sknr_gradient at the
    solution (envelope theorem: the solver loop is not differentiated)."""

    @staticmethod
    def forward(actx, ctx, x, y, a, b, eps_ladder, tol, max_iter, ell, warm_mode, cost_scale):
        prob = Problem(a=a.detach().contiguous(), b=b.detach().contiguous(), x=x.detach().contiguous(),
                       y=y.detach().contiguous(), cost_scale=cost_scale)
        f, g, res = solve(ctx, prob, eps_ladder, tol=tol, max_iter=max_iter, ell=ell, warm_mode=warm_mode)
        actx.save_for_backward(f, g)
        actx.sk = (ctx, prob, float(eps_ladder[-1]))
        return torch.tensor(res["dual_value"], dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(actx, gout):
        f, g = actx.saved_tensors
        ctx, prob, eps = actx.sk
        need = actx.needs_input_grad
        gr = gradient(ctx, prob, eps, f, g, x=need[1], y=need[2], a=need[3], b=need[4])
        conv = lambda k, t: (gout * gr[k]).to(t.dtype) if k in gr else None
        return (None, conv("x", prob.x), conv("y", prob.y), conv("a", prob.a), conv("b", prob.b),
                None, None, None, None, None, None)


def entropic_ot_loss(ctx, x, y, a, b, eps, tol: float = 1e-6, max_iter: int = 100000, ell: int = 0,
                     warm_mode: int = WARM_SEQUENTIAL, cost_scale: float = 1.0):
    """W_eps between the weighted point clouds (a, x) and (b, y) (squared
    Euclidean cost times cost_scale) as a differentiable torch scalar: x, y
    float32 (n x d, m x d), a, b float64 device tensors; eps a value or a
    ladder (the last entry is the target)."""
    ladder = [float(e) for e in (eps if hasattr(eps, "__len__") else [eps])]
    return _EntropicOTLoss.apply(ctx, x, y, a, b, ladder, tol, max_iter, ell, warm_mode, cost_scale)


def coupling(ctx, prob: Problem, eps: float, f, g, stream=None):
    import torch
    n, m = int(prob.a.shape[0]), int(prob.b.shape[0])
    P = torch.empty((n, m), dtype=torch.float32, device=f.device)
    ps = prob.c_struct()
    _check(lib.sknr_coupling(ctx.handle, ctypes.byref(ps), eps, _ptr(f), _ptr(g), _ptr(P), _stream(stream)),
           "sknr_coupling")
    return P
