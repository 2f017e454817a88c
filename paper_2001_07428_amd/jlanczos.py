"""Python binding of libjlanczos.so (ctypes).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch provides device memory (tensors, including the solver
workspace) and the stream (torch's current stream on the tensor's device).

Vectors are passed as torch tensors of shape (k, n) -- row r is the r-th
column of the column-major n x k block the C ABI expects (leading dimension
n).  complex64 selects the mixed-precision solver (FP32 storage, FP64
reductions and Ritz problem), complex128 the FP64 solver.

The library is required: importing works without it, but every call raises
if libjlanczos.so has not been built (python -m paper_2001_07428_amd.build).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjlanczos.so")

JL_OK, JL_EINVAL, JL_EHIP, JL_ENOMEM, JL_EUNSUPPORTED = 0, -1, -2, -3, -4
JL_NOT_CONVERGED, JL_BREAKDOWN = 1, 2
JL_C64, JL_C128 = 1, 2
JL_LOWEST, JL_LARGEST = 0, 1

EXPORTS = (
    "jl_ctx_create", "jl_ctx_destroy", "jl_last_error", "jl_status_string",
    "jl_op_create_dense", "jl_op_create_stencil", "jl_op_create_tek", "jl_op_destroy", "jl_op_dim",
    "jl_op_apply", "jl_workspace_bytes", "jl_solve", "jl_pair_vectors",
    "jl_reorth_pass_workspace_bytes", "jl_reorth_pass", "jl_reorth_pass_noalloc",
    "jl_ritz_workspace_bytes", "jl_ritz",
    "jl_ritz_restart_workspace_bytes", "jl_ritz_restart",
    "jl_basis_update", "jl_batch_workspace_bytes", "jl_batch_create", "jl_batch_shape_used",
    "jl_batch_run", "jl_batch_destroy",
)


class JlParams(ctypes.Structure):
    _fields_ = [
        ("nev", ctypes.c_int32), ("m", ctypes.c_int32), ("mwin", ctypes.c_int32),
        ("which", ctypes.c_int32), ("tol", ctypes.c_double), ("tol_relative", ctypes.c_int32),
        ("max_cycles", ctypes.c_int32),
        ("max_passes", ctypes.c_int32), ("min_passes", ctypes.c_int32), ("timing", ctypes.c_int32),
        ("trace_cap", ctypes.c_int32),
        ("trace_ab", ctypes.POINTER(ctypes.c_double)), ("verbose", ctypes.c_int32),
        ("standard", ctypes.c_int32), ("invert", ctypes.c_int32), ("cg_maxit", ctypes.c_int32),
        ("cg_tol", ctypes.c_double), ("b0_rule", ctypes.c_int32), ("basis_cycle", ctypes.c_int32),
        ("basis_out", ctypes.c_void_p), ("T_out", ctypes.POINTER(ctypes.c_double)),
        ("cycle_times_cap", ctypes.c_int32), ("cycle_times", ctypes.POINTER(ctypes.c_double)),
    ]


class JlStats(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int32), ("n_mv", ctypes.c_int32), ("n_resid", ctypes.c_int32),
        ("gs_passes", ctypes.c_int32), ("icnv", ctypes.c_int32), ("status", ctypes.c_int32),
        ("sum_ncol", ctypes.c_int64), ("t_total", ctypes.c_double), ("t_matvec", ctypes.c_double), ("t_dots", ctypes.c_double),
        ("t_update", ctypes.c_double), ("t_gemm", ctypes.c_double), ("t_ritz", ctypes.c_double),
        ("t_resid", ctypes.c_double),
        ("n_matvec_launch", ctypes.c_int64), ("n_dots_launch", ctypes.c_int64),
        ("n_update_launch", ctypes.c_int64), ("n_gemm_launch", ctypes.c_int64),
        ("bytes_matvec", ctypes.c_double), ("bytes_dots", ctypes.c_double),
        ("bytes_update", ctypes.c_double), ("flops_gemm", ctypes.c_double),
        ("cg_iters", ctypes.c_int64), ("cg_max_iters", ctypes.c_int32),
        ("cg_unconverged", ctypes.c_int32), ("t_cg", ctypes.c_double),
        ("bytes_cg", ctypes.c_double),
    ]

    def to_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class JlBatchShape(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("rows_per_wave", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("lds_matrix_bytes", ctypes.c_int32)]

    def to_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class JlBatchStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("n_mv", ctypes.c_int32),
                ("gs_passes", ctypes.c_int32), ("icnv", ctypes.c_int32),
                ("n_resid", ctypes.c_int32), ("t_apply", ctypes.c_double),
                ("t_gs", ctypes.c_double), ("t_ritz", ctypes.c_double),
                ("t_restart", ctypes.c_double), ("t_resid", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libjlanczos.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2001_07428_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "jl_ctx_create": (i32, [ctypes.POINTER(vp), i32, vp]),
        "jl_ctx_destroy": (i32, [vp]),
        "jl_last_error": (ctypes.c_char_p, [vp]),
        "jl_status_string": (ctypes.c_char_p, [i32]),
        "jl_op_create_dense": (i32, [vp, i64, vp, vp, i64, i32, ctypes.POINTER(vp)]),
        "jl_op_create_stencil": (i32, [vp, ctypes.POINTER(i32), i32, dbl, dbl, vp, vp, i32, i32,
                                       ctypes.POINTER(vp)]),
        "jl_op_create_tek": (i32, [vp, i32, dbl, vp, i32, ctypes.POINTER(vp)]),
        "jl_op_destroy": (i32, [vp]),
        "jl_op_dim": (i32, [vp, ctypes.POINTER(i64)]),
        "jl_op_apply": (i32, [vp, vp, vp, i32]),
        "jl_workspace_bytes": (i32, [vp, ctypes.POINTER(JlParams), ctypes.POINTER(ctypes.c_size_t)]),
        "jl_solve": (i32, [vp, ctypes.POINTER(JlParams), vp, vp, ctypes.c_size_t,
                           ctypes.POINTER(dbl), vp, i64, ctypes.POINTER(dbl), ctypes.POINTER(JlStats)]),
        "jl_pair_vectors": (i32, [vp, i64, i32, i32, vp, i64, vp, i64]),
        "jl_reorth_pass_workspace_bytes": (i32, [i64, i32, ctypes.POINTER(ctypes.c_size_t)]),
        "jl_reorth_pass": (i32, [vp, i32, i64, i32, vp, i64, vp, vp, vp, ctypes.c_size_t]),
        "jl_reorth_pass_noalloc": (i32, [vp, i32, i64, i32, vp, i64, vp, vp]),
        "jl_ritz_workspace_bytes": (i32, [i32, ctypes.POINTER(ctypes.c_size_t)]),
        "jl_ritz": (i32, [vp, i32, vp, i32, vp, vp, vp, ctypes.c_size_t]),
        "jl_ritz_restart_workspace_bytes": (i32, [i32, ctypes.POINTER(ctypes.c_size_t)]),
        "jl_ritz_restart": (i32, [vp, i32, i32, ctypes.POINTER(ctypes.c_double), i32, vp, vp, vp,
                                  ctypes.c_size_t]),
        "jl_basis_update": (i32, [vp, i32, i64, i32, i32, vp, i64, vp, i64, vp, i64]),
        "jl_batch_workspace_bytes": (i32, [i32, ctypes.POINTER(i64), i32, ctypes.POINTER(JlParams),
                                           ctypes.POINTER(JlBatchShape),
                                           ctypes.POINTER(ctypes.c_size_t)]),
        "jl_batch_create": (i32, [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  i32, ctypes.POINTER(JlParams), ctypes.POINTER(vp), vp,
                                  ctypes.c_size_t, ctypes.POINTER(JlBatchShape), ctypes.POINTER(vp)]),
        "jl_batch_shape_used": (i32, [vp, ctypes.POINTER(JlBatchShape)]),
        "jl_batch_run": (i32, [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(i32),
                               ctypes.POINTER(JlBatchStats)]),
        "jl_batch_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class JLError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"jlanczos status {status}: {msg}")
        self.status = status


def _check(status, ctx_handle=None):
    if status < 0:
        lib = load_library()
        msg = lib.jl_last_error(ctx_handle)
        raise JLError(status, msg.decode() if msg else "")
    return status


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.complex64:
        return JL_C64
    if t.dtype == torch.complex128:
        return JL_C128
    raise TypeError(f"expected complex64 or complex128, got {t.dtype}")


class Context:
    """jl_ctx on the device of `device`, ordered on torch's current stream."""

    def __init__(self, device=0, stream=None):
        torch = _torch()
        lib = load_library()
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.device = dev
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.jl_ctx_create(ctypes.byref(h), dev.index or 0, ctypes.c_void_p(stream.cuda_stream)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load_library().jl_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """jl_op; keeps the tensors it borrows alive."""

    def __init__(self, ctx: Context, handle, keep, n, dtype):
        self.ctx, self.handle, self._keep, self.n, self.dtype = ctx, handle, keep, n, dtype

    def close(self):
        if getattr(self, "handle", None):
            load_library().jl_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def jl_op_create_dense(ctx: Context, A11, A12) -> Operator:
    """Dense operator from device tensors A11, A12 (h x h, row-major, same dtype)."""
    lib = load_library()
    if A11.shape != A12.shape or A11.dim() != 2 or A11.shape[0] != A11.shape[1]:
        raise ValueError("A11 and A12 must be square with the same shape")
    if A11.dtype != A12.dtype:
        raise TypeError("A11 and A12 must share a dtype")
    if A11.stride(1) != 1 or A12.stride(1) != 1 or A11.stride(0) != A12.stride(0):
        raise ValueError("A11 and A12 must be row-major with the same row stride")
    h = A11.shape[0]
    op = ctypes.c_void_p()
    _check(lib.jl_op_create_dense(ctx.handle, 2 * h, ctypes.c_void_p(A11.data_ptr()),
                                  ctypes.c_void_p(A12.data_ptr()), A11.stride(0), _dtype_code(A11),
                                  ctypes.byref(op)), ctx.handle)
    return Operator(ctx, op, (A11, A12), 2 * h, A11.dtype)


def jl_op_create_stencil(ctx: Context, L, U, B, diag=8.1, a12_scale=0.3) -> Operator:
    """4D J-stencil from device tensors U (4, V, 4, 4) and B (4, 4, 4) or (4, V, 4, 4)."""
    lib = load_library()
    L = tuple(int(x) for x in (L if not np.isscalar(L) else (L,) * 4))
    V = int(np.prod(L))
    if tuple(U.shape) != (4, V, 4, 4) or not U.is_contiguous():
        raise ValueError(f"U must be contiguous (4, {V}, 4, 4)")
    per_site = B.dim() == 4
    if not B.is_contiguous() or tuple(B.shape) not in ((4, 4, 4), (4, V, 4, 4)):
        raise ValueError("B must be contiguous (4, 4, 4) or (4, V, 4, 4)")
    if U.dtype != B.dtype:
        raise TypeError("U and B must share a dtype")
    Larr = (ctypes.c_int32 * 4)(*L)
    op = ctypes.c_void_p()
    _check(lib.jl_op_create_stencil(ctx.handle, Larr, 4, float(diag), float(a12_scale),
                                    ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                    int(per_site), _dtype_code(U), ctypes.byref(op)), ctx.handle)
    return Operator(ctx, op, (U, B), 2 * V * 4, U.dtype)


def jl_op_create_tek(ctx: Context, U, kappa) -> Operator:
    """Case B operator A = D D^H (twisted Eguchi-Kawai Wilson-Dirac, J = C gamma_5)
    from device links U of shape (4, N, N); vectors in the layout
    [psi_0; psi_2; psi_1; psi_3] of su(N) coefficients (n = 4 (N^2 - 1))."""
    lib = load_library()
    if U.dim() != 3 or U.shape[0] != 4 or U.shape[1] != U.shape[2] or not U.is_contiguous():
        raise ValueError("U must be contiguous (4, N, N)")
    N = int(U.shape[1])
    op = ctypes.c_void_p()
    _check(lib.jl_op_create_tek(ctx.handle, N, float(kappa), ctypes.c_void_p(U.data_ptr()),
                                _dtype_code(U), ctypes.byref(op)), ctx.handle)
    return Operator(ctx, op, (U,), 4 * (N * N - 1), U.dtype)


def jl_op_apply(op: Operator, x, y=None):
    """y = A x for x of shape (n,) or (k, n); returns y."""
    torch = _torch()
    lib = load_library()
    x2 = x.reshape(-1, op.n)
    if x2.dtype != op.dtype or not x2.is_contiguous():
        raise ValueError("x must be contiguous with the operator dtype")
    if y is None:
        y = torch.empty_like(x)
    y2 = y.reshape(-1, op.n)
    _check(lib.jl_op_apply(op.handle, ctypes.c_void_p(x2.data_ptr()), ctypes.c_void_p(y2.data_ptr()),
                           x2.shape[0]), op.ctx.handle)
    return y


@dataclass
class SolveResult:
    status: int
    evals: np.ndarray
    X: object          # torch tensor (nev, n)
    res: np.ndarray
    stats: dict
    trace_alpha: np.ndarray | None = None
    trace_beta: np.ndarray | None = None
    basis: object = None              # torch tensor (m_eff + 1, n) of the exported iteration
    T: np.ndarray | None = None       # its projected matrix Tbar ((m + 1) x m, lower triangle)
    cycle_times: np.ndarray | None = None   # wall time [s] at the end of each outer iteration


def _params(nev, m, mwin, tol, which, max_cycles, max_passes, timing, trace_buf, min_passes=0,
            tol_relative=False, verbose=False, standard=False, invert=False, cg_tol=0.0,
            cg_maxit=0, b0_rule=0):
    p = JlParams()
    p.b0_rule = int(b0_rule)
    p.standard = int(bool(standard))
    p.invert = int(bool(invert))
    p.cg_tol = float(cg_tol)
    p.cg_maxit = int(cg_maxit)
    p.nev, p.m, p.mwin = nev, m, mwin
    p.which = JL_LARGEST if which in ("largest", JL_LARGEST) else JL_LOWEST
    p.tol = float(tol)
    p.tol_relative = int(bool(tol_relative))
    p.verbose = int(bool(verbose))
    p.max_cycles = int(max_cycles)
    p.max_passes = int(max_passes)
    p.min_passes = int(min_passes)
    p.timing = int(timing) if not isinstance(timing, bool) else int(timing)
    if trace_buf is not None:
        p.trace_cap = len(trace_buf) // 2
        p.trace_ab = trace_buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    else:
        p.trace_cap = 0
        p.trace_ab = None
    return p


def jl_workspace_bytes(op: Operator, nev, m, mwin, tol=1e-10, which="lowest", standard=False,
                       invert=False) -> int:
    lib = load_library()
    p = _params(nev, m, mwin, tol, which, 0, 0, 0, None, standard=standard, invert=invert)
    nb = ctypes.c_size_t()
    _check(lib.jl_workspace_bytes(op.handle, ctypes.byref(p), ctypes.byref(nb)), op.ctx.handle)
    return nb.value


def jl_solve(op: Operator, nev, m, mwin, tol, which="lowest", v1=None, max_cycles=0,
             max_passes=0, min_passes=0, timing=False, trace_cap=0, workspace=None,
             tol_relative=False, verbose=False, standard=False, invert=False, cg_tol=0.0,
             cg_maxit=0, b0_rule=0, basis_cycle=0, cycle_times_cap=0) -> SolveResult:
    """Thick-restart J-Lanczos for the nev lowest (or largest) pairs
    (standard=True: the standard thick-restart Lanczos without the
    J-restriction, which finds every pair twice; invert=True: the Lanczos
    steps take A^-1 v_j by conjugate gradients, for positive definite A).
    b0_rule=1 takes the first sqrt(2) test against the norm after t_jj v_j
    alone (Alg. 2 as printed); basis_cycle=c > 0 returns the Lanczos basis
    and Tbar of outer iteration c in .basis / .T; cycle_times_cap=C returns
    the wall time at the end of each of the first C outer iterations."""
    torch = _torch()
    lib = load_library()
    trace_buf = np.zeros(2 * trace_cap) if trace_cap else None
    p = _params(nev, m, mwin, tol, which, max_cycles, max_passes, timing, trace_buf, min_passes,
                tol_relative, verbose, standard, invert, cg_tol, cg_maxit, b0_rule)
    basis = T_out = ctimes = None
    if basis_cycle > 0:
        basis = torch.zeros((m + 1, op.n), dtype=op.dtype, device=op.ctx.device)
        T_out = np.zeros((m, m + 1))   # row j = column j of the column-major (m + 1) x m Tbar
        p.basis_cycle = int(basis_cycle)
        p.basis_out = ctypes.c_void_p(basis.data_ptr())
        p.T_out = T_out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if cycle_times_cap > 0:
        ctimes = np.full(cycle_times_cap, np.nan)
        p.cycle_times_cap = int(cycle_times_cap)
        p.cycle_times = ctimes.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    nb = ctypes.c_size_t()
    _check(lib.jl_workspace_bytes(op.handle, ctypes.byref(p), ctypes.byref(nb)), op.ctx.handle)
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=op.ctx.device)
    X = torch.empty((nev, op.n), dtype=op.dtype, device=op.ctx.device)
    evals = np.zeros(nev)
    res = np.zeros(nev)
    st = JlStats()
    if v1 is not None:
        v1 = v1.reshape(op.n)
        if v1.dtype != op.dtype or not v1.is_contiguous():
            raise ValueError("v1 must be contiguous with the operator dtype")
    status = lib.jl_solve(op.handle, ctypes.byref(p),
                          ctypes.c_void_p(v1.data_ptr()) if v1 is not None else None,
                          ctypes.c_void_p(workspace.data_ptr()), nb.value,
                          evals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          ctypes.c_void_p(X.data_ptr()), op.n,
                          res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(st))
    _check(status, op.ctx.handle)
    out = SolveResult(status, evals, X, res, st.to_dict())
    if basis is not None:
        out.basis, out.T = basis, T_out.T.copy()
    if ctimes is not None:
        out.cycle_times = ctimes[:min(cycle_times_cap, out.stats["cycles"])]
    if trace_buf is not None:
        out.trace_alpha = trace_buf[:trace_cap].copy()
        out.trace_beta = trace_buf[trace_cap:].copy()
    return out


def jl_pair_vectors(ctx: Context, X, Y=None):
    """Y = J X^* for X of shape (k, n)."""
    torch = _torch()
    lib = load_library()
    X2 = X.reshape(-1, X.shape[-1])
    if Y is None:
        Y = torch.empty_like(X2)
    n = X2.shape[1]
    _check(lib.jl_pair_vectors(ctx.handle, n, X2.shape[0], _dtype_code(X2),
                               ctypes.c_void_p(X2.data_ptr()), n, ctypes.c_void_p(Y.data_ptr()), n),
           ctx.handle)
    return Y


# ------------------------------------------------------------ step-level calls
def jl_reorth_pass(ctx: Context, V, u):
    """One J-restricted block Gram-Schmidt pass of u (n,) against the rows of
    V (ncol, n); u is updated in place.  Returns the FP64 coefficient tensor
    [4*ncol + 2] (Re/Im c_v, Re/Im c_w per column, ||u||^2 before, after)."""
    torch = _torch()
    lib = load_library()
    n = u.shape[-1]
    ncol = 0 if V is None else V.shape[0]
    nb = ctypes.c_size_t()
    _check(lib.jl_reorth_pass_workspace_bytes(n, ncol, ctypes.byref(nb)))
    ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=ctx.device)
    coef = torch.empty(4 * ncol + 2, dtype=torch.float64, device=ctx.device)
    _check(lib.jl_reorth_pass(ctx.handle, _dtype_code(u), n, ncol,
                              ctypes.c_void_p(V.data_ptr()) if ncol else None, n,
                              ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(coef.data_ptr()),
                              ctypes.c_void_p(ws.data_ptr()), nb.value), ctx.handle)
    return coef


def jl_reorth_pass_noalloc(ctx: Context, V, u, coef):
    """As jl_reorth_pass, with the library's static scratch (no workspace,
    no device allocation): coef is the caller's FP64 device tensor of at least
    4*ncol + 2 entries, filled as jl_reorth_pass returns it."""
    lib = load_library()
    n = u.shape[-1]
    ncol = 0 if V is None else V.shape[0]
    if coef.dtype != _torch().float64 or coef.numel() < 4 * ncol + 2 or not coef.is_contiguous():
        raise ValueError("coef must be a contiguous float64 tensor of >= 4*ncol + 2 entries")
    _check(lib.jl_reorth_pass_noalloc(ctx.handle, _dtype_code(u), n, ncol,
                                      ctypes.c_void_p(V.data_ptr()) if ncol else None, n,
                                      ctypes.c_void_p(u.data_ptr()),
                                      ctypes.c_void_p(coef.data_ptr())), ctx.handle)
    return coef


def jl_ritz(ctx: Context, T, which="lowest"):
    """Eigen-decomposition of the real symmetric FP64 device matrix T (m, m),
    sorted; returns (lam (m,), Z (m, m) with eigenvectors as columns)."""
    torch = _torch()
    lib = load_library()
    m = T.shape[0]
    Tc = T.t().contiguous()   # column-major
    nb = ctypes.c_size_t()
    _check(lib.jl_ritz_workspace_bytes(m, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=ctx.device)
    lam = torch.empty(m, dtype=torch.float64, device=ctx.device)
    Zc = torch.empty((m, m), dtype=torch.float64, device=ctx.device)   # rows = eigenvectors
    _check(lib.jl_ritz(ctx.handle, m, ctypes.c_void_p(Tc.data_ptr()),
                       JL_LARGEST if which == "largest" else JL_LOWEST,
                       ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(Zc.data_ptr()),
                       ctypes.c_void_p(ws.data_ptr()), nb.value), ctx.handle)
    return lam, Zc.t()


def jl_ritz_restart(ctx: Context, theta, s, alpha, beta, which="lowest"):
    """Rayleigh-Ritz for the restart structure of T_m: kept Ritz values theta
    (k), couplings s (k), then the tridiagonal alpha (m - k) / beta (m - k - 1)
    starting at index k.  Returns (lam (m,), Z (m, m) with eigenvectors as
    columns), sorted like jl_ritz."""
    torch = _torch()
    lib = load_library()
    theta, s = np.asarray(theta, float).ravel(), np.asarray(s, float).ravel()
    alpha, beta = np.asarray(alpha, float).ravel(), np.asarray(beta, float).ravel()
    k, m = len(theta), len(theta) + len(alpha)
    if len(s) != k or len(beta) != max(len(alpha) - 1, 0):
        raise ValueError("inconsistent restart structure")
    packed = np.ascontiguousarray(np.concatenate([theta, s, alpha, beta]))
    nb = ctypes.c_size_t()
    _check(lib.jl_ritz_restart_workspace_bytes(m, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=ctx.device)
    lam = torch.empty(m, dtype=torch.float64, device=ctx.device)
    Zc = torch.empty((m, m), dtype=torch.float64, device=ctx.device)   # rows = eigenvectors
    _check(lib.jl_ritz_restart(ctx.handle, m, k, packed.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               JL_LARGEST if which == "largest" else JL_LOWEST,
                               ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(Zc.data_ptr()),
                               ctypes.c_void_p(ws.data_ptr()), nb.value), ctx.handle)
    return lam, Zc.t()


def jl_basis_update(ctx: Context, V, Z):
    """Y = V Z for basis rows V (m, n) complex and real Z (m, k); returns (k, n)."""
    torch = _torch()
    lib = load_library()
    m, n = V.shape
    k = Z.shape[1]
    Zc = Z.to(torch.float64).t().contiguous()        # column-major m x k
    Y = torch.empty((k, n), dtype=V.dtype, device=V.device)
    _check(lib.jl_basis_update(ctx.handle, _dtype_code(V), n, m, k, ctypes.c_void_p(V.data_ptr()), n,
                               ctypes.c_void_p(Zc.data_ptr()), m, ctypes.c_void_p(Y.data_ptr()), n),
           ctx.handle)
    return Y


# ---------------------------------------------------------------- batched solve
class Batch:
    """jl_batch: many dense problems solved by one persistent launch replayed
    from a hipGraph.  A11s/A12s: lists of device tensors (h_i x h_i, same
    dtype); eigenvectors land in self.X[i] (nev, n_i)."""

    def __init__(self, ctx: Context, A11s, A12s, nev, m, mwin, tol, which="lowest",
                 tol_relative=False, max_cycles=0, shape=None, standard=False, invert=False):
        """shape: dict of jl_batch_shape knobs (threads, blocks, rows_per_wave,
        unroll, lds_matrix_bytes); None takes the autotuner's cached shape for
        this batch and device, or the library defaults (with a warning)."""
        torch = _torch()
        lib = load_library()
        count = len(A11s)
        if count != len(A12s) or count == 0:
            raise ValueError("A11s and A12s must be non-empty lists of equal length")
        dt = A11s[0].dtype
        for a, b in zip(A11s, A12s):
            if a.dtype != dt or b.dtype != dt or a.shape != b.shape or not a.is_contiguous() \
                    or not b.is_contiguous() or a.dim() != 2 or a.shape[0] != a.shape[1]:
                raise ValueError("every A11/A12 must be a contiguous square tensor of one dtype")
        self.ctx, self.count, self.nev = ctx, count, nev
        self.n = np.array([2 * a.shape[0] for a in A11s], dtype=np.int64)
        self.tuned = False
        if shape is None:   # shape from the autotuner's cache, if any
            from . import tune
            shape = tune.lookup(self.n, nev, m, "c64" if dt == torch.complex64 else "c128")
            if shape is not None:
                self.tuned = True
            else:
                import warnings
                warnings.warn(f"no tuned launch shape for this batch and device {tune.device_key()} "
                              "(python -m paper_2001_07428_amd.tune): library defaults")
                shape = {}
        self._shape = JlBatchShape(**{k: int(v) for k, v in shape.items()})
        self.p = _params(nev, m, mwin, tol, which, max_cycles, 0, 0, None, 0, tol_relative, False,
                         standard, invert)
        code = _dtype_code(A11s[0])
        nb = ctypes.c_size_t()
        n_c = self.n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        _check(lib.jl_batch_workspace_bytes(count, n_c, code, ctypes.byref(self.p),
                                            ctypes.byref(self._shape), ctypes.byref(nb)), ctx.handle)
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=ctx.device)
        self.X = [torch.empty((nev, int(ni)), dtype=dt, device=ctx.device) for ni in self.n]
        vp = ctypes.c_void_p
        a11 = (vp * count)(*[a.data_ptr() for a in A11s])
        a12 = (vp * count)(*[a.data_ptr() for a in A12s])
        xs = (vp * count)(*[x.data_ptr() for x in self.X])
        self._keep = (A11s, A12s)
        h = vp()
        _check(lib.jl_batch_create(ctx.handle, count, n_c, a11, a12, code, ctypes.byref(self.p), xs,
                                   vp(self.ws.data_ptr()), nb.value, ctypes.byref(self._shape),
                                   ctypes.byref(h)), ctx.handle)
        self.handle = h
        used = JlBatchShape()
        _check(lib.jl_batch_shape_used(h, ctypes.byref(used)), ctx.handle)
        self.shape = used.to_dict()   # the launch shape in use, defaults resolved
        self.threads, self.blocks = used.threads, used.blocks

    def run(self):
        """Replays the graph; returns (status, evals (count, nev), res, per-problem
        status, stats dict of arrays)."""
        lib = load_library()
        evals = np.zeros((self.count, self.nev))
        res = np.zeros((self.count, self.nev))
        st = np.zeros(self.count, dtype=np.int32)
        stats = (JlBatchStats * self.count)()
        rc = lib.jl_batch_run(self.handle, evals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), stats)
        _check(rc, self.ctx.handle)
        sd = {f: np.array([getattr(x, f) for x in stats]) for f, _ in JlBatchStats._fields_}
        return rc, evals, res, st, sd

    def close(self):
        if getattr(self, "handle", None):
            load_library().jl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
