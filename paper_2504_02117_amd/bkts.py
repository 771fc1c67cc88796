"""Thin ctypes binding of libbkts.so (include/bkts.h).

Argument marshalling only: every step runs in the HIP library.  Functions keep
the C names; device buffers are passed as torch tensors (their ``data_ptr()``)
and the library enqueues on the stream given to :func:`bkts_ctx_create`.

There is no fallback: if ``libbkts.so`` is missing or cannot be loaded this
module raises ``ImportError``.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  -- loads the HIP runtime first, so the library shares it

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbkts.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2504_02117_amd.build`")
_lib = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)

BKTS_MAX_K = 32
BKTS_OK, BKTS_EINVAL, BKTS_ENOMEM, BKTS_EDEVICE, BKTS_EBREAKDOWN, BKTS_ENOCONV, BKTS_EBUSY = 0, -1, -2, -3, -4, -5, -6
BKTS_F64, BKTS_F32 = 0, 1
BKTS_FMT_CSR, BKTS_FMT_SELL, BKTS_FMT_STENCIL = 0, 1, 2
BKTS_BC_DIRICHLET, BKTS_BC_NEUMANN = 0, 1
BKTS_IE, BKTS_THETA, BKTS_SDIRK2, BKTS_DIRK_CUSTOM, BKTS_RADAU2 = 0, 1, 2, 3, 4
BKTS_RI_NO_FLOW, BKTS_RI_DIRICHLET, BKTS_RI_FREE_DRAINAGE = 0, 1, 2
BKTS_WINDOW_FGMRES, BKTS_WINDOW_SPLITTING = 0, 1
BKTS_CG, BKTS_GMRES, BKTS_BICGSTAB = 0, 1, 2
BKTS_PREC_NONE, BKTS_PREC_JACOBI, BKTS_PREC_MG = 0, 1, 2
BKTS_PRECISION_F64, BKTS_PRECISION_F32_REFINE = 0, 1
KERNELS = ("spmm", "gram", "norms", "cg_update", "cg_pupdate", "residual", "small", "cast", "other", "mg_restrict",
           "mg_prolong", "mg_coarse")

_STATUS_NAMES = {0: "BKTS_OK", -1: "BKTS_EINVAL", -2: "BKTS_ENOMEM", -3: "BKTS_EDEVICE",
                 -4: "BKTS_EBREAKDOWN", -5: "BKTS_ENOCONV", -6: "BKTS_EBUSY"}


class BktsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class bkts_grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3)]


class bkts_fv_coeffs(C.Structure):
    _fields_ = [("kappa", C.c_void_p), ("kappa_const", C.c_double), ("velocity", C.c_double * 3),
                ("bc_type", C.c_int * 6), ("bc_value", C.c_double * 6)]


class bkts_tc_desc(C.Structure):
    _fields_ = [("method", C.c_int), ("theta", C.c_double), ("stages", C.c_int), ("A", C.c_void_p),
                ("c", C.c_void_p), ("k", C.c_int), ("tau", C.c_double)]


class bkts_solve_opts(C.Structure):
    _fields_ = [("krylov", C.c_int), ("precond", C.c_int), ("precision", C.c_int), ("rtol", C.c_double),
                ("maxit", C.c_int), ("restart", C.c_int), ("inner_rtol", C.c_double)]


class bkts_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("refinements", C.c_int), ("converged", C.c_int),
                ("deflations", C.c_int), ("max_rel_residual", C.c_double)]


class bkts_run_info(C.Structure):
    _fields_ = [("accepted_steps", C.c_int), ("outer_iterations", C.c_int), ("krylov_iterations", C.c_int),
                ("refinements", C.c_int), ("final_front_rel_residual", C.c_double)]


class bkts_window_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("inner_iterations", C.c_int), ("precond_applications", C.c_int),
                ("converged", C.c_int), ("rel_residual", C.c_double)]


class bkts_nl_coeffs(C.Structure):
    _fields_ = [("dcoef", C.c_double * 4), ("rcoef", C.c_double * 4), ("bc_type", C.c_int * 6),
                ("bc_value", C.c_double * 6)]


class bkts_richards_params(C.Structure):
    _fields_ = [("theta_r", C.c_double), ("theta_s", C.c_double), ("alpha", C.c_double), ("n", C.c_double),
                ("top", C.c_int), ("top_value", C.c_double), ("bottom", C.c_int), ("lin_L", C.c_double)]


class bkts_request(C.Structure):
    _fields_ = [("grid", bkts_grid), ("kappa", C.c_void_p), ("kappa_const", C.c_double), ("bc_type", C.c_int * 6),
                ("bc_value", C.c_double * 6), ("y0", C.c_void_p), ("y_out", C.c_void_p), ("method", C.c_int),
                ("theta", C.c_double), ("k", C.c_int), ("tau", C.c_double), ("rtol", C.c_double),
                ("inner_rtol", C.c_double), ("max_outer", C.c_int), ("max_inner", C.c_int), ("tag", C.c_uint64),
                ("mode", C.c_int), ("window", C.c_int)]


class bkts_result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_int), ("outer_iterations", C.c_int),
                ("krylov_iterations", C.c_int), ("rel_residual", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("footprint_bytes", C.c_size_t)]


class bkts_server_stats(C.Structure):
    _fields_ = [("queued", C.c_int), ("active", C.c_int), ("done_unpolled", C.c_int), ("max_active", C.c_int),
                ("rounds", C.c_long), ("grouped_launches", C.c_long), ("bytes_in_use", C.c_size_t),
                ("bytes_peak", C.c_size_t)]


bkts_step_cb = C.CFUNCTYPE(None, C.c_int, C.c_double, C.c_void_p, C.c_void_p)

_P, _I, _D, _I64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
_SIGS = {
    "bkts_ctx_create": (_I, [_I, _P, C.POINTER(_P)]),
    "bkts_ctx_destroy": (None, [_P]),
    "bkts_ctx_synchronize": (_I, [_P]),
    "bkts_last_error": (C.c_char_p, []),
    "bkts_version": (C.c_char_p, []),
    "bkts_fv_assemble": (_I, [_P, C.POINTER(bkts_grid), C.POINTER(bkts_fv_coeffs), _I, C.POINTER(_P)]),
    "bkts_op_create_csr": (_I, [_P, _I64, _I64, _P, _P, _P, _I, C.POINTER(_P)]),
    "bkts_op_info": (_I, [_P, C.POINTER(_I64), C.POINTER(_I64)]),
    "bkts_op_export_csr": (_I, [_P, _P, _P, _P, _P]),
    "bkts_op_destroy": (None, [_P]),
    "bkts_spmm": (_I, [_P, _P, _I, _I, _D, _D, _P, _I, _P, _I]),
    "bkts_gram": (_I, [_P, _I, _I64, _I, _P, _I, _P, _I, _P]),
    "bkts_gram_noalloc": (_I, [_P, _I, _I64, _I, _P, _I, _P, _I, _P]),
    "bkts_mg_apply": (_I, [_P, _P, _I, _I, _D, _D, _P, _I, _P, _I]),
    "bkts_tc_create": (_I, [_P, C.POINTER(bkts_tc_desc), C.POINTER(_P)]),
    "bkts_tc_get": (_I, [_P, _I, _P, _P, C.POINTER(_D), C.POINTER(_I), C.POINTER(_I)]),
    "bkts_tc_destroy": (None, [_P]),
    "bkts_residual": (_I, [_P, _P, _P, _I, _P, _I, _P, _I, _I, _P, _I, _P]),
    "bkts_block_solve": (_I, [_P, _P, _D, _D, _I, _P, _I, _P, _I, C.POINTER(bkts_solve_opts),
                              C.POINTER(bkts_solve_info)]),
    "bkts_advance": (_I, [_P, _P, _P, _P, _I, C.POINTER(bkts_solve_opts), _D, _I, _P, bkts_step_cb, _P,
                          C.POINTER(bkts_run_info)]),
    "bkts_window_solve": (_I, [_P, _P, _P, _I, _P, _I, _I, _P, _I, C.POINTER(bkts_solve_opts), _D, _I, _I,
                               C.POINTER(bkts_window_info)]),
    "bkts_profile_enable": (_I, [_P, _I]),
    "bkts_profile_query": (_I, [_P, _I, C.POINTER(_I64), C.POINTER(_D), C.POINTER(_D)]),
    "bkts_profile_samples": (_I, [_P, _I, _P, _I, C.POINTER(_I)]),
    "bkts_stepper_create": (_I, [_P, _P, _P, _P, C.POINTER(_P)]),
    "bkts_stepper_advance": (_I, [_P, _I, C.POINTER(bkts_solve_opts), _D, _I, _P, bkts_step_cb, _P,
                                  C.POINTER(bkts_run_info)]),
    "bkts_stepper_state": (_I, [_P, _P, C.POINTER(_I64)]),
    "bkts_stepper_destroy": (None, [_P]),
    "bkts_nlop_create": (_I, [_P, C.POINTER(bkts_grid), C.POINTER(bkts_nl_coeffs), C.POINTER(_P)]),
    "bkts_nlop_destroy": (None, [_P]),
    "bkts_nl_eval": (_I, [_P, _P, _I, _P, _I, _P, _I]),
    "bkts_nl_jacobian": (_I, [_P, _P, _P, _D, _D, C.POINTER(_P)]),
    "bkts_nl_residual": (_I, [_P, _P, _P, _I, _P, _I, _P, _I, _I, _P, _I, _P]),
    "bkts_newton_step": (_I, [_P, _P, _P, _I, _P, _I, _I, _P, _P, C.POINTER(bkts_solve_opts),
                              C.POINTER(bkts_solve_info)]),
    "bkts_nl_stepper_create": (_I, [_P, _P, _P, _P, C.POINTER(_P)]),
    "bkts_richards_create": (_I, [_P, C.POINTER(bkts_grid), _P, C.POINTER(bkts_richards_params), C.POINTER(_P)]),
    "bkts_nl_mass": (_I, [_P, _P, _I, _P, _I, _P, _I]),
    "bkts_server_create": (_I, [_P, C.c_size_t, _I, C.POINTER(_P)]),
    "bkts_server_submit": (_I, [_P, C.POINTER(bkts_request), C.POINTER(C.c_uint64)]),
    "bkts_server_poll": (_I, [_P, C.POINTER(bkts_result), _I, C.POINTER(_I)]),
    "bkts_server_wait": (_I, [_P, _I, _D, C.POINTER(_I)]),
    "bkts_server_stats_get": (_I, [_P, C.POINTER(bkts_server_stats)]),
    "bkts_server_clock": (_D, [_P]),
    "bkts_server_destroy": (None, [_P]),
}

EXPORTED = tuple(_SIGS)

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(status):
    if status != BKTS_OK:
        raise BktsError(status, _lib.bkts_last_error().decode())
    return status


def _ptr(t):
    """Device (or host) address of a tensor / numpy array / None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data  # numpy


def _f64_host(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------- raw C names

def bkts_last_error():
    return _lib.bkts_last_error().decode()


def bkts_version():
    return _lib.bkts_version().decode()


def bkts_ctx_create(device=0, stream=None):
    out = C.c_void_p()
    s = None if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
    _check(_lib.bkts_ctx_create(device, s, C.byref(out)))
    return out.value


def bkts_ctx_destroy(ctx):
    _lib.bkts_ctx_destroy(ctx)


def bkts_ctx_synchronize(ctx):
    _check(_lib.bkts_ctx_synchronize(ctx))


def bkts_fv_assemble(ctx, n, kappa=None, kappa_const=1.0, velocity=(0.0, 0.0, 0.0), bc_type=None, bc_value=None,
                     fmt=BKTS_FMT_SELL):
    """Assemble the FV operator on the device.  ``n`` is the per-axis cell count (x first);
    ``kappa`` a device float64 tensor with one value per cell, or None."""
    g = bkts_grid()
    g.dim = len(n)
    for d in range(3):
        g.n[d] = int(n[d]) if d < len(n) else 1
    c = bkts_fv_coeffs()
    c.kappa = _ptr(kappa)
    c.kappa_const = float(kappa_const)
    for d in range(3):
        c.velocity[d] = float(velocity[d]) if d < len(velocity) else 0.0
    for f in range(6):
        c.bc_type[f] = BKTS_BC_DIRICHLET if bc_type is None else int(bc_type[f])
        c.bc_value[f] = 0.0 if bc_value is None else float(bc_value[f])
    out = C.c_void_p()
    _check(_lib.bkts_fv_assemble(ctx, C.byref(g), C.byref(c), fmt, C.byref(out)))
    return out.value


def bkts_op_create_csr(ctx, N, nnz, rowptr, col, val, fmt=BKTS_FMT_CSR):
    out = C.c_void_p()
    _check(_lib.bkts_op_create_csr(ctx, N, nnz, _ptr(rowptr), _ptr(col), _ptr(val), fmt, C.byref(out)))
    return out.value


def bkts_op_info(op):
    N, nnz = C.c_int64(), C.c_int64()
    _check(_lib.bkts_op_info(op, C.byref(N), C.byref(nnz)))
    return N.value, nnz.value


def bkts_op_export_csr(op):
    import numpy as np
    N, nnz = bkts_op_info(op)
    rowptr = np.empty(N + 1, np.int32)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    b = np.empty(N, np.float64)
    _check(_lib.bkts_op_export_csr(op, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(b)))
    return rowptr, col, val, b


def bkts_op_destroy(op):
    _lib.bkts_op_destroy(op)


def _dtype_code(t):
    return BKTS_F32 if str(t.dtype) == "torch.float32" else BKTS_F64


def bkts_spmm(ctx, op, X, Y, alpha=0.0, beta=1.0):
    """Y = alpha X + beta K X for (N, k) device tensors (float64 or float32)."""
    k = X.shape[1]
    _check(_lib.bkts_spmm(ctx, op, _dtype_code(X), k, alpha, beta, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0)))


def bkts_gram(ctx, X, Y, G):
    """G (k x k float64 device tensor) = X^T Y."""
    N, k = X.shape
    _check(_lib.bkts_gram(ctx, _dtype_code(X), N, k, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0), _ptr(G)))


def bkts_gram_noalloc(ctx, X, Y, G):
    """G (k x k float64 device tensor) = X^T Y, partials in the library's fixed scratch array."""
    N, k = X.shape
    _check(_lib.bkts_gram_noalloc(ctx, _dtype_code(X), N, k, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0), _ptr(G)))


def bkts_mg_apply(ctx, op, F, Z, a, b):
    """Z = one multigrid V-cycle applied to F (contiguous N x k device tensors) for a I + b K."""
    N, k = F.shape
    _check(_lib.bkts_mg_apply(ctx, op, _dtype_code(F), k, a, b, _ptr(F), F.stride(0), _ptr(Z), Z.stride(0)))


def bkts_tc_create(ctx, method, k, tau, theta=0.5, A=None, c=None):
    d = bkts_tc_desc()
    d.method = method
    d.theta = theta
    d.k = k
    d.tau = tau
    keep = []
    if method == BKTS_DIRK_CUSTOM:
        A_ = _f64_host(A)
        c_ = _f64_host(c)
        keep = [A_, c_]
        d.stages = A_.shape[0]
        d.A = A_.ctypes.data
        d.c = c_.ctypes.data
    out = C.c_void_p()
    _check(_lib.bkts_tc_create(ctx, C.byref(d), C.byref(out)))
    del keep
    return out.value


def bkts_tc_get(tc, phase=0):
    import numpy as np
    k, mi, beta = C.c_int(), C.c_int(), C.c_double()
    _check(_lib.bkts_tc_get(tc, phase, None, None, C.byref(beta), C.byref(k), C.byref(mi)))
    A1 = np.empty((k.value, k.value))
    A2 = np.empty((k.value, k.value))
    _check(_lib.bkts_tc_get(tc, phase, A1.ctypes.data, A2.ctypes.data, None, None, None))
    return A1, A2, beta.value, mi.value


def bkts_tc_destroy(tc):
    _lib.bkts_tc_destroy(tc)


def bkts_residual(ctx, op, tc, Y, R, B0=None, phase=0, want_norms=True):
    import numpy as np
    k = Y.shape[1]
    norms = np.empty(k) if want_norms else None
    nb0 = 0 if B0 is None else B0.shape[1]
    ldb0 = 0 if B0 is None else B0.stride(0)
    _check(_lib.bkts_residual(ctx, op, tc, phase, _ptr(Y), Y.stride(0), _ptr(B0), ldb0, nb0, _ptr(R), R.stride(0),
                              _ptr(norms)))
    return norms


def solve_opts(krylov=BKTS_CG, precond=BKTS_PREC_JACOBI, precision=BKTS_PRECISION_F64, rtol=1e-10, maxit=10000,
               restart=30, inner_rtol=1e-4):
    o = bkts_solve_opts()
    o.krylov, o.precond, o.precision = krylov, precond, precision
    o.rtol, o.maxit, o.restart, o.inner_rtol = rtol, maxit, restart, inner_rtol
    return o


def bkts_block_solve(ctx, op, alpha, beta, B, X, opts=None, raise_on_noconv=True):
    """Solve (alpha I + beta K) X = B in place of X; returns bkts_solve_info."""
    opts = opts or solve_opts()
    info = bkts_solve_info()
    k = B.shape[1]
    st = _lib.bkts_block_solve(ctx, op, alpha, beta, k, _ptr(B), B.stride(0), _ptr(X), X.stride(0), C.byref(opts),
                               C.byref(info))
    if st != BKTS_OK and (raise_on_noconv or st != BKTS_ENOCONV):
        _check(st)
    return info


def bkts_advance(ctx, op, tc, y, n_steps, inner=None, outer_rtol=1e-8, max_outer=200, y_hist=None, cb=None):
    """Algorithm 1 (linear).  ``y``: device float64 tensor (N,), updated in place."""
    inner = inner or solve_opts(rtol=1e-2)
    info = bkts_run_info()
    cfun = bkts_step_cb(cb) if cb is not None else C.cast(None, bkts_step_cb)
    _check(_lib.bkts_advance(ctx, op, tc, _ptr(y), n_steps, C.byref(inner), outer_rtol, max_outer, _ptr(y_hist), cfun,
                             None, C.byref(info)))
    return info


def bkts_window_solve(ctx, op, tc, Y, B0=None, phase=0, method=BKTS_WINDOW_FGMRES, inner=None, rtol=1e-8,
                      restart=30, maxit=200, raise_on_noconv=True):
    """Solve the all-at-once window system for the (N, k) float64 device tensor Y in place (Y is the
    initial guess); returns bkts_window_info."""
    inner = inner or solve_opts(rtol=1e-2)
    info = bkts_window_info()
    nb0 = 0 if B0 is None else B0.shape[1]
    ldb0 = 0 if B0 is None else B0.stride(0)
    st = _lib.bkts_window_solve(ctx, op, tc, phase, _ptr(B0), ldb0, nb0, _ptr(Y), method, C.byref(inner), rtol,
                                restart, maxit, C.byref(info))
    if st != BKTS_OK and (raise_on_noconv or st != BKTS_ENOCONV):
        _check(st)
    return info


def bkts_profile_enable(ctx, enable=True, period=1):
    """Enable the per-kernel timers on every `period`-th launch of each kernel id (or disable)."""
    _check(_lib.bkts_profile_enable(ctx, max(1, int(period)) if enable else 0))


def bkts_profile_query(ctx, kernel):
    """(launches, total_ms, algorithmic_bytes) for kernel id or name."""
    kid = KERNELS.index(kernel) if isinstance(kernel, str) else int(kernel)
    n, ms, by = C.c_int64(), C.c_double(), C.c_double()
    _check(_lib.bkts_profile_query(ctx, kid, C.byref(n), C.byref(ms), C.byref(by)))
    return n.value, ms.value, by.value


def bkts_profile_samples(ctx, kernel):
    """The individual timed durations (ms) of kernel id or name, in launch order."""
    kid = KERNELS.index(kernel) if isinstance(kernel, str) else int(kernel)
    n = C.c_int()
    _check(_lib.bkts_profile_samples(ctx, kid, None, 0, C.byref(n)))
    buf = (C.c_float * max(1, n.value))()
    _check(_lib.bkts_profile_samples(ctx, kid, buf, n.value, C.byref(n)))
    return list(buf)[:n.value]


def bkts_stepper_create(ctx, op, tc, y0):
    out = C.c_void_p()
    _check(_lib.bkts_stepper_create(ctx, op, tc, _ptr(y0), C.byref(out)))
    return out.value


def bkts_stepper_advance(st, n_steps, inner=None, outer_rtol=1e-8, max_outer=200, y_hist=None, cb=None):
    inner = inner or solve_opts(rtol=1e-2)
    info = bkts_run_info()
    cfun = bkts_step_cb(cb) if cb is not None else C.cast(None, bkts_step_cb)
    _check(_lib.bkts_stepper_advance(st, n_steps, C.byref(inner), outer_rtol, max_outer, _ptr(y_hist), cfun, None,
                                     C.byref(info)))
    return info


def bkts_stepper_state(st, y=None):
    acc = C.c_int64()
    _check(_lib.bkts_stepper_state(st, _ptr(y), C.byref(acc)))
    return acc.value


def bkts_stepper_destroy(st):
    _lib.bkts_stepper_destroy(st)


def _grid(n):
    g = bkts_grid()
    g.dim = len(n)
    for d in range(3):
        g.n[d] = int(n[d]) if d < len(n) else 1
    return g


def bkts_nlop_create(ctx, n, dcoef=(1.0, 0.0, 0.0, 0.0), rcoef=(0.0, 0.0, 0.0, 0.0), bc_type=None, bc_value=None):
    """Nonlinear FV operator f(u) = -div(D(u) grad u) - r(u); ``dcoef``/``rcoef`` are the
    polynomial coefficients of D and r (constant term first); faces default to zero flux."""
    c = bkts_nl_coeffs()
    for i in range(4):
        c.dcoef[i] = float(dcoef[i]) if i < len(dcoef) else 0.0
        c.rcoef[i] = float(rcoef[i]) if i < len(rcoef) else 0.0
    for f in range(6):
        c.bc_type[f] = BKTS_BC_NEUMANN if bc_type is None else int(bc_type[f])
        c.bc_value[f] = 0.0 if bc_value is None else float(bc_value[f])
    g = _grid(n)
    out = C.c_void_p()
    _check(_lib.bkts_nlop_create(ctx, C.byref(g), C.byref(c), C.byref(out)))
    return out.value


def bkts_nlop_destroy(nl):
    _lib.bkts_nlop_destroy(nl)


def bkts_nl_eval(ctx, nl, Y, F):
    """F[:, j] = f(Y[:, j]) for (N, k) float64 device tensors."""
    k = Y.shape[1]
    _check(_lib.bkts_nl_eval(ctx, nl, k, _ptr(Y), Y.stride(0), _ptr(F), F.stride(0)))


def bkts_nl_jacobian(ctx, nl, u, alpha, beta):
    """Operator handle of alpha I + beta Df(u), owned by ``nl``."""
    out = C.c_void_p()
    _check(_lib.bkts_nl_jacobian(ctx, nl, _ptr(u), alpha, beta, C.byref(out)))
    return out.value


def bkts_nl_residual(ctx, nl, tc, Y, R, B0=None, phase=0, want_norms=True):
    import numpy as np
    k = Y.shape[1]
    norms = np.empty(k) if want_norms else None
    nb0 = 0 if B0 is None else B0.shape[1]
    ldb0 = 0 if B0 is None else B0.stride(0)
    _check(_lib.bkts_nl_residual(ctx, nl, tc, phase, _ptr(Y), Y.stride(0), _ptr(B0), ldb0, nb0, _ptr(R),
                                 R.stride(0), _ptr(norms)))
    return norms


def bkts_newton_step(ctx, nl, tc, Y, B0=None, phase=0, opts=None):
    """One Newton iteration on the window Y (N, k) in place; returns (pre-update column norms^2, info)."""
    import numpy as np
    opts = opts or solve_opts(rtol=1e-2)
    k = Y.shape[1]
    norms = np.empty(k)
    info = bkts_solve_info()
    nb0 = 0 if B0 is None else B0.shape[1]
    ldb0 = 0 if B0 is None else B0.stride(0)
    _check(_lib.bkts_newton_step(ctx, nl, tc, phase, _ptr(B0), ldb0, nb0, _ptr(Y), _ptr(norms), C.byref(opts),
                                 C.byref(info)))
    return norms, info


def bkts_nl_stepper_create(ctx, nl, tc, y0):
    out = C.c_void_p()
    _check(_lib.bkts_nl_stepper_create(ctx, nl, tc, _ptr(y0), C.byref(out)))
    return out.value


def bkts_richards_create(ctx, n, ks, theta_r=0.05, theta_s=0.4, alpha=2.0, vg_n=2.0, top=BKTS_RI_DIRICHLET,
                         top_value=0.0, bottom=BKTS_RI_FREE_DRAINAGE, lin_L=0.0):
    """Richards operator on the grid ``n`` (last axis = height) with the float64 device tensor ``ks``
    of saturated conductivities (copied)."""
    p = bkts_richards_params(theta_r, theta_s, alpha, vg_n, int(top), top_value, int(bottom), lin_L)
    g = _grid(n)
    out = C.c_void_p()
    _check(_lib.bkts_richards_create(ctx, C.byref(g), _ptr(ks), C.byref(p), C.byref(out)))
    return out.value


def bkts_nl_mass(ctx, nl, Y, M):
    """M[:, j] = m(Y[:, j]) for (N, k) float64 device tensors."""
    k = Y.shape[1]
    _check(_lib.bkts_nl_mass(ctx, nl, k, _ptr(Y), Y.stride(0), _ptr(M), M.stride(0)))


def bkts_server_create(ctx, hbm_budget_bytes, max_slots=64):
    out = C.c_void_p()
    _check(_lib.bkts_server_create(ctx, int(hbm_budget_bytes), max_slots, C.byref(out)))
    return out.value


def make_request(n, y0, y_out, k, tau, kappa=None, kappa_const=1.0, method=BKTS_IE, theta=0.5, rtol=1e-8,
                 inner_rtol=1e-2, bc_type=None, bc_value=None, max_outer=0, max_inner=0, tag=0, mode=0, window=0):
    """A serving request; device buffers are torch tensors (y_out: (N, k) float64).  mode 0: grouped
    window splitting; mode 1: pipelined Algorithm 1 with multigrid (implicit Euler), window columns
    (0: min(k, 4))."""
    r = bkts_request()
    r.grid = _grid(n)
    r.kappa = _ptr(kappa)
    r.kappa_const = kappa_const
    for f in range(6):
        r.bc_type[f] = BKTS_BC_DIRICHLET if bc_type is None else int(bc_type[f])
        r.bc_value[f] = 0.0 if bc_value is None else float(bc_value[f])
    r.y0, r.y_out = _ptr(y0), _ptr(y_out)
    r.method, r.theta, r.k, r.tau = method, theta, k, tau
    r.rtol, r.inner_rtol, r.max_outer, r.max_inner, r.tag = rtol, inner_rtol, max_outer, max_inner, tag
    r.mode, r.window = mode, window
    return r


def bkts_server_submit(srv, req):
    t = C.c_uint64()
    _check(_lib.bkts_server_submit(srv, C.byref(req), C.byref(t)))
    return t.value


def bkts_server_poll(srv, max_results=64):
    buf = (bkts_result * max_results)()
    n = C.c_int()
    _check(_lib.bkts_server_poll(srv, buf, max_results, C.byref(n)))
    return [buf[i] for i in range(n.value)]


def bkts_server_wait(srv, n, timeout_s):
    r = C.c_int()
    _check(_lib.bkts_server_wait(srv, n, timeout_s, C.byref(r)))
    return r.value


def bkts_server_stats_get(srv):
    s = bkts_server_stats()
    _check(_lib.bkts_server_stats_get(srv, C.byref(s)))
    return s


def bkts_server_clock(srv):
    return _lib.bkts_server_clock(srv)


def bkts_server_destroy(srv):
    _lib.bkts_server_destroy(srv)
