"""Interior singular triplets of large sparse matrices on AMD MI355X (gfx950).

Python binding of the C ABI declared in ``include/csvd.h``: every function
here has the same name as its C counterpart and only marshals arguments
(NumPy arrays in and out, ctypes structs for the parameter and info
records).  All computation runs in ``libcsvd.so`` (hand-written HIP kernels
for gfx950 plus the host orchestration in C++).  Importing the package does
not touch the GPU; the library is loaded on first use and a missing library
raises immediately instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "CsvdError", "csvd_params", "csvd_info", "load", "lib_path",
    "csvd_params_default", "csvd_create", "csvd_solve_interval", "csvd_get_triplets",
    "csvd_get_info", "csvd_get_residual_estimates", "csvd_get_moment", "csvd_get_solution", "csvd_quadrature", "csvd_spmm", "csvd_spmm_noalloc", "csvd_probe_gather",
    "csvd_get_transpose", "csvd_dense_gemm", "csvd_last_error", "csvd_destroy", "csvd_trim", "csvd_solve_batch",
    "csvd_server_create", "csvd_server_submit", "csvd_server_step", "csvd_server_poll",
    "csvd_server_cancel", "csvd_server_last_error", "csvd_server_destroy",
    "CSVD_OK", "CSVD_EINVAL", "CSVD_ENOMEM", "CSVD_ENOTCONV", "CSVD_EDEVICE", "CSVD_ESTATE",
    "CSVD_ENUMERIC", "CSVD_PLAIN", "CSVD_EXP", "CSVD_FP64", "CSVD_MIXED", "CSVD_SOLVER_AUTO",
    "CSVD_SOLVER_BLOCK", "CSVD_SOLVER_SINGLE",
]

CSVD_OK, CSVD_EINVAL, CSVD_ENOMEM, CSVD_ENOTCONV, CSVD_EDEVICE, CSVD_ESTATE, CSVD_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
CSVD_PLAIN, CSVD_EXP = 0, 1
CSVD_FP64, CSVD_MIXED = 0, 1
CSVD_SOLVER_AUTO, CSVD_SOLVER_BLOCK, CSVD_SOLVER_SINGLE = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libcsvd.so")


class csvd_params(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("M", C.c_int32), ("N", C.c_int32), ("ell", C.c_int32),
        ("delta", C.c_double), ("alpha", C.c_double),
        ("transform", C.c_int32), ("precision", C.c_int32),
        ("solve_rtol", C.c_double), ("max_iters", C.c_int32),
        ("spurious_eps", C.c_double), ("seed", C.c_uint64), ("norm_a", C.c_double),
        ("window", C.c_int32), ("check_solves", C.c_int32), ("solver", C.c_int32),
        ("keep_basis", C.c_int32), ("cholqr_passes", C.c_int32), ("resid_target", C.c_double),
        ("ell_adaptive", C.c_int32),
    ]


class csvd_info(C.Structure):
    _fields_ = [
        ("iterations", C.c_int64), ("iterations_total", C.c_int64),
        ("rank", C.c_int32), ("t_hat", C.c_int32), ("converged", C.c_int32), ("n_shift", C.c_int32),
        ("max_solve_resid_est", C.c_double), ("max_solve_resid_true", C.c_double),
        ("max_triplet_resid", C.c_double), ("norm_a", C.c_double), ("sigma_s1", C.c_double),
        ("t_solve_ms", C.c_double), ("t_lowrank_ms", C.c_double), ("t_qr_ms", C.c_double),
        ("t_extract_ms", C.c_double), ("t_total_ms", C.c_double),
        ("spmm_a_ms", C.c_double), ("spmm_at_ms", C.c_double), ("window_ms", C.c_double),
        ("spmm_samples", C.c_int64),
        ("spmm_a_bytes", C.c_double), ("spmm_at_bytes", C.c_double), ("window_bytes", C.c_double),
        ("window", C.c_int32), ("L_padded", C.c_int32), ("solver", C.c_int32), ("deflated", C.c_int32),
        ("rest_ms", C.c_double), ("basis_stored", C.c_int32), ("one_pass_steps", C.c_int32),
        ("moments_ms", C.c_double), ("svd_sweeps_exhausted", C.c_int32),
        ("column_groups", C.c_int32), ("mixed_refined", C.c_int32), ("dropped", C.c_int32),
        ("mixed_resid_fp32", C.c_double), ("rounds", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CsvdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"csvd error {code}: {msg}")
        self.code = code


_lib = None
_shape = {}  # (m, n) of every live context handle, for argument checks
_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)


def load(build_if_missing: bool = True):
    """Load ``libcsvd.so`` (building it first only when it does not exist)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        if not build_if_missing:
            raise CsvdError(CSVD_EDEVICE, f"{lib_path} is not built")
        from .build import build
        build(verbose=False)
    lib = C.CDLL(lib_path)
    sig = {
        "csvd_params_default": (C.c_int, [C.POINTER(csvd_params)]),
        "csvd_create": (C.c_int, [C.POINTER(_P), C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, C.c_int32, _P]),
        "csvd_solve_interval": (C.c_int, [_P, C.c_double, C.c_double, C.POINTER(csvd_params), _P]),
        "csvd_get_triplets": (C.c_int, [_P, C.POINTER(C.c_int64), C.c_int64, _P, _P, _P, _P]),
        "csvd_get_info": (C.c_int, [_P, C.POINTER(csvd_info)]),
        "csvd_get_residual_estimates": (C.c_int, [_P, C.c_int64, _P]),
        "csvd_get_moment": (C.c_int, [_P, C.c_int32, _P]),
        "csvd_get_solution": (C.c_int, [_P, C.c_int32, _P, _P]),
        "csvd_quadrature": (C.c_int, [C.c_double, C.c_double, C.POINTER(csvd_params), _P, _P, _P, _P, _P, _P]),
        "csvd_spmm": (C.c_int, [_P, C.c_int32, C.c_int64, _P, _P]),
        "csvd_spmm_noalloc": (C.c_int, [_P, C.c_int32, C.c_int64, _P, _P]),
        "csvd_probe_gather": (C.c_int, [C.c_int64, C.c_int32, C.c_int64, C.c_int32, C.c_uint64, C.c_int32,
                                        C.POINTER(C.c_double)]),
        "csvd_get_transpose": (C.c_int, [_P, _P, _P, _P]),
        "csvd_dense_gemm": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P, _P, _P]),
        "csvd_last_error": (C.c_char_p, [_P]),
        "csvd_destroy": (None, [_P]),
        "csvd_trim": (C.c_int, [_P]),
        "csvd_solve_batch": (C.c_int, [C.c_int32, _P, _P, _P, C.POINTER(csvd_params), _P, _P]),
        "csvd_server_create": (C.c_int, [C.POINTER(_P), C.c_int64, C.c_int32, _P]),
        "csvd_server_submit": (C.c_int, [_P, _P, C.c_double, C.c_double, C.POINTER(csvd_params), _P,
                                         C.POINTER(C.c_int64)]),
        "csvd_server_step": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32)]),
        "csvd_server_poll": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "csvd_server_cancel": (C.c_int, [_P, C.c_int64]),
        "csvd_server_last_error": (C.c_char_p, [_P]),
        "csvd_server_destroy": (None, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.asfortranarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _check(rc, ctx=None, allow=(CSVD_OK,)):
    if rc in allow:
        return rc
    msg = ""
    if ctx is not None:
        m = load().csvd_last_error(ctx)
        msg = m.decode() if m else ""
    raise CsvdError(rc, msg)


def csvd_params_default(**overrides) -> csvd_params:
    p = csvd_params()
    _check(load().csvd_params_default(C.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def csvd_create(m, n, rowptr, colidx, vals, hip_stream=None):
    """Returns an opaque context handle for host CSR arrays (NumPy)."""
    lib = load()
    h = C.c_void_p()
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colidx, dtype=np.int32)
    va = np.ascontiguousarray(vals, dtype=np.float64)
    if rp.ndim != 1 or rp.size != int(m) + 1:
        raise ValueError(f"rowptr must hold m + 1 = {int(m) + 1} entries, got {rp.size}")
    if ci.shape != va.shape or ci.ndim != 1:
        raise ValueError(f"colidx and vals must be 1-D of equal length, got {ci.shape} and {va.shape}")
    rc = lib.csvd_create(C.byref(h), int(m), int(n), int(va.size), _ptr(rp), _ptr(ci), _ptr(va), 0,
                         C.c_void_p(hip_stream) if hip_stream else None)
    _check(rc)
    _shape[h.value] = (int(m), int(n))
    return h


def csvd_create_device(m, n, nnz, rowptr_addr, colidx_addr, vals_addr, hip_stream=None):
    """Same as csvd_create with device-resident CSR arrays (integer addresses)."""
    h = C.c_void_p()
    rc = load().csvd_create(C.byref(h), int(m), int(n), int(nnz), C.c_void_p(rowptr_addr),
                            C.c_void_p(colidx_addr), C.c_void_p(vals_addr), 1,
                            C.c_void_p(hip_stream) if hip_stream else None)
    _check(rc)
    _shape[h.value] = (int(m), int(n))
    return h


def _check_vin(ctx, V_in, L):
    """V_in as a column-major float64 n x L array (n of the context)."""
    V_in = _f64(V_in)
    key = ctx.value if isinstance(ctx, C.c_void_p) else ctx
    n = _shape.get(key, (None, None))[1]
    if V_in.ndim != 2 or V_in.shape[1] != int(L) or (n is not None and V_in.shape[0] != n):
        raise ValueError(f"V_in must be n x L = {n} x {int(L)}, got {V_in.shape}")
    return V_in


def csvd_solve_interval(ctx, a, b, params, V_in=None):
    """Returns the status (CSVD_OK or CSVD_ENOTCONV); raises on errors."""
    Vp = None
    if V_in is not None:
        V_in = _check_vin(ctx, V_in, params.L)
        Vp = _ptr(V_in)
    rc = load().csvd_solve_interval(ctx, float(a), float(b), C.byref(params), Vp)
    return _check(rc, ctx, allow=(CSVD_OK, CSVD_ENOTCONV))


def csvd_get_triplets(ctx, m, n, want_vectors=True):
    """Returns (sigma, U, V, resid) of the last solve (ascending sigma)."""
    lib = load()
    t = C.c_int64()
    _check(lib.csvd_get_triplets(ctx, C.byref(t), 0, None, None, None, None), ctx)
    k = t.value
    sigma = np.zeros(k)
    resid = np.zeros(k)
    U = np.zeros((m, k), order="F") if want_vectors else None
    V = np.zeros((n, k), order="F") if want_vectors else None
    if k:
        _check(lib.csvd_get_triplets(ctx, C.byref(t), k, _ptr(sigma), _ptr(U), _ptr(V), _ptr(resid)), ctx)
    return sigma, U, V, resid


def csvd_get_residual_estimates(ctx, t_hat):
    """Residual estimates of Sec. 3.4.1 per triplet (relative to ||A||_2)."""
    est = np.zeros(int(t_hat))
    _check(load().csvd_get_residual_estimates(ctx, int(t_hat), _ptr(est) if t_hat else None), ctx)
    return est


def csvd_get_info(ctx) -> csvd_info:
    info = csvd_info()
    _check(load().csvd_get_info(ctx, C.byref(info)), ctx)
    return info


def csvd_get_moment(ctx, k, n, L):
    out = np.zeros((n, L), order="F")
    _check(load().csvd_get_moment(ctx, int(k), _ptr(out)), ctx)
    return out


def csvd_get_solution(ctx, j, n, L):
    re = np.zeros((n, L), order="F")
    im = np.zeros((n, L), order="F")
    _check(load().csvd_get_solution(ctx, int(j), _ptr(re), _ptr(im)), ctx)
    return re + 1j * im


def csvd_quadrature(a, b, params):
    """(shifts, weights, c) of the upper-half rule; c has shape (N/2, M+1)."""
    S, K = params.N // 2, params.M + 1
    sr, si, wr, wi = (np.zeros(S) for _ in range(4))
    cr, ci = np.zeros(S * K), np.zeros(S * K)
    _check(load().csvd_quadrature(float(a), float(b), C.byref(params), _ptr(sr), _ptr(si), _ptr(wr), _ptr(wi),
                                  _ptr(cr), _ptr(ci)))
    return sr + 1j * si, wr + 1j * wi, (cr + 1j * ci).reshape(S, K)


def csvd_spmm(ctx, transpose, X, rows_out):
    X = _f64(X)
    k = X.shape[1]
    Y = np.zeros((rows_out, k), order="F")
    _check(load().csvd_spmm(ctx, int(transpose), int(k), _ptr(X), _ptr(Y)), ctx)
    return Y


def csvd_spmm_noalloc(ctx, transpose, X, rows_out):
    X = _f64(X)
    k = X.shape[1]
    Y = np.zeros((rows_out, k), order="F")
    _check(load().csvd_spmm_noalloc(ctx, int(transpose), int(k), _ptr(X), _ptr(Y)), ctx)
    return Y


def csvd_probe_gather(table_rows, variant, out_rows, per_out, seed=1, reps=20):
    """Average ms of one random 512-byte-row gather launch (include/csvd_diag.h)."""
    ms = C.c_double()
    _check(load().csvd_probe_gather(int(table_rows), int(variant), int(out_rows), int(per_out), int(seed),
                                    int(reps), C.byref(ms)))
    return ms.value


def csvd_get_transpose(ctx, n, nnz):
    rp = np.zeros(n + 1, dtype=np.int32)
    ci = np.zeros(nnz, dtype=np.int32)
    va = np.zeros(nnz)
    _check(load().csvd_get_transpose(ctx, _ptr(rp), _ptr(ci), _ptr(va)), ctx)
    return rp, ci, va


def csvd_dense_gemm(A, B):
    A = _f64(A)
    B = _f64(B)
    R, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    Cm = np.zeros((R, N), order="F")
    _check(load().csvd_dense_gemm(R, N, K, _ptr(A), _ptr(B), _ptr(Cm)))
    return Cm


def csvd_last_error(ctx) -> str:
    m = load().csvd_last_error(ctx)
    return m.decode() if m else ""


def csvd_trim(ctx):
    _check(load().csvd_trim(ctx), ctx)


def csvd_destroy(ctx):
    if ctx:
        _shape.pop(ctx.value if isinstance(ctx, C.c_void_p) else ctx, None)
        load().csvd_destroy(ctx)


def csvd_solve_batch(ctxs, a, b, params, V_in=None):
    """Batched solve; returns the per-problem status list."""
    n = len(ctxs)
    arr_ctx = (C.c_void_p * n)(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    aa = np.ascontiguousarray(a, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    ps = (csvd_params * n)(*params)
    keep = []
    vptr = None
    if V_in is not None:
        arr = (C.c_void_p * n)()
        for i, v in enumerate(V_in):
            if v is None:
                arr[i] = None
            else:
                vv = _check_vin(ctxs[i], v, params[i].L)
                keep.append(vv)
                arr[i] = vv.ctypes.data
        vptr = C.cast(arr, C.c_void_p)
    st = np.zeros(n, dtype=np.int32)
    _check(load().csvd_solve_batch(n, C.cast(arr_ctx, C.c_void_p), _ptr(aa), _ptr(bb), ps, vptr, _ptr(st)))
    return [int(x) for x in st]


def csvd_server_create(budget_bytes, max_batch, hip_stream=None):
    h = C.c_void_p()
    _check(load().csvd_server_create(C.byref(h), int(budget_bytes), int(max_batch),
                                     C.c_void_p(hip_stream) if hip_stream else None))
    return h


def _srv_check(rc, srv, allow=(CSVD_OK,)):
    if rc in allow:
        return rc
    m = load().csvd_server_last_error(srv)
    raise CsvdError(rc, m.decode() if m else "")


def csvd_server_submit(srv, ctx, a, b, params, V_in=None):
    req = C.c_int64()
    Vp = None
    if V_in is not None:
        V_in = _check_vin(ctx, V_in, params.L)
        Vp = _ptr(V_in)
    _srv_check(load().csvd_server_submit(srv, ctx, float(a), float(b), C.byref(params), Vp, C.byref(req)), srv)
    return req.value


def csvd_server_step(srv, steps):
    na = C.c_int32()
    _srv_check(load().csvd_server_step(srv, int(steps), C.byref(na)), srv)
    return na.value


def csvd_server_poll(srv, req):
    d, s = C.c_int32(), C.c_int32()
    _srv_check(load().csvd_server_poll(srv, int(req), C.byref(d), C.byref(s)), srv)
    return bool(d.value), s.value


def csvd_server_cancel(srv, req):
    _srv_check(load().csvd_server_cancel(srv, int(req)), srv)


def csvd_server_last_error(srv) -> str:
    m = load().csvd_server_last_error(srv)
    return m.decode() if m else ""


def csvd_server_destroy(srv):
    if srv:
        load().csvd_server_destroy(srv)
