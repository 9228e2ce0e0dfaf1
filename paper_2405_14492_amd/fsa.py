"""Thin ctypes binding of libfsa.so (the C ABI declared in include/fsa.h).

Only argument marshalling lives here: every numerical step runs in the HIP
kernels of the library.  The library must have been built
(`python -m paper_2405_14492_amd.build`); importing this module without it
raises ImportError -- there is no CPU fallback.

Covariance parameters are passed as a tuple (cov, sigma1_sq, rho, sigma_sq)
with cov = EXPONENTIAL (0) or MATERN32 (1).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

EXPONENTIAL = 0
MATERN32 = 1
FP64 = 0
MIXED_FP32 = 1
MIXED_BF16A = 2
PROFILE_ALL = 0x1f  # fsa_options.profile: all five kernel classes
CV_NONE, CV_ONE, CV_OPT, CV_OPT_PRINTED = range(4)  # fsa_options.control_variate
F32P_SPLIT, F32P_MFMA = range(2)  # fsa_options.fp32_products

OP_SIGMA_DAGGER, OP_SIGMA_S, OP_P_INV, OP_D_SIGMA1, OP_D_RHO, OP_PROBES = range(6)
V_SIGMA, V_PRECISION, V_OPERATOR, V_P_INV = range(4)

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "NOT_SPD", 4: "NOT_CONVERGED", 5: "BREAKDOWN", 6: "DEVICE"}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfsa.so")

EXPORTED = ["fsa_default_options", "fsa_build", "fsa_build_dev", "fsa_nll_grad", "fsa_grad", "fsa_predict_var",
            "fsa_destroy",
            "fsa_last_error", "fsa_nnz", "fsa_export_csr", "fsa_export_diag", "fsa_export_lanczos", "fsa_export_solution",
            "fsa_apply",
            "fsa_pool_trim", "fsa_scores", "fsa_scores_noalloc", "fsa_set_allocator", "fsa_nll_grad_dev",
            "fsa_vecchia_build_dev", "fsa_vecchia_factor_dev", "fsa_vecchia_apply_dev", "fsa_vecchia_solve_logdet_dev",
            "fsa_vecchia_destroy", "fsa_vecchia_laplace_dev",
            "fsa_request_footprint", "fsa_server_create", "fsa_server_clock_ms", "fsa_server_submit",
            "fsa_server_wait", "fsa_server_get_stats", "fsa_server_destroy"]


class FsaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class NotConverged(FsaError):
    pass


class fsa_theta(C.Structure):
    _fields_ = [("cov", C.c_int32), ("sigma1_sq", C.c_double), ("rho", C.c_double), ("sigma_sq", C.c_double)]


class fsa_options(C.Structure):
    _fields_ = [("num_probes", C.c_int32), ("control_variate", C.c_int32), ("seed", C.c_uint64),
                ("cg_rel_tol", C.c_double),
                ("max_iter", C.c_int32), ("fixed_iter", C.c_int32), ("precision", C.c_int32),
                ("rr_period", C.c_int32), ("slq_weight_n", C.c_int32), ("profile", C.c_int32),
                ("sigma_m_jitter", C.c_double),
                ("hip_stream", C.c_void_p), ("graph", C.c_int32), ("fp32_products", C.c_int32)]


class fsa_stats(C.Structure):
    _fields_ = [("iters_min", C.c_int32), ("iters_max", C.c_int32), ("probe_iters", C.c_int64),
                ("rel_res_max", C.c_double), ("logdet", C.c_double), ("logdet_P", C.c_double),
                ("quad", C.c_double), ("ms_build", C.c_double), ("ms_pcg", C.c_double),
                ("ms_backward", C.c_double), ("ms_total", C.c_double), ("nnz", C.c_int64),
                ("kernel_ms", C.c_double * 5), ("kernel_launches", C.c_int32 * 5),
                ("grad_trace", C.c_double * 3), ("grad_quad", C.c_double * 3),
                ("cv_c", C.c_double * 3), ("trace_P", C.c_double * 3), ("fp64_fallback", C.c_int32),
                ("reserved1", C.c_int32), ("fallback_probe_iters", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        for k in ("kernel_ms", "kernel_launches", "grad_trace", "grad_quad", "cv_c", "trace_P"):
            d[k] = list(getattr(self, k))
        return d


class fsa_vecchia_stats(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("iters_max", C.c_int32), ("iters_rhs", C.c_int32), ("converged", C.c_int32),
                ("probe_iters", C.c_int64), ("logdet_P", C.c_double), ("logdet_offset", C.c_double), ("logdet_sw", C.c_double),
                ("ms_solve", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fsa_vecchia_laplace_stats(C.Structure):
    _fields_ = [("newton_steps", C.c_int32), ("converged", C.c_int32), ("cg_iters_max", C.c_int32),
                ("reserved0", C.c_int32), ("probe_iters", C.c_int64), ("loglik", C.c_double), ("quad", C.c_double),
                ("sum_log_d", C.c_double), ("logdet", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# fsa_set_allocator callbacks: alloc(bytes, hip_stream, user) -> device pointer, release(ptr, user)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2405_14492_amd.build`")
    lib = C.CDLL(path)
    P = C.POINTER
    dp = P(C.c_double)
    vp = C.c_void_p
    lib.fsa_default_options.argtypes = [P(fsa_options)]
    lib.fsa_default_options.restype = None
    for name in ("fsa_build", "fsa_build_dev"):
        f = getattr(lib, name)
        f.argtypes = [vp, C.c_int64, C.c_int32, vp, P(fsa_theta), vp, C.c_int32, C.c_double, P(fsa_options),
                      P(vp)]
        f.restype = C.c_int
    lib.fsa_nll_grad.argtypes = [vp, P(fsa_theta), dp, dp, P(fsa_stats)]
    lib.fsa_nll_grad.restype = C.c_int
    lib.fsa_nll_grad_dev.argtypes = [vp, P(fsa_theta), vp, vp, P(fsa_stats)]
    lib.fsa_nll_grad_dev.restype = C.c_int
    lib.fsa_set_allocator.argtypes = [ALLOC_FN, RELEASE_FN, vp]
    lib.fsa_set_allocator.restype = C.c_int
    lib.fsa_grad.argtypes = [vp, dp, P(fsa_stats)]
    lib.fsa_grad.restype = C.c_int
    lib.fsa_predict_var.argtypes = [vp, dp, C.c_int64, C.c_int32, dp, dp, P(fsa_stats)]
    lib.fsa_predict_var.restype = C.c_int
    lib.fsa_destroy.argtypes = [vp]
    lib.fsa_destroy.restype = None
    lib.fsa_last_error.argtypes = []
    lib.fsa_last_error.restype = C.c_char_p
    lib.fsa_nnz.argtypes = [vp]
    lib.fsa_nnz.restype = C.c_int64
    lib.fsa_export_csr.argtypes = [vp, P(C.c_int64), P(C.c_int32), dp]
    lib.fsa_export_csr.restype = C.c_int
    lib.fsa_export_diag.argtypes = [vp, dp, dp]
    lib.fsa_export_diag.restype = C.c_int
    lib.fsa_export_lanczos.argtypes = [vp, P(C.c_int32), dp, dp, dp, dp]
    lib.fsa_export_lanczos.restype = C.c_int
    lib.fsa_export_solution.argtypes = [vp, dp]
    lib.fsa_export_solution.restype = C.c_int
    lib.fsa_apply.argtypes = [vp, C.c_int32, dp, dp, C.c_int32]
    lib.fsa_apply.restype = C.c_int
    lib.fsa_pool_trim.argtypes = []
    lib.fsa_pool_trim.restype = None
    lib.fsa_scores.argtypes = [dp, dp, dp, C.c_int64, dp]
    lib.fsa_scores.restype = C.c_int
    lib.fsa_scores_noalloc.argtypes = [dp, dp, dp, C.c_int64, dp]
    lib.fsa_scores_noalloc.restype = C.c_int
    lib.fsa_vecchia_build_dev.argtypes = [vp, C.c_int64, vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                          vp, vp, P(vp)]
    lib.fsa_vecchia_build_dev.restype = C.c_int
    lib.fsa_vecchia_factor_dev.argtypes = [vp, vp, vp, vp]
    lib.fsa_vecchia_factor_dev.restype = C.c_int
    lib.fsa_vecchia_apply_dev.argtypes = [vp, C.c_int32, vp, C.c_int64, C.c_int32, vp, C.c_int64]
    lib.fsa_vecchia_apply_dev.restype = C.c_int
    lib.fsa_vecchia_solve_logdet_dev.argtypes = [vp, vp, vp, C.c_int32, C.c_uint64, C.c_double, C.c_int32,
                                                 C.c_int32, dp, P(fsa_vecchia_stats)]
    lib.fsa_vecchia_solve_logdet_dev.restype = C.c_int
    lib.fsa_vecchia_destroy.argtypes = [vp]
    lib.fsa_vecchia_destroy.restype = C.c_int
    lib.fsa_vecchia_laplace_dev.argtypes = [vp, vp, C.c_int32, C.c_uint64, C.c_double, C.c_int32, C.c_int32,
                                            C.c_double, C.c_int32, C.c_int32, vp, dp, P(fsa_vecchia_laplace_stats)]
    lib.fsa_vecchia_laplace_dev.restype = C.c_int
    lib.fsa_request_footprint.argtypes = [P(fsa_request), P(fsa_options), P(C.c_uint64)]
    lib.fsa_request_footprint.restype = C.c_int
    lib.fsa_server_create.argtypes = [P(fsa_server_options), P(vp)]
    lib.fsa_server_create.restype = C.c_int
    lib.fsa_server_clock_ms.argtypes = [vp]
    lib.fsa_server_clock_ms.restype = C.c_double
    lib.fsa_server_submit.argtypes = [vp, P(fsa_request), P(C.c_int64)]
    lib.fsa_server_submit.restype = C.c_int
    lib.fsa_server_wait.argtypes = [vp, C.c_int64, P(fsa_result), dp]
    lib.fsa_server_wait.restype = C.c_int
    lib.fsa_server_get_stats.argtypes = [vp, P(fsa_server_stats)]
    lib.fsa_server_get_stats.restype = C.c_int
    lib.fsa_server_destroy.argtypes = [vp]
    lib.fsa_server_destroy.restype = None
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check(status: int, allow_not_converged: bool = False):
    if status == 0:
        return
    msg = lib().fsa_last_error().decode()
    if status == 4:
        if allow_not_converged:
            return
        raise NotConverged(status, msg)
    raise FsaError(status, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def make_theta(theta) -> fsa_theta:
    cov, s1, rho, s2 = theta
    return fsa_theta(int(cov), float(s1), float(rho), float(s2))


def make_options(num_probes=50, seed=0, tol=1e-8, max_iter=1000, fixed_iter=0, precision=FP64, rr_period=10,
                 slq_weight_n=False, jitter=0.0, stream=None, profile=False, control_variate=CV_NONE,
                 graph=False, fp32_products=F32P_SPLIT) -> fsa_options:
    o = fsa_options()
    lib().fsa_default_options(C.byref(o))
    o.num_probes = int(num_probes)
    o.seed = int(seed)
    o.cg_rel_tol = float(tol)
    o.max_iter = int(max_iter)
    o.fixed_iter = int(fixed_iter)
    o.precision = int(precision)
    o.rr_period = int(rr_period)
    o.slq_weight_n = int(bool(slq_weight_n))
    o.sigma_m_jitter = float(jitter)
    o.hip_stream = stream
    # True: every kernel class; an int: the class bit mask itself
    o.profile = PROFILE_ALL if profile is True else int(profile)
    o.control_variate = int(control_variate)
    o.graph = int(bool(graph))
    o.fp32_products = int(fp32_products)
    return o


# ---------------------------------------------------------------- C names
def fsa_build(locs, y, theta, inducing, taper_range, opt: fsa_options | None = None) -> C.c_void_p:
    """Host arrays in; returns the context handle."""
    locs, y, ind = _f64(locs), _f64(y), _f64(inducing)
    ctx = C.c_void_p()
    th = make_theta(theta)
    _check(lib().fsa_build(locs.ctypes.data, locs.shape[0], locs.shape[1], y.ctypes.data, C.byref(th),
                           ind.ctypes.data, ind.shape[0], float(taper_range), C.byref(opt) if opt else None,
                           C.byref(ctx)))
    return ctx


def fsa_build_dev(locs, y, theta, inducing, taper_range, opt: fsa_options | None = None) -> C.c_void_p:
    """Device tensors (torch, float64, contiguous, on the GPU) in."""
    ctx = C.c_void_p()
    th = make_theta(theta)
    _check(lib().fsa_build_dev(locs.data_ptr(), locs.shape[0], locs.shape[1], y.data_ptr(), C.byref(th),
                               inducing.data_ptr(), inducing.shape[0], float(taper_range),
                               C.byref(opt) if opt else None, C.byref(ctx)))
    return ctx


def fsa_nll_grad(ctx, theta=None, with_grad=True, allow_not_converged=False):
    nll = C.c_double()
    g = np.zeros(3)
    st = fsa_stats()
    th = make_theta(theta) if theta is not None else None
    s = lib().fsa_nll_grad(ctx, C.byref(th) if th is not None else None, C.byref(nll),
                           _dptr(g) if with_grad else None, C.byref(st))
    _check(s, allow_not_converged)
    return nll.value, (g if with_grad else None), st.as_dict()


def fsa_nll_grad_dev(ctx, nll_out, grad_out=None, theta=None, allow_not_converged=False):
    """Device outputs: nll_out (1 float64 element) and grad_out (3, or None)
    are torch CUDA tensors written by the library on the context's stream."""
    st = fsa_stats()
    th = make_theta(theta) if theta is not None else None
    s = lib().fsa_nll_grad_dev(ctx, C.byref(th) if th is not None else None, nll_out.data_ptr(),
                               grad_out.data_ptr() if grad_out is not None else None, C.byref(st))
    _check(s, allow_not_converged)
    return st.as_dict()


_ALLOCATOR = None  # the registered callbacks (kept alive while registered)


def fsa_set_allocator(allocator=None):
    """Register an object with alloc(nbytes, stream) -> int and
    release(ptr) (e.g. TorchAllocator) as the library's source of device
    memory, or None for the library's own pool.  The previous object is
    kept referenced by its blocks' release path until they are returned."""
    global _ALLOCATOR
    if allocator is None:
        _check(lib().fsa_set_allocator(ALLOC_FN(), RELEASE_FN(), None))
        _ALLOCATOR = None
        return

    def _alloc(nbytes, stream, user):
        try:
            return allocator.alloc(int(nbytes), int(stream or 0)) or None
        except Exception:  # an allocation failure is the library's OOM
            return None

    def _release(ptr, user):
        allocator.release(int(ptr))

    cbs = (ALLOC_FN(_alloc), RELEASE_FN(_release), allocator)
    _check(lib().fsa_set_allocator(cbs[0], cbs[1], None))
    allocator._fsa_callbacks = cbs  # must outlive every block handed out
    _ALLOCATOR = cbs


class TorchAllocator:
    """Device memory for the library from torch's caching allocator, on the
    stream the library names; counts what it hands out and gets back."""

    def __init__(self):
        import torch
        self._torch = torch
        self.live = {}
        self.allocs = 0
        self.releases = 0

    def alloc(self, nbytes, stream):
        torch = self._torch
        p = torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device(), stream)
        self.live[p] = nbytes
        self.allocs += 1
        return p

    def release(self, ptr):
        self.live.pop(ptr)
        self.releases += 1
        self._torch.cuda.caching_allocator_delete(ptr)


def fsa_grad(ctx):
    g = np.zeros(3)
    st = fsa_stats()
    _check(lib().fsa_grad(ctx, _dptr(g), C.byref(st)))
    return g, st.as_dict()


def fsa_predict_var(ctx, pred_locs, num_samples, with_mean=False, allow_not_converged=False):
    P = _f64(pred_locs)
    var = np.zeros(P.shape[0])
    mean = np.zeros(P.shape[0]) if with_mean else None
    st = fsa_stats()
    s = lib().fsa_predict_var(ctx, _dptr(P), P.shape[0], int(num_samples), _dptr(var),
                              _dptr(mean) if with_mean else None, C.byref(st))
    _check(s, allow_not_converged)
    return var, mean, st.as_dict()


def fsa_destroy(ctx):
    if ctx:
        lib().fsa_destroy(ctx)


def fsa_nnz(ctx) -> int:
    return int(lib().fsa_nnz(ctx))


def fsa_export_csr(ctx, n, with_values=False):
    nnz = fsa_nnz(ctx)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int32)
    vals = np.zeros(nnz) if with_values else None
    _check(lib().fsa_export_csr(ctx, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                col.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(vals) if with_values else None))
    return rp, col, vals


def fsa_export_diag(ctx, n):
    D = np.zeros(n)
    ld = C.c_double()
    _check(lib().fsa_export_diag(ctx, _dptr(D), C.byref(ld)))
    return D, ld.value


def fsa_export_lanczos(ctx, ncols, max_iter):
    """Lanczos record of the last likelihood solve: per column iterations,
    alpha and beta (max_iter x ncols, by iteration), quadrature weights and
    the weighted terms e_1^T log(T) e_1 (column 0: 0)."""
    it = np.zeros(ncols, dtype=np.int32)
    a = np.zeros((max_iter, ncols))
    b = np.zeros((max_iter, ncols))
    w = np.zeros(ncols)
    q = np.zeros(ncols)
    _check(lib().fsa_export_lanczos(ctx, it.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(a), _dptr(b), _dptr(w),
                                    _dptr(q)))
    return {"iters": it, "alpha": a, "beta": b, "weight": w, "slq": q}


def fsa_export_solution(ctx, n, ncols):
    """Solution block Sigma~^{-1} [y, z_1 .. z_t] of the last likelihood solve
    (n x ncols, caller's point order)."""
    U = np.zeros((n, ncols))
    _check(lib().fsa_export_solution(ctx, _dptr(U)))
    return U


def fsa_scores(y, mean, var):
    """(log-score, CRPS, RMSE) of Gaussian predictive distributions against
    test responses y (Section 4), computed on the device."""
    y, mean, var = _f64(y).ravel(), _f64(mean).ravel(), _f64(var).ravel()
    if not (y.shape == mean.shape == var.shape):
        raise ValueError("y, mean and var must have the same length")
    out = np.zeros(3)
    _check(lib().fsa_scores(_dptr(y), _dptr(mean), _dptr(var), y.shape[0], _dptr(out)))
    return float(out[0]), float(out[1]), float(out[2])


SCORES_NOALLOC_MAX_N = 1 << 18  # the fixed device scratch of fsa_scores_noalloc


def fsa_scores_noalloc(y, mean, var):
    """fsa_scores through the entry point that allocates no device memory
    (fixed library scratch; n <= SCORES_NOALLOC_MAX_N)."""
    y, mean, var = _f64(y).ravel(), _f64(mean).ravel(), _f64(var).ravel()
    if not (y.shape == mean.shape == var.shape):
        raise ValueError("y, mean and var must have the same length")
    out = np.zeros(3)
    _check(lib().fsa_scores_noalloc(_dptr(y), _dptr(mean), _dptr(var), y.shape[0], _dptr(out)))
    return float(out[0]), float(out[1]), float(out[2])


def fsa_apply(ctx, which, X, ncols=None):
    if which == OP_PROBES:
        n = int(X)
        Y = np.zeros((n, ncols))
        _check(lib().fsa_apply(ctx, which, None, _dptr(Y), ncols))
        return Y
    X = _f64(X)
    if X.ndim == 1:
        X = X[:, None]
    Y = np.zeros_like(X)
    _check(lib().fsa_apply(ctx, which, _dptr(X), _dptr(Y), X.shape[1]))
    return Y


def fsa_pool_trim():
    lib().fsa_pool_trim()


# ---------------------------------------------------------------- convenience
class FSA:
    """Owns one context.  Host numpy inputs (or torch GPU tensors with device=True)."""

    def __init__(self, locs, y, theta, inducing, taper_range, num_probes=50, seed=0, tol=1e-8, max_iter=1000,
                 fixed_iter=0, precision=FP64, rr_period=10, slq_weight_n=False, jitter=0.0, stream=None,
                 device=False, profile=False, control_variate=CV_NONE, graph=False, fp32_products=F32P_SPLIT):
        self.opt = make_options(num_probes, seed, tol, max_iter, fixed_iter, precision, rr_period, slq_weight_n,
                                jitter, stream, profile, control_variate, graph, fp32_products)
        self.n = int(locs.shape[0])
        self.theta = tuple(theta)
        build = fsa_build_dev if device else fsa_build
        self.ctx = build(locs, y, theta, inducing, taper_range, self.opt)

    def nll_grad(self, theta=None, with_grad=True, allow_not_converged=False):
        out = fsa_nll_grad(self.ctx, theta, with_grad, allow_not_converged)
        if theta is not None:
            self.theta = tuple(theta)
        return out

    def nll_grad_dev(self, nll_out, grad_out=None, theta=None, allow_not_converged=False):
        st = fsa_nll_grad_dev(self.ctx, nll_out, grad_out, theta, allow_not_converged)
        if theta is not None:
            self.theta = tuple(theta)
        return st

    def grad(self):
        return fsa_grad(self.ctx)

    def predict_var(self, pred_locs, num_samples, with_mean=False, allow_not_converged=False):
        return fsa_predict_var(self.ctx, pred_locs, num_samples, with_mean, allow_not_converged)

    def export_csr(self, with_values=False):
        return fsa_export_csr(self.ctx, self.n, with_values)

    def export_diag(self):
        return fsa_export_diag(self.ctx, self.n)

    def export_lanczos(self):
        L = self.opt.fixed_iter if self.opt.fixed_iter > 0 else self.opt.max_iter
        return fsa_export_lanczos(self.ctx, self.opt.num_probes + 1, L)

    def export_solution(self):
        return fsa_export_solution(self.ctx, self.n, self.opt.num_probes + 1)

    def apply(self, which, X, ncols=None):
        return fsa_apply(self.ctx, which, X if which != OP_PROBES else self.n, ncols)

    @property
    def nnz(self):
        return fsa_nnz(self.ctx)

    def close(self):
        if self.ctx:
            fsa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Vecchia:
    """The FITC preconditioner for a Vecchia approximation (Section 5) on
    device tensors: build with locations (n x 2), inducing points (m x 2) and
    weights W (n), all float64 CUDA tensors; then factor(), apply() and
    solve_logdet().  Argument marshalling only: every step runs in libfsa."""

    def __init__(self, locs, inducing, kind, sigma1_sq, rho, mv, w, stream=None):
        import torch
        self._torch = torch
        self.locs = locs.contiguous()
        self.n = self.locs.shape[0]
        self.mv = int(mv)
        ind = inducing.contiguous()
        wc = w.contiguous()
        for t in (self.locs, ind, wc):
            if t.dtype != torch.float64 or not t.is_cuda:
                raise TypeError("Vecchia takes float64 device tensors")
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        st = self._stream.cuda_stream
        self._stream.wait_stream(torch.cuda.current_stream())  # inputs written on the caller's stream
        h = C.c_void_p()
        _check(lib().fsa_vecchia_build_dev(self.locs.data_ptr(), self.n, ind.data_ptr(), ind.shape[0], int(kind),
                                           float(sigma1_sq), float(rho), self.mv, wc.data_ptr(), C.c_void_p(st),
                                           C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().fsa_vecchia_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factor(self):
        torch = self._torch
        mv = max(self.mv, 1)
        nbr = torch.empty((self.n, mv), dtype=torch.int32, device=self.locs.device)
        coef = torch.empty((self.n, mv), dtype=torch.float64, device=self.locs.device)
        d = torch.empty(self.n, dtype=torch.float64, device=self.locs.device)
        _check(lib().fsa_vecchia_factor_dev(self._h, nbr.data_ptr(), coef.data_ptr(), d.data_ptr()))
        return nbr[:, :self.mv], coef[:, :self.mv], d

    def _order_after_caller(self):
        # the library runs on the handle's stream; inputs (and the copies
        # .contiguous() makes) come from torch's current stream
        cur = self._torch.cuda.current_stream()
        if cur != self._stream:
            self._stream.wait_stream(cur)

    def apply(self, which, X):
        X2 = X.contiguous() if X.dim() == 2 else X.reshape(-1, 1).contiguous()
        Y = self._torch.empty_like(X2)
        k = X2.shape[1]
        self._order_after_caller()
        _check(lib().fsa_vecchia_apply_dev(self._h, int(which), X2.data_ptr(), k, k, Y.data_ptr(), k))
        return Y if X.dim() == 2 else Y[:, 0]

    def solve_logdet(self, rhs, num_probes, seed, tol=1e-8, max_iter=1000, fixed_iter=0, allow_not_converged=False):
        r = rhs.contiguous()
        x = self._torch.empty_like(r)
        ld = C.c_double()
        st = fsa_vecchia_stats()
        self._order_after_caller()
        _check(lib().fsa_vecchia_solve_logdet_dev(self._h, r.data_ptr(), x.data_ptr(), int(num_probes), int(seed),
                                                  float(tol), int(max_iter), int(fixed_iter), C.byref(ld),
                                                  C.byref(st)),
               allow_not_converged)
        return x, ld.value, st.as_dict()

    def laplace(self, y, num_probes, seed, tol=1e-8, max_iter=1000, fixed_iter=0, newton_tol=1e-8, max_newton=50,
                fixed_newton=0, allow_not_converged=False):
        """Vecchia-Laplace NLL of Bernoulli responses y (float64 0/1 device
        tensor): (mode, nll, stats).  The handle's weights become those at
        the mode."""
        yy = y.contiguous()
        mode = self._torch.empty_like(yy)
        nll = C.c_double()
        st = fsa_vecchia_laplace_stats()
        self._order_after_caller()
        _check(lib().fsa_vecchia_laplace_dev(self._h, yy.data_ptr(), int(num_probes), int(seed), float(tol),
                                             int(max_iter), int(fixed_iter), float(newton_tol), int(max_newton),
                                             int(fixed_newton), mode.data_ptr(), C.byref(nll), C.byref(st)),
               allow_not_converged)
        return mode, nll.value, st.as_dict()


# ---------------------------------------------------------------- serving
REQ_NLL_GRAD, REQ_PREDICT_VAR = 0, 1


class fsa_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int32), ("n", C.c_int64), ("locs", C.c_void_p), ("y", C.c_void_p),
                ("inducing", C.c_void_p), ("theta", fsa_theta), ("taper_range", C.c_double), ("n_p", C.c_int64),
                ("pred_locs", C.c_void_p), ("num_samples", C.c_int32), ("reserved0", C.c_int32),
                ("arrival_ms", C.c_double)]


class fsa_server_options(C.Structure):
    _fields_ = [("slots", C.c_int32), ("reserved0", C.c_int32), ("hbm_budget", C.c_uint64), ("opt", fsa_options)]


class fsa_result(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int32), ("kind", C.c_int32), ("nll", C.c_double),
                ("grad", C.c_double * 3), ("arrival_ms", C.c_double), ("admit_ms", C.c_double),
                ("done_ms", C.c_double), ("footprint", C.c_uint64), ("peak_bytes", C.c_uint64),
                ("worker", C.c_int32), ("iters_max", C.c_int32), ("probe_iters", C.c_int64), ("n_p", C.c_int64),
                ("message", C.c_char * 192)]


class fsa_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("hbm_budget", C.c_uint64), ("peak_reserved", C.c_uint64), ("slots", C.c_int32),
                ("peak_active", C.c_int32), ("first_arrival_ms", C.c_double), ("last_done_ms", C.c_double)]


def _request(kind, locs, y, theta, inducing, taper_range, pred_locs=None, num_samples=0, arrival_ms=0.0):
    locs, y, inducing = _f64(locs), _f64(y).ravel(), _f64(inducing)
    r = fsa_request()
    r.kind = kind
    r.n = locs.shape[0]
    r.m = inducing.shape[0]
    r.locs, r.y, r.inducing = locs.ctypes.data, y.ctypes.data, inducing.ctypes.data
    r.theta = make_theta(theta)
    r.taper_range = float(taper_range)
    keep = [locs, y, inducing]
    if kind == REQ_PREDICT_VAR:
        pred = _f64(pred_locs)
        r.n_p = pred.shape[0]
        r.pred_locs = pred.ctypes.data
        r.num_samples = int(num_samples)
        keep.append(pred)
    r.arrival_ms = float(arrival_ms)
    return r, keep


def request_footprint(kind, locs, y, theta, inducing, taper_range, pred_locs=None, num_samples=0, **opts):
    """Device bytes fsa_request_footprint reserves for a request."""
    r, keep = _request(kind, locs, y, theta, inducing, taper_range, pred_locs, num_samples)
    o = make_options(**opts)
    b = C.c_uint64()
    _check(lib().fsa_request_footprint(C.byref(r), C.byref(o), C.byref(b)))
    del keep
    return int(b.value)


class Server:
    """A serving loop on the current GPU (fsa_server_*): `slots` workers with
    a stream each, admission by footprint against `hbm_budget` bytes of device
    memory reserved at creation.  Solver options as for FSA (precision,
    num_probes, seed, tol, ...)."""

    def __init__(self, slots=4, hbm_budget=64 << 30, **opts):
        o = fsa_server_options()
        o.slots = int(slots)
        o.hbm_budget = int(hbm_budget)
        o.opt = make_options(**opts)
        h = C.c_void_p()
        _check(lib().fsa_server_create(C.byref(o), C.byref(h)))
        self.h = h
        self._np = {}

    def clock_ms(self):
        return lib().fsa_server_clock_ms(self.h)

    def submit(self, kind, locs, y, theta, inducing, taper_range, pred_locs=None, num_samples=0, arrival_ms=None):
        """Queue a request (its arrays are copied); returns its id."""
        r, keep = _request(kind, locs, y, theta, inducing, taper_range, pred_locs, num_samples,
                           self.clock_ms() if arrival_ms is None else arrival_ms)
        i = C.c_int64()
        _check(lib().fsa_server_submit(self.h, C.byref(r), C.byref(i)))
        del keep
        self._np[i.value] = r.n_p
        return i.value

    def wait(self, rid):
        """Block until request `rid` is done: (result dict, variances or None)."""
        res = fsa_result()
        n_p = self._np.pop(rid, 0)
        var = np.zeros(max(n_p, 1))
        _check(lib().fsa_server_wait(self.h, rid, C.byref(res), _dptr(var)))
        d = {k: getattr(res, k) for k, _ in fsa_result._fields_}
        d["grad"] = np.array(res.grad[:])
        d["message"] = res.message.decode(errors="replace")
        d["status_name"] = STATUS.get(res.status, res.status)
        return d, (var[:n_p] if n_p else None)

    def stats(self):
        st = fsa_server_stats()
        _check(lib().fsa_server_get_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in fsa_server_stats._fields_}

    def close(self):
        if self.h:
            lib().fsa_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
