"""ctypes binding of libkryging.so (C ABI in include/kryging.h).

Argument marshalling only: every function here converts numpy arrays to
pointers, calls the C entry point of the same name and turns a non-zero
status into ``KryError``.  There is no fallback: if the HIP library is not
built, importing this module raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkryging.so")

KRY_OK, KRY_EINVAL, KRY_ENOMEM, KRY_EDEVICE, KRY_ENOTPSD, KRY_ENOCONV, KRY_EBUSY, KRY_ENOTIMPL = range(8)
KRY_FP64, KRY_FP32 = 0, 1
KRY_PROBE_RADEMACHER, KRY_PROBE_COLOURED = 0, 1
KRY_SOLVER_CG, KRY_SOLVER_GENGK = 0, 1


class KryError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (status %d): %s" % (_STATUS_NAMES.get(status, "?"), status, message))
        self.status = status


_STATUS_NAMES = {0: "KRY_OK", 1: "KRY_EINVAL", 2: "KRY_ENOMEM", 3: "KRY_EDEVICE", 4: "KRY_ENOTPSD",
                 5: "KRY_ENOCONV", 6: "KRY_EBUSY", 7: "KRY_ENOTIMPL"}


class kry_grid(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("dx1", C.c_double), ("dx2", C.c_double)]


class kry_matern(C.Structure):
    _fields_ = [("sigma2", C.c_double), ("tau2", C.c_double), ("range", C.c_double), ("nu", C.c_double),
                ("aniso_ratio", C.c_double), ("aniso_angle", C.c_double)]


class kry_opts(C.Structure):
    _fields_ = [("lanczos_steps", C.c_int32), ("num_probes", C.c_int32), ("probe_kind", C.c_int32),
                ("colour_period", C.c_int32), ("seed", C.c_uint64), ("reorth", C.c_int32),
                ("precision", C.c_int32), ("cg_rtol", C.c_double), ("cg_maxit", C.c_int32),
                ("solver", C.c_int32), ("gk_steps", C.c_int32), ("shift_share", C.c_int32),
                ("lanczos_max_steps", C.c_int32), ("lanczos_rtol", C.c_double), ("reml", C.c_int32)]


KRY_MAX_COVARIATES = 8


class kry_loglik_result(C.Structure):
    _fields_ = [("loglik", C.c_double), ("loglik_profiled", C.c_double), ("sigma2_hat", C.c_double),
                ("logdet", C.c_double), ("logdet_se", C.c_double), ("quad", C.c_double), ("p", C.c_int64),
                ("lanczos_steps_used", C.c_int32), ("cg_iters", C.c_int32), ("cg_relres", C.c_double),
                ("ncov", C.c_int32), ("beta", C.c_double * KRY_MAX_COVARIATES),
                ("beta_se", C.c_double * KRY_MAX_COVARIATES), ("logdet_xkx", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["beta"] = list(d["beta"][:self.ncov])
        d["beta_se"] = list(d["beta_se"][:self.ncov])
        return d


class kry_plik_result(C.Structure):
    _fields_ = [("pl", C.c_double), ("logdet_bccb", C.c_double), ("dlogdet_bccb", C.c_double),
                ("psi2", C.c_double), ("z2", C.c_double), ("grad_lam2", C.c_double), ("grad_range", C.c_double),
                ("grad_lame2", C.c_double), ("grad_beta", C.c_double * KRY_MAX_COVARIATES),
                ("ncov", C.c_int32), ("gk_steps", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["grad_beta"] = list(d["grad_beta"][:self.ncov])
        return d


class kry_tuning(C.Structure):
    _fields_ = [("col_vectors", C.c_int32), ("row_tile_scale", C.c_int32), ("row_vthreads", C.c_int32),
                ("col_split", C.c_int32), ("row_split", C.c_int32), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class kry_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("prob", C.c_void_p), ("theta", kry_matern), ("opts", kry_opts),
                ("targets", C.POINTER(C.c_int64)), ("ntargets", C.c_int64), ("variances", C.c_int32),
                ("mean_x", C.POINTER(C.c_double)), ("var_x", C.POINTER(C.c_double)),
                ("var_y", C.POINTER(C.c_double))]


class kry_response(C.Structure):
    _fields_ = [("status", C.c_int32), ("batch", C.c_int32), ("problems", C.c_int32), ("loglik", kry_loglik_result),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_end", C.c_double),
                ("footprint_bytes", C.c_uint64), ("workspace_bytes", C.c_uint64)]


KRY_REQ_LOGLIK, KRY_REQ_KRIGE = 0, 1

_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_I32P = C.POINTER(C.c_int32)
_SIGS = {
    "kry_status_string": (C.c_char_p, [C.c_int]),
    "kry_last_error": (C.c_char_p, []),
    "kry_opts_default": (C.c_int, [C.POINTER(kry_opts)]),
    "kry_ctx_create": (C.c_int, [C.c_int32, C.c_uint64, C.POINTER(_P)]),
    "kry_ctx_destroy": (None, [_P]),
    "kry_ctx_memory": (C.c_int, [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.c_int32]),
    "kry_ctx_set_embedding": (C.c_int, [_P, C.c_int32]),
    "kry_profile_begin": (C.c_int, [_P]),
    "kry_profile_end": (C.c_int, [_P, _DP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "kry_problem_create": (C.c_int, [_P, C.POINTER(kry_grid), C.POINTER(C.c_uint8), _DP, C.POINTER(_P)]),
    "kry_problem_set_data": (C.c_int, [_P, _DP]),
    "kry_problem_create_irregular": (C.c_int, [_P, C.POINTER(kry_grid), C.c_int64, _DP, _DP, C.POINTER(_P)]),
    "kry_problem_set_covariates": (C.c_int, [_P, C.c_int32, _DP]),
    "kry_problem_info": (C.c_int, [_P, C.POINTER(C.c_int64), _I32P, _I32P]),
    "kry_problem_destroy": (None, [_P]),
    "kry_lag_grid": (C.c_int, [_P, C.POINTER(kry_matern), C.c_int32, C.c_int32, _DP]),
    "kry_spectrum": (C.c_int, [_P, C.POINTER(kry_matern), C.c_int32, C.c_int32, _DP, _DP]),
    "kry_matvec": (C.c_int, [_P, C.POINTER(kry_matern), C.c_int32, C.c_int32, _DP, _DP]),
    "kry_matvec_device": (C.c_int, [_P, C.POINTER(kry_matern), C.c_int32, C.c_int32, _P, _P, _P]),
    "kry_matvec_device_noalloc": (C.c_int, [_P, C.POINTER(kry_matern), C.c_int32, C.c_int32, _P, _P, _P]),
    "kry_cov_apply_full": (C.c_int, [_P, C.POINTER(kry_matern), C.c_int32, C.c_int32, _DP, _DP]),
    "kry_probes": (C.c_int, [_P, C.POINTER(kry_opts), _I32P, _DP]),
    "kry_lanczos": (C.c_int, [_P, C.POINTER(kry_matern), C.POINTER(kry_opts), _DP, _DP, _I32P]),
    "kry_logdet": (C.c_int, [_P, C.POINTER(kry_matern), C.POINTER(kry_opts), _DP, _DP, _DP]),
    "kry_gauss_quadrature": (C.c_int, [C.c_int32, C.c_int32, _DP, _DP, _I32P, _DP, _DP]),
    "kry_solve": (C.c_int, [_P, C.POINTER(kry_matern), C.POINTER(kry_opts), C.c_int32, _DP, _DP, _I32P, _DP]),
    "kry_gengk": (C.c_int, [_P, C.POINTER(kry_matern), C.POINTER(kry_opts), _DP, _DP, _DP, _DP, _DP]),
    "kry_loglik": (C.c_int, [_P, C.POINTER(kry_matern), C.POINTER(kry_opts), C.POINTER(kry_loglik_result)]),
    "kry_loglik_batch": (C.c_int, [_P, C.POINTER(kry_matern), C.c_int32, C.POINTER(kry_opts),
                                   C.POINTER(kry_loglik_result)]),
    "kry_set_graphs": (C.c_int, [_P, C.c_int32]),
    "kry_autotune": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(kry_tuning)]),
    "kry_set_tuning": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(kry_tuning)]),
    "kry_get_tuning": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(kry_tuning)]),
    "kry_loglik_multi": (C.c_int, [C.POINTER(_P), C.POINTER(kry_matern), C.c_int32, C.POINTER(kry_opts),
                                   C.POINTER(kry_loglik_result)]),
    "kry_fit": (C.c_int, [_P, C.POINTER(kry_matern), C.c_uint32, C.POINTER(kry_opts), C.c_double, C.c_int32,
                          C.POINTER(kry_matern), C.POINTER(kry_loglik_result)]),
    "kry_bootstrap_theta": (C.c_int, [_P, C.POINTER(kry_matern), C.c_uint32, C.POINTER(kry_opts), C.c_double,
                                      C.c_int32, C.c_int32, C.POINTER(kry_matern), _DP]),
    "kry_krige": (C.c_int, [_P, C.POINTER(kry_matern), C.POINTER(kry_opts), C.POINTER(C.c_int64), C.c_int64,
                            _DP, _DP, _DP, C.c_int32]),
    "kry_psd_torus": (C.c_int, [_P, C.POINTER(kry_matern), _I32P, _I32P]),
    "kry_plik": (C.c_int, [_P, C.POINTER(kry_matern), _DP, C.POINTER(kry_opts), C.POINTER(kry_plik_result)]),
    "kry_plik_fit": (C.c_int, [_P, C.POINTER(kry_matern), _DP, C.c_uint32, C.POINTER(kry_opts), C.c_double,
                               C.c_double, C.c_int32, C.POINTER(kry_matern), _DP, C.POINTER(kry_plik_result),
                               _I32P]),
    "kry_posterior_variance": (C.c_int, [_P, C.POINTER(kry_matern), _DP, C.POINTER(kry_opts), _DP, _DP, _DP]),
    "kry_tridiag_eigen": (C.c_int, [C.c_int32, _DP, _DP, _DP, _DP]),
    "kry_sample": (C.c_int, [_P, C.POINTER(kry_matern), C.c_int32, C.c_int32, C.c_uint64, C.c_int32, C.c_int32,
                             _DP, _DP]),
    "kry_server_create": (C.c_int, [_P, C.c_int32, C.c_uint64, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "kry_server_submit": (C.c_int, [_P, C.POINTER(kry_request), C.POINTER(C.c_uint64)]),
    "kry_server_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(kry_response), C.POINTER(C.c_int32)]),
    "kry_server_wait": (C.c_int, [_P, C.c_uint64, C.POINTER(kry_response)]),
    "kry_server_destroy": (None, [_P]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libkryging.so is not built (%s); run `python -c \"import __graft_entry__ as g; "
                          "g.build()\"` first" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _check(status):
    if status != KRY_OK:
        raise KryError(status, lib.kry_last_error().decode(errors="replace"))


def _dp(a):
    return a.ctypes.data_as(_DP) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def theta(sigma2=1.0, tau2=0.1, range=0.1, nu=0.5, aniso_ratio=1.0, aniso_angle=0.0):
    return kry_matern(sigma2, tau2, range, nu, aniso_ratio, aniso_angle)


def theta_from_dict(d):
    return kry_matern(d.get("sigma2", 1.0), d.get("tau2", 0.1), d["range"], d["nu"],
                      d.get("aniso_ratio", 1.0), d.get("aniso_angle", 0.0))


# ---- functions with the ABI's names ---------------------------------------------------
def kry_status_string(s):
    return lib.kry_status_string(s).decode()


def kry_opts_default(**overrides):
    o = kry_opts()
    _check(lib.kry_opts_default(C.byref(o)))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def kry_ctx_create(device=0, hbm_budget_bytes=0):
    h = _P()
    _check(lib.kry_ctx_create(device, hbm_budget_bytes, C.byref(h)))
    return h


def kry_ctx_destroy(ctx):
    lib.kry_ctx_destroy(ctx)


KRY_EMBED_FAST, KRY_EMBED_SMALLEST = 0, 1


def kry_ctx_set_embedding(ctx, rule):
    _check(lib.kry_ctx_set_embedding(ctx, rule))


def kry_ctx_memory(ctx, reset_peak=False):
    """(bytes held now, most bytes held since creation or the last reset)"""
    a, pk = C.c_uint64(), C.c_uint64()
    _check(lib.kry_ctx_memory(ctx, C.byref(a), C.byref(pk), 1 if reset_peak else 0))
    return a.value, pk.value


def kry_profile_begin(ctx):
    _check(lib.kry_profile_begin(ctx))


def kry_profile_end(ctx):
    ms = np.zeros(3)
    n = np.zeros(3, dtype=np.int64)
    v = C.c_int64()
    _check(lib.kry_profile_end(ctx, _dp(ms), n.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(v)))
    return ms, n, v.value


def kry_problem_create(ctx, n1, n2, mask, y=None, dx1=None, dx2=None):
    g = kry_grid(n1, n2, 1.0 / n1 if dx1 is None else dx1, 1.0 / n2 if dx2 is None else dx2)
    m = np.ascontiguousarray(np.asarray(mask).reshape(n1 * n2) != 0, dtype=np.uint8)
    yy = None if y is None else _f64(np.asarray(y).reshape(n1 * n2))
    h = _P()
    _check(lib.kry_problem_create(ctx, C.byref(g), m.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(yy), C.byref(h)))
    return h


def kry_problem_create_irregular(ctx, n1, n2, locs, y=None, dx1=None, dx2=None):
    """locs: (p, 2) fractional (row, column) grid coordinates."""
    g = kry_grid(n1, n2, 1.0 / n1 if dx1 is None else dx1, 1.0 / n2 if dx2 is None else dx2)
    L = _f64(np.asarray(locs).reshape(-1, 2))
    yy = None if y is None else _f64(np.asarray(y).ravel())
    h = _P()
    _check(lib.kry_problem_create_irregular(ctx, C.byref(g), L.shape[0], _dp(L), _dp(yy), C.byref(h)))
    return h


def kry_problem_set_data(prob, y):
    yy = _f64(np.asarray(y).ravel())
    _check(lib.kry_problem_set_data(prob, _dp(yy)))


def kry_problem_set_covariates(prob, X):
    """X: (q, n1, n2) or (q, n1*n2) covariates over every cell; q = 0 or
    None restores the zero mean."""
    if X is None or np.size(X) == 0:
        _check(lib.kry_problem_set_covariates(prob, 0, None))
        return
    X = np.asarray(X)
    q = X.shape[0]
    xx = _f64(X.reshape(q, -1))
    _check(lib.kry_problem_set_covariates(prob, q, _dp(xx)))


def kry_problem_info(prob):
    p = C.c_int64()
    a = C.c_int32()
    b = C.c_int32()
    _check(lib.kry_problem_info(prob, C.byref(p), C.byref(a), C.byref(b)))
    return p.value, a.value, b.value


def kry_problem_destroy(prob):
    lib.kry_problem_destroy(prob)


def kry_lag_grid(prob, th, N1=0, N2=0):
    if N1 == 0:
        _, N1, N2 = kry_problem_info(prob)
    out = np.empty((N1, N2))
    _check(lib.kry_lag_grid(prob, C.byref(th), N1, N2, _dp(out)))
    return out


def kry_spectrum(prob, th, N1=0, N2=0):
    if N1 == 0:
        _, N1, N2 = kry_problem_info(prob)
    out = np.empty((N2 // 2 + 1, N1))
    mm = np.empty(2)
    _check(lib.kry_spectrum(prob, C.byref(th), N1, N2, _dp(out), _dp(mm)))
    return out, mm


def kry_matvec(prob, th, v, precision=KRY_FP64):
    v = _f64(np.atleast_2d(v))
    out = np.empty_like(v)
    _check(lib.kry_matvec(prob, C.byref(th), precision, v.shape[0], _dp(v), _dp(out)))
    return out


def kry_matvec_device_noalloc(prob, th, precision, nvec, d_v, d_out, stream=None):
    """kry_matvec_device without device allocation (scratch array; see the header)."""
    _check(lib.kry_matvec_device_noalloc(prob, C.byref(th), precision, nvec, C.c_void_p(d_v), C.c_void_p(d_out),
                                         C.c_void_p(stream) if stream else None))


def kry_matvec_device(prob, th, precision, nvec, d_v, d_out, stream=None):
    """d_v, d_out: device pointers (int), e.g. torch tensors' data_ptr()."""
    _check(lib.kry_matvec_device(prob, C.byref(th), precision, nvec, C.c_void_p(d_v), C.c_void_p(d_out),
                                 C.c_void_p(stream) if stream else None))


def kry_cov_apply_full(prob, th, w, n, precision=KRY_FP64):
    w = _f64(np.atleast_2d(w))
    out = np.empty((w.shape[0], n))
    _check(lib.kry_cov_apply_full(prob, C.byref(th), precision, w.shape[0], _dp(w), _dp(out)))
    return out


def kry_probes(prob, opts):
    n = C.c_int32()
    _check(lib.kry_probes(prob, C.byref(opts), C.byref(n), None))
    p, _, _ = kry_problem_info(prob)
    out = np.empty((n.value, p))
    _check(lib.kry_probes(prob, C.byref(opts), C.byref(n), _dp(out)))
    return out


def kry_lanczos(prob, th, opts):
    n = C.c_int32()
    _check(lib.kry_probes(prob, C.byref(opts), C.byref(n), None))
    m = opts.lanczos_steps
    a = np.empty((n.value, m))
    b = np.empty((n.value, m))
    s = np.empty(n.value, dtype=np.int32)
    _check(lib.kry_lanczos(prob, C.byref(th), C.byref(opts), _dp(a), _dp(b), s.ctypes.data_as(_I32P)))
    return a, b, s


def kry_logdet(prob, th, opts):
    n = C.c_int32()
    _check(lib.kry_probes(prob, C.byref(opts), C.byref(n), None))
    ld = C.c_double()
    se = C.c_double()
    per = np.empty(n.value)
    _check(lib.kry_logdet(prob, C.byref(th), C.byref(opts), C.byref(ld), C.byref(se), _dp(per)))
    return ld.value, se.value, per


def kry_gauss_quadrature(alpha, beta, steps, znorm2):
    alpha = _f64(alpha)
    beta = _f64(beta)
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    znorm2 = _f64(znorm2)
    n, m = alpha.shape
    out = np.empty(n)
    _check(lib.kry_gauss_quadrature(n, m, _dp(alpha), _dp(beta), steps.ctypes.data_as(_I32P), _dp(znorm2),
                                    _dp(out)))
    return out


def kry_solve(prob, th, opts, b, allow_noconv=False):
    b = _f64(np.atleast_2d(b))
    x = np.empty_like(b)
    it = np.empty(b.shape[0], dtype=np.int32)
    rr = np.empty(b.shape[0])
    s = lib.kry_solve(prob, C.byref(th), C.byref(opts), b.shape[0], _dp(b), _dp(x), it.ctypes.data_as(_I32P), _dp(rr))
    if not (allow_noconv and s == KRY_ENOCONV):
        _check(s)
    return x, it, rr


def kry_gengk(prob, th, opts, n=None):
    k = opts.gk_steps
    a = np.empty(k + 1)
    b = np.empty(k + 1)
    z = np.empty(k)
    x = None if n is None else np.empty(n)
    J = C.c_double()
    _check(lib.kry_gengk(prob, C.byref(th), C.byref(opts), _dp(a), _dp(b), _dp(z), _dp(x), C.byref(J)))
    return a, b, z, x, J.value


def kry_loglik(prob, th, opts, allow_noconv=False):
    r = kry_loglik_result()
    s = lib.kry_loglik(prob, C.byref(th), C.byref(opts), C.byref(r))
    if not (allow_noconv and s == KRY_ENOCONV):
        _check(s)
    return r.as_dict()


def kry_loglik_batch(prob, thetas, opts, allow_noconv=False):
    arr = (kry_matern * len(thetas))(*thetas)
    res = (kry_loglik_result * len(thetas))()
    s = lib.kry_loglik_batch(prob, arr, len(thetas), C.byref(opts), res)
    if not (allow_noconv and s == KRY_ENOCONV):
        _check(s)
    return [r.as_dict() for r in res]


def kry_loglik_multi(probs, thetas, opts, allow_noconv=False):
    """One parameter point per problem (handles from kry_problem_create or
    Problem.h), all problems on one context."""
    assert len(probs) == len(thetas)
    ps = (_P * len(probs))(*[p.value if isinstance(p, _P) else p for p in probs])
    arr = (kry_matern * len(thetas))(*thetas)
    res = (kry_loglik_result * len(thetas))()
    s = lib.kry_loglik_multi(ps, arr, len(thetas), C.byref(opts), res)
    if not (allow_noconv and s == KRY_ENOCONV):
        _check(s)
    return [r.as_dict() for r in res]


def kry_set_graphs(ctx, enable):
    _check(lib.kry_set_graphs(ctx, 1 if enable else 0))


def kry_autotune(prob, precision, nvec=32):
    t = kry_tuning()
    _check(lib.kry_autotune(prob, precision, nvec, C.byref(t)))
    return t.as_dict()


def kry_set_tuning(ctx, N1, N2, precision, col_vectors=None, row_tile_scale=1, row_vthreads=1, col_split=0,
                   row_split=0):
    """col_vectors None resets the configuration to the built-in default."""
    if col_vectors is None:
        _check(lib.kry_set_tuning(ctx, N1, N2, precision, None))
    else:
        t = kry_tuning(col_vectors, row_tile_scale, row_vthreads, col_split, row_split, 0.0)
        _check(lib.kry_set_tuning(ctx, N1, N2, precision, C.byref(t)))


def kry_get_tuning(ctx, N1, N2, precision):
    t = kry_tuning()
    _check(lib.kry_get_tuning(ctx, N1, N2, precision, C.byref(t)))
    return t.as_dict()


def kry_fit(prob, init, free_mask, opts, xtol=1e-3, maxiter=200):
    est = kry_matern()
    r = kry_loglik_result()
    _check(lib.kry_fit(prob, C.byref(init), free_mask, C.byref(opts), xtol, maxiter, C.byref(est), C.byref(r)))
    return est, r.as_dict()


def kry_krige(prob, th, opts, targets=None, ntargets=None, want_var=True, bootstrap_B=0):
    if targets is None:
        tg = None
        nt = ntargets
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tg.size
    mean = np.empty(nt)
    vx = np.empty(nt) if want_var else None
    vy = np.empty(nt) if want_var else None
    _check(lib.kry_krige(prob, C.byref(th), C.byref(opts),
                         tg.ctypes.data_as(C.POINTER(C.c_int64)) if tg is not None else None, nt,
                         _dp(mean), _dp(vx), _dp(vy), bootstrap_B))
    return mean, vx, vy


def kry_psd_torus(prob, th):
    a = C.c_int32()
    b = C.c_int32()
    _check(lib.kry_psd_torus(prob, C.byref(th), C.byref(a), C.byref(b)))
    return a.value, b.value


def kry_sample(prob, th, N1, N2, seed, first_stream, count, n1, n2):
    """count fields on the n1 x n2 grid of `prob` (n1, n2 as given to
    kry_problem_create); returns (fields (count, n1, n2), minmax)."""
    out = np.empty((count, n1, n2))
    mm = np.empty(2)
    _check(lib.kry_sample(prob, C.byref(th), N1, N2, seed, first_stream, count, _dp(out), _dp(mm)))
    return out, mm


def kry_bootstrap_theta(prob, theta_hat, opts, B, free_mask=3, xtol=1e-4, maxiter=300):
    est = (kry_matern * B)()
    sd = np.empty(2)
    _check(lib.kry_bootstrap_theta(prob, C.byref(theta_hat), free_mask, C.byref(opts), xtol, maxiter, B, est,
                                   _dp(sd)))
    return list(est), sd


def _beta_arg(beta):
    return None if beta is None else _f64(np.asarray(beta, dtype=np.float64).ravel())


def kry_plik(prob, th, opts, beta=None):
    r = kry_plik_result()
    b = _beta_arg(beta)
    _check(lib.kry_plik(prob, C.byref(th), _dp(b), C.byref(opts), C.byref(r)))
    return r.as_dict()


def kry_plik_fit(prob, init, opts, free_mask=7, beta0=None, delta0=0.5, gtol=1e-6, maxiter=100, q=0):
    est = kry_matern()
    b0 = _beta_arg(beta0)
    be = np.empty(max(q, 1))
    r = kry_plik_result()
    it = C.c_int32()
    _check(lib.kry_plik_fit(prob, C.byref(init), _dp(b0), free_mask, C.byref(opts), delta0, gtol, maxiter,
                            C.byref(est), _dp(be), C.byref(r), C.byref(it)))
    return est, be[:q], r.as_dict(), it.value


def kry_posterior_variance(prob, th, opts, n, beta=None, want_mean=False):
    vx = np.empty(n)
    vy = np.empty(n)
    mean = np.empty(n) if want_mean else None
    b = _beta_arg(beta)
    _check(lib.kry_posterior_variance(prob, C.byref(th), _dp(b), C.byref(opts), _dp(vx), _dp(vy), _dp(mean)))
    return vx, vy, mean


def kry_tridiag_eigen(d, e):
    d = _f64(np.asarray(d, dtype=np.float64))
    e = _f64(np.asarray(e, dtype=np.float64))
    k = d.size
    theta = np.empty(k)
    W = np.empty(k * k)
    _check(lib.kry_tridiag_eigen(k, _dp(d), _dp(e) if k > 1 else None, _dp(theta), _dp(W)))
    return theta, W.reshape(k, k).T  # column j = eigenvector j


def kry_server_create(ctx, slots=4, hbm_budget_bytes=0, max_batch=16, max_queue=4096):
    h = _P()
    _check(lib.kry_server_create(ctx, slots, hbm_budget_bytes, max_batch, max_queue, C.byref(h)))
    return h


class PendingRequest:
    """Keeps a submitted request's structure and output arrays alive."""

    def __init__(self, ticket, req, outputs):
        self.ticket, self.req, self.outputs = ticket, req, outputs


def kry_server_submit(srv, kind, prob, th, opts, targets=None, variances=False):
    """Submit a request; returns a PendingRequest (its outputs are filled when done)."""
    req = kry_request()
    req.kind = kind
    req.prob = prob
    req.theta = th
    req.opts = opts
    outputs = {}
    if kind == KRY_REQ_KRIGE:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        outputs["targets"] = tg
        outputs["mean_x"] = np.empty(tg.size)
        req.targets = tg.ctypes.data_as(C.POINTER(C.c_int64))
        req.ntargets = tg.size
        req.mean_x = _dp(outputs["mean_x"])
        if variances:
            req.variances = 1
            outputs["var_x"] = np.empty(tg.size)
            outputs["var_y"] = np.empty(tg.size)
            req.var_x = _dp(outputs["var_x"])
            req.var_y = _dp(outputs["var_y"])
    t = C.c_uint64()
    _check(lib.kry_server_submit(srv, C.byref(req), C.byref(t)))
    return PendingRequest(t.value, req, outputs)


def kry_server_poll(srv, pending):
    r = kry_response()
    d = C.c_int32()
    _check(lib.kry_server_poll(srv, pending.ticket, C.byref(r), C.byref(d)))
    return r if d.value else None


def kry_server_wait(srv, pending):
    r = kry_response()
    _check(lib.kry_server_wait(srv, pending.ticket, C.byref(r)))
    return r


def kry_server_destroy(srv):
    lib.kry_server_destroy(srv)


class Problem:
    """Owns a context and a problem handle (closes both)."""

    def __init__(self, n1, n2, mask, y=None, device=0, dx1=None, dx2=None, hbm_budget_bytes=0, embedding=None):
        self.n1, self.n2 = n1, n2
        self.ctx = kry_ctx_create(device, hbm_budget_bytes)
        try:
            if embedding is not None:
                kry_ctx_set_embedding(self.ctx, embedding)
            self.h = kry_problem_create(self.ctx, n1, n2, mask, y, dx1, dx2)
        except Exception:
            kry_ctx_destroy(self.ctx)
            raise
        self.p, self.N1, self.N2 = kry_problem_info(self.h)

    def close(self):
        if getattr(self, "h", None):
            kry_problem_destroy(self.h)
            self.h = None
        if getattr(self, "ctx", None):
            kry_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IrregularProblem(Problem):
    """Owns a context and an irregular problem handle (closes both)."""

    def __init__(self, n1, n2, locs, y=None, device=0, dx1=None, dx2=None, hbm_budget_bytes=0, embedding=None):
        self.n1, self.n2 = n1, n2
        self.ctx = kry_ctx_create(device, hbm_budget_bytes)
        try:
            if embedding is not None:
                kry_ctx_set_embedding(self.ctx, embedding)
            self.h = kry_problem_create_irregular(self.ctx, n1, n2, locs, y, dx1, dx2)
        except Exception:
            kry_ctx_destroy(self.ctx)
            raise
        self.p, self.N1, self.N2 = kry_problem_info(self.h)
