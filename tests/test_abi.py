"""CPU checks of the C ABI: the library loads and exports every function that
include/kryging.h declares; host-side validation and error paths that need no
GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kryging.h")


def _lib_path():
    from paper_2012_13133_amd import build as b
    if not os.path.exists(b.OUT):
        b.build()
    return b.OUT


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(kry_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("kry_matvec", "kry_matvec_device", "kry_loglik", "kry_loglik_batch", "kry_krige", "kry_fit",
                 "kry_lanczos", "kry_logdet", "kry_gauss_quadrature", "kry_solve", "kry_gengk", "kry_lag_grid",
                 "kry_spectrum", "kry_sample", "kry_psd_torus", "kry_probes", "kry_server_create",
                 "kry_server_submit", "kry_server_poll", "kry_server_wait", "kry_server_destroy",
                 "kry_loglik_multi", "kry_autotune", "kry_set_tuning", "kry_get_tuning", "kry_set_graphs",
                 "kry_problem_set_covariates"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_paths_without_gpu():
    _lib_path()
    from paper_2012_13133_amd import kryging as K
    o = K.kry_opts_default()
    assert (o.lanczos_steps, o.num_probes, o.seed, o.precision, o.cg_rtol) == (30, 10, 303, 0, 1e-8)
    assert K.kry_status_string(K.KRY_ENOTPSD).startswith("circulant")
    # problem creation with a NULL context is rejected before any device work
    g = K.kry_grid(8, 8, 0.125, 0.125)
    h = ctypes.c_void_p()
    m = (ctypes.c_uint8 * 64)(*([1] * 64))
    st = K.lib.kry_problem_create(None, ctypes.byref(g), m, None, ctypes.byref(h))
    assert st == K.KRY_EINVAL
    # the embedding rule setting rejects a NULL context
    assert K.lib.kry_ctx_set_embedding(None, K.KRY_EMBED_SMALLEST) == K.KRY_EINVAL
    # gauss quadrature validates its sizes before touching the device
    one = (ctypes.c_double * 1)(1.0)
    steps = (ctypes.c_int32 * 1)(5)
    st = K.lib.kry_gauss_quadrature(1, 2, one, one, steps, one, one)
    assert st == K.KRY_EINVAL
    assert b"steps" in K.lib.kry_last_error()
    # server creation rejects bad arguments
    assert K.lib.kry_server_create(None, 2, 0, 4, 16, ctypes.byref(h)) == K.KRY_EINVAL
    # shift sharing is off by default; tuning, graphs and the multi-problem
    # call reject NULL handles before any device work
    assert o.shift_share == 0
    t = K.kry_tuning(2, 1, 1, 0, 0, 0.0)
    assert K.lib.kry_set_tuning(None, 64, 64, 1, ctypes.byref(t)) == K.KRY_EINVAL
    assert K.lib.kry_get_tuning(None, 64, 64, 1, ctypes.byref(t)) == K.KRY_EINVAL
    assert K.lib.kry_set_graphs(None, 1) == K.KRY_EINVAL
    assert K.lib.kry_autotune(None, 1, 8, ctypes.byref(t)) == K.KRY_EINVAL
    res = K.kry_loglik_result()
    assert K.lib.kry_loglik_multi(None, None, 1, ctypes.byref(o), ctypes.byref(res)) == K.KRY_EINVAL
    # covariates: NULL problem rejected; the restricted-likelihood switch is off by default
    assert K.lib.kry_problem_set_covariates(None, 1, None) == K.KRY_EINVAL
    assert o.reml == 0
    assert ctypes.sizeof(K.kry_loglik_result) == 8 * 7 + 4 * 2 + 8 + 8 + 8 * 2 * K.KRY_MAX_COVARIATES + 8


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_context_without_device_reports_edevice():
    _lib_path()
    from paper_2012_13133_amd import kryging as K
    with pytest.raises(K.KryError) as e:
        K.kry_ctx_create()
    assert e.value.status == K.KRY_EDEVICE


@pytest.mark.parametrize("k", [1, 2, 7, 60, 300])
def test_host_tridiagonal_eigen_solver(k):
    # the host step of the low-rank posterior variance, against numpy
    _lib_path()
    from paper_2012_13133_amd import kryging as K
    import numpy as np
    rng = np.random.default_rng(k)
    d = rng.uniform(0.1, 5.0, k)
    e = rng.uniform(-1.0, 1.0, max(k - 1, 0))
    if k >= 7:
        e[3] = 0.0  # a split
        d[:3] = 1.0  # a repeated diagonal block
        e[:2] = 0.0
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    theta, W = K.kry_tridiag_eigen(d, e)
    ref = np.linalg.eigvalsh(T)
    scale = np.abs(ref).max()
    assert np.all(np.diff(theta) >= 0)
    assert np.abs(theta - ref).max() <= 1e-13 * scale * max(1, k) ** 0.5
    assert np.abs(W.T @ W - np.eye(k)).max() <= 1e-13 * k
    assert np.abs(W @ np.diag(theta) @ W.T - T).max() <= 1e-13 * scale * k
