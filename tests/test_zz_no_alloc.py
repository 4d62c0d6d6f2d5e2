"""GPU: the product for callers that cannot allocate (kry_matvec_device_noalloc)
gives the results of kry_matvec_device, call after call."""
import numpy as np
import pytest

from oracle import sampler
from paper_2012_13133_amd import synth
from tests.gpu_util import DeviceArrays
from tests.oracle_cases import theta

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_2012_13133_amd.kryging")


def _device_product(fn, P, th, prec, V):
    # inputs and outputs in device memory; the library's own stream (NULL)
    D = DeviceArrays()
    try:
        Vt = V.astype(np.float64 if prec == K.KRY_FP64 else np.float32)
        dv = D.upload(Vt)
        do = D.empty_like(Vt, np.nan)
        fn(P.h, th, prec, V.shape[0], dv, do, None)
        return D.download(do, Vt).astype(np.float64)
    finally:
        D.close()


def _problem(n1, n2, frac, seed):
    mask = synth.uniform_mask(n1, n2, frac, seed=seed)
    y = synth.random_vectors(n1 * n2, 1, seed=seed + 1)[0].reshape(n1, n2)
    return K.Problem(n1, n2, mask, y)


@pytest.mark.parametrize("prec", [0, 1])
def test_no_alloc_product_equals_the_allocating_one(prec):
    th = K.theta_from_dict(theta(0.08, 1.5, sigma2=1.3, tau2=0.2, ratio=1.7, angle=0.4))
    # two calls in a row, the second on a smaller problem with fewer vectors:
    # the scratch array keeps the first call's contents, which must not leak
    for (n1, n2, frac, nvec, seed) in [(72, 90, 0.3, 5, 3), (20, 24, 0.45, 2, 7)]:
        with _problem(n1, n2, frac, seed) as P:
            V = synth.random_vectors(P.p, nvec, seed=seed + 5)
            print("no-alloc product", n1, n2, nvec, "precision", prec, flush=True)
            got = _device_product(K.kry_matvec_device_noalloc, P, th, prec, V)
            ref = _device_product(K.kry_matvec_device, P, th, prec, V)
            np.testing.assert_array_equal(got, ref)


def test_no_alloc_product_in_chunks_and_its_limit():
    # 1024 x 1024 (embedding 2048 x 2048): 20 FP64 vectors do not fit the
    # scratch at once and go through in chunks, with the same results
    n = 1024
    th = K.theta_from_dict(theta(0.05, 0.5, tau2=0.2))
    with _problem(n, n, 0.3, 11) as P:
        V = synth.random_vectors(P.p, 20, seed=12)
        print("no-alloc product 1024^2, 20 FP64 vectors", flush=True)
        got = _device_product(K.kry_matvec_device_noalloc, P, th, K.KRY_FP64, V)
        ref = _device_product(K.kry_matvec_device, P, th, K.KRY_FP64, V)
        np.testing.assert_array_equal(got, ref)
    # a 2048 x 2048 grid (embedding 4096 x 4096) needs more scratch than the
    # array holds: refused before any work, outputs untouched
    n = 2048
    mask = np.ones((n, n), dtype=np.uint8)
    mask[::7, ::5] = 0
    with K.Problem(n, n, mask, np.zeros((n, n))) as P:
        D = DeviceArrays()
        try:
            z = np.zeros(P.p, dtype=np.float32)
            dv = D.upload(z)
            do = D.empty_like(z, 7.0)
            with pytest.raises(K.KryError) as e:
                K.kry_matvec_device_noalloc(P.h, th, K.KRY_FP32, 1, dv, do, None)
            assert e.value.status == K.KRY_EINVAL
            assert np.all(D.download(do, z) == 7.0)
        finally:
            D.close()
