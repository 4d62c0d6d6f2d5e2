"""Pins for the lag tables and the circulant embedding (Sec. 3, 3.3)."""
import numpy as np
import pytest

from oracle.dense import full_correlation
from oracle.geometry import embedding_lags, lag_table, spectrum
from tests.oracle_cases import grid, theta


def _bccb(c):
    N1, N2 = c.shape
    i1, i2 = np.divmod(np.arange(N1 * N2), N2)
    return c[(i1[:, None] - i1[None, :]) % N1, (i2[:, None] - i2[None, :]) % N2]


@pytest.mark.parametrize("th", [theta(0.2, 0.5), theta(0.1, 1.0, ratio=2.0, angle=np.pi / 6),
                                theta(0.3, 2.5, ratio=1.5, angle=1.0)])
@pytest.mark.parametrize("shape", [(5, 4, 10, 8), (4, 6, 8, 12), (3, 3, 5, 6), (4, 4, 9, 7)])
def test_embedding_contains_sigma_and_spectrum_is_eigenvalues(th, shape):
    n1, n2, N1, N2 = shape
    g = grid(n1, n2)
    c = embedding_lags(N1, N2, g[2], g[3], th)
    C = _bccb(c)
    # symmetric, and its n1 x n2 corner (as a sub-grid of the torus) is Sigma
    np.testing.assert_allclose(C, C.T, atol=1e-15)
    ids = (np.arange(n1)[:, None] * N2 + np.arange(n2)[None, :]).ravel()
    np.testing.assert_allclose(C[np.ix_(ids, ids)], full_correlation(g, th), atol=1e-15)
    lam = spectrum(c)
    np.testing.assert_allclose(np.sort(lam.ravel()), np.linalg.eigvalsh(C), atol=1e-12)
    assert abs(lam.sum() - N1 * N2 * c[0, 0]) < 1e-9 * N1 * N2
    assert np.max(np.abs(np.imag(np.fft.fft2(c)))) < 1e-12


def test_lag_table_symmetry():
    th = theta(0.15, 1.5, ratio=2.0, angle=0.5)
    T = lag_table(6, 5, 1 / 6, 1 / 5, th)
    np.testing.assert_array_equal(T, T[::-1, ::-1])
    assert T[5, 4] == 1.0


def test_fast_size_rule():
    # supported sides: powers of two, or multiples of 16 with prime factors
    # 2, 3, 5, 7 only; "smallest" takes the first, "fast" weighs mixed sides
    from oracle.geometry import fast_size, supported_side
    smallest = {5: 16, 17: 32, 47: 48, 99: 112, 111: 112, 119: 128, 199: 224, 783: 784, 1199: 1200,
                1399: 1440, 1759: 1792, 2047: 2048, 3199: 3200, 4079: 4096, 8192: 8192}
    for m, want in smallest.items():
        assert fast_size(m, "smallest") == want, (m, fast_size(m, "smallest"), want)
    # fast: w = 1.2 for one odd factor (1280 = 1536 < 2048; 1536 = 1843 <
    # 2048; 1792 = 2150 > 2048), 1.75 for more (1200, 1440, 2240 lose)
    fast = {79: 80, 1199: 1280, 1399: 1536, 1759: 2048, 1025: 1280, 2199: 2560, 4079: 4096, 47: 48, 2047: 2048,
            3199: 4096, 99: 128}
    for m, want in fast.items():
        assert fast_size(m) == want, (m, fast_size(m), want)
    assert fast_size(8193) is None and fast_size(8193, "smallest") is None
    assert supported_side(1400) is False and supported_side(1440) and not supported_side(1408)
