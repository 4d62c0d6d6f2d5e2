"""Pins for the direct O(p^2) masked covariance product."""
import numpy as np
import pytest
from scipy.linalg import toeplitz

from oracle.direct import full_matvec, masked_matvec
from oracle.geometry import embedding_lags, spectrum
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta


def test_one_row_exponential_is_ar1_toeplitz():
    n = 40
    g = grid(1, n)
    th = theta(0.1, 0.5, tau2=0.3)
    phi = np.exp(-(1.0 / n) / 0.1)
    K = toeplitz(phi ** np.arange(n)) + 0.3 * np.eye(n)
    v = synth.random_vectors(n, 2, seed=1).T
    got = masked_matvec(g, np.ones((1, n)), th, v)
    np.testing.assert_allclose(got, K @ v, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("th", [theta(0.2, 0.5), theta(0.1, 1.0, ratio=2.0, angle=np.pi / 6)])
def test_matches_circulant_fft_route(th):
    n1, n2 = 7, 9
    g = grid(n1, n2)
    mask = synth.uniform_mask(n1, n2, 0.3, seed=3)
    v = synth.random_vectors(int(mask.sum()), 1, seed=4)[0]
    got = masked_matvec(g, mask, th, v)
    # independent route: zero-padded circular convolution on a 16 x 18 torus
    lam = spectrum(embedding_lags(16, 18, g[2], g[3], th))
    X = np.zeros((16, 18))
    X[:n1, :n2][mask.astype(bool)] = v
    Y = np.real(np.fft.ifft2(lam * np.fft.fft2(X)))[:n1, :n2][mask.astype(bool)]
    eta = th["tau2"] / th["sigma2"]
    np.testing.assert_allclose(got, Y + eta * v, rtol=1e-12, atol=1e-12)
    full = full_matvec(g, th, X[:n1, :n2].ravel())
    Yf = np.real(np.fft.ifft2(lam * np.fft.fft2(X)))[:n1, :n2].ravel()
    np.testing.assert_allclose(full, Yf, rtol=1e-12, atol=1e-12)


def test_symmetric_positive_and_nugget_only():
    g = grid(6, 5)
    th = theta(0.3, 1.5, tau2=0.2, ratio=1.7, angle=0.3)
    mask = synth.uniform_mask(6, 5, 0.25, seed=8)
    p = int(mask.sum())
    u, v = synth.random_vectors(p, 2, seed=9)
    Ku = masked_matvec(g, mask, th, u)
    Kv = masked_matvec(g, mask, th, v)
    assert abs(u @ Kv - v @ Ku) < 1e-12 * np.linalg.norm(u) * np.linalg.norm(v)
    assert v @ Kv > 0
    # a range far below the cell spacing leaves only the diagonal
    th0 = theta(1e-5, 0.5, tau2=0.4)
    np.testing.assert_allclose(masked_matvec(g, mask, th0, v), 1.4 * v, rtol=1e-15)


def test_sampled_rows_equal_full_output():
    g = grid(8, 8)
    th = theta(0.2, 2.5)
    mask = synth.uniform_mask(8, 8, 0.4, seed=2)
    v = synth.random_vectors(int(mask.sum()), 1, seed=5)[0]
    full = masked_matvec(g, mask, th, v)
    rows = np.array([0, 3, 7, int(mask.sum()) - 1])
    np.testing.assert_array_equal(masked_matvec(g, mask, th, v, rows=rows), full[rows])
