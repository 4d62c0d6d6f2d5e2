"""Gaussian-field samplers: exact Cholesky and circulant embedding.

Test infrastructure only (see ``oracle/__init__``).

Sec. 3.5 draws bootstrap fields x_b ~ N(0, sigma^2 Sigma) on the grid; the
closing caveat of Sec. 3.6 says this is done by circulant embedding, which
needs a positive semi-definite embedding and otherwise resets small negative
eigenvalues.  With C the block-circulant embedding (lag grid c, eigenvalues
lam = DFT2(c)) and xi white noise on the N1 x N2 torus,
    x_torus = C^{1/2} xi = IDFT2( sqrt(lam) * DFT2(xi) ),
has covariance C, and its n1 x n2 corner has covariance Sigma.
"""
import numpy as np

from . import philox
from .geometry import embedding_lags, spectrum


def cholesky_field(grid, theta, seed, stream=0):
    """x = chol(sigma^2 Sigma) xi1 on all cells and y = x + tau xi2 (every
    cell), xi from the Philox normal streams (cell id as index)."""
    from .dense import full_correlation
    n1, n2 = grid[0], grid[1]
    S = full_correlation(grid, theta) * theta["sigma2"]
    L = np.linalg.cholesky(S)
    ids = np.arange(n1 * n2)
    xi1 = philox.normals(ids, stream, seed, philox.DOMAIN_FIELD)
    xi2 = philox.normals(ids, stream, seed, philox.DOMAIN_NOISE)
    x = L @ xi1
    y = x + np.sqrt(theta["tau2"]) * xi2
    return x.reshape(n1, n2), y.reshape(n1, n2)


def torus_spectrum(grid, theta, N1, N2):
    """Eigenvalues of the N1 x N2 block-circulant embedding, full array."""
    _, _, dx1, dx2 = grid
    return spectrum(embedding_lags(N1, N2, dx1, dx2, theta))


def circulant_field(grid, theta, N1, N2, seed, stream=0, clip_tol=1e-10):
    """One field on the n1 x n2 grid by circulant embedding on an N1 x N2 torus.

    Returns (x, min_lam / max_lam).  Raises ValueError if the embedding is not
    PSD within clip_tol (relative); tiny negative eigenvalues are reset to 0.
    """
    n1, n2 = grid[0], grid[1]
    lam = torus_spectrum(grid, theta, N1, N2)
    ratio = lam.min() / lam.max()
    if ratio < -clip_tol:
        raise ValueError("embedding not PSD: min/max = %g" % ratio)
    lam = np.maximum(lam, 0.0)
    ids = np.arange(N1 * N2)
    xi = philox.normals(ids, stream, seed, philox.DOMAIN_FIELD).reshape(N1, N2)
    xt = circulant_sqrt_apply(lam, xi)
    return np.sqrt(theta["sigma2"]) * xt[:n1, :n2], float(ratio)


def circulant_sqrt_apply(lam, xi):
    """C^{1/2} xi on the torus for a non-negative spectrum lam (N1 x N2)."""
    return np.real(np.fft.ifft2(np.sqrt(lam) * np.fft.fft2(xi)))


def psd_torus(grid, theta, N1, N2, cap=8192, tol=1e-10):
    """Reading of the Sec. 3.6 caveat: starting from (N1, N2), double both
    torus sides until the embedding spectrum has min >= -tol * max; None if
    the cap is passed first."""
    while True:
        lam = torus_spectrum(grid, theta, N1, N2)
        if lam.min() >= -tol * lam.max():
            return N1, N2
        if 2 * N1 > cap or 2 * N2 > cap:
            return None
        N1 *= 2
        N2 *= 2
