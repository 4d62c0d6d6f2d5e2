"""Grid geometry, lag tables and the circulant-embedding lag grid.

Test infrastructure only (see ``oracle/__init__``).

Sec. 2: the latent field lives on a regular n1 x n2 grid; for gridded data
the mapping matrix A is the identity with the rows of unobserved cells
removed, so A Sigma A^T is the covariance among observed cells.  Sec. 3
notes that on a regular grid Sigma is symmetric block-Toeplitz with Toeplitz
blocks (BTTB): entry (a, b) depends only on the lag (i_a - i_b, j_a - j_b),
so the (2 n1 - 1) x (2 n2 - 1) lag table determines it.

Conventions (readings): cell (i, j) is row i (y direction, spacing dx1) and
column j (x direction, spacing dx2), row-major id i * n2 + j; observed cells
are numbered in row-major order ("compact" order).
"""
import numpy as np

from .matern import correlation


def observed_cells(mask):
    """(rows, cols) of observed cells of an n1 x n2 0/1 mask, in compact
    (row-major) order."""
    mask = np.asarray(mask).astype(bool)
    r, c = np.nonzero(mask)
    return r.astype(np.int64), c.astype(np.int64)


def lag_table(n1, n2, dx1, dx2, theta, drange=False):
    """Correlation at every lag (h1, h2), |h1| < n1, |h2| < n2, as an array T
    with T[h1 + n1 - 1, h2 + n2 - 1] = C(h2 dx2, h1 dx1) (Sec. 2 Matern,
    BTTB structure of Sec. 3); the range derivative of it when drange."""
    h1 = np.arange(-(n1 - 1), n1, dtype=np.float64)
    h2 = np.arange(-(n2 - 1), n2, dtype=np.float64)
    H1, H2 = np.meshgrid(h1, h2, indexing="ij")
    return correlation(H2 * dx2, H1 * dx1, theta, drange)


def wrapped_lag(l, N):
    """Signed lag represented by index l on a circle of length N: l for
    l < N/2, l - N for l > N/2; N/2 (even N) is the Nyquist alias."""
    l = np.asarray(l)
    return np.where(l <= N // 2, l, l - N)


def embedding_lags(N1, N2, dx1, dx2, theta, drange=False):
    """Lag grid c (N1 x N2) of the block-circulant embedding (Sec. 3.3: the
    circulant C is built exactly as for the circulant-embedding product).

    c[l1, l2] = C(h2 dx2, h1 dx1) with (h1, h2) the wrapped lags.  Reading for
    even N: index N/2 stands for both lags +N/2 and -N/2, so the value there
    is the mean of the correlation over all aliases.  This keeps
    c[l] = c[-l], hence a real spectrum.  The masked product only needs lags
    |h| <= n - 1, and n - 1 < N/2 whenever N >= 2n - 1, so it never reads a
    Nyquist line.  With drange the lag grid holds the derivative of the
    correlation with respect to the range instead.
    """
    def aliases(N):
        out = []
        for l in range(N):
            if N % 2 == 0 and l == N // 2:
                out.append((l, -l))
            else:
                out.append((l if l < N / 2 else l - N,))
        return out
    a1 = aliases(N1)
    a2 = aliases(N2)
    c = np.zeros((N1, N2))
    # rows/columns without an alias pair are evaluated in one vectorised call
    h1 = np.array([a[0] for a in a1], dtype=np.float64)
    h2 = np.array([a[0] for a in a2], dtype=np.float64)
    H1, H2 = np.meshgrid(h1, h2, indexing="ij")
    c[:] = correlation(H2 * dx2, H1 * dx1, theta, drange)
    for i, al1 in enumerate(a1):
        for j, al2 in (list(enumerate(a2)) if len(al1) > 1 else
                       [(j, a) for j, a in enumerate(a2) if len(a) > 1]):
            vals = [correlation(s2 * dx2, s1 * dx1, theta, drange) for s1 in al1 for s2 in al2]
            c[i, j] = float(np.mean(vals))
    return c


def spectrum(c):
    """Eigenvalues of the block-circulant matrix whose first row is the lag
    grid c: the 2-D DFT of c (real for an even lag grid).  Returns the full
    N1 x N2 real array."""
    return np.real(np.fft.fft2(c))


def fast_size(m):
    """Smallest side >= max(16, m) of the form 2^a 3^b 5^c with 16 | side whose
    half has at most one factor 3 or 5 beyond 2^3, within 8192 (the sides the
    library's transforms take: powers of two, 3 * 2^a, 5 * 2^a; any side
    >= 2n - 1 gives the exact product, so this only sets the cost)."""
    N = max(16, int(m))
    while N <= 8192:
        k = N // 16
        if N % 16 == 0 and (k & (k - 1) == 0 or (k % 3 == 0 and (k // 3) & (k // 3 - 1) == 0)
                            or (k % 5 == 0 and (k // 5) & (k // 5 - 1) == 0)):
            return N
        N += 1
    return None
