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


def _odd_factors(N):
    """(the part of N without factors 2, 3, 5, 7; how many factors 3, 5, 7)."""
    k = 0
    while N % 2 == 0:
        N //= 2
    for q in (3, 5, 7):
        while N % q == 0:
            N //= q
            k += 1
    return N, k


def supported_side(N):
    """The sides the library's transforms take: powers of two, and multiples
    of 16 with no prime factor above 7, in [16, 8192]."""
    if N < 16 or N > 8192:
        return False
    if N & (N - 1) == 0:
        return True
    return N % 16 == 0 and _odd_factors(N)[0] == 1


def fast_size(m, rule="fast"):
    """Embedding side for a need of m >= 2n - 1 (any such side gives the
    exact product; this only sets cost and memory).  rule "smallest": the
    smallest supported side >= max(16, m).  rule "fast": the supported side
    >= max(16, m) with the least N w(N), w = 1 for powers of two, 1.2 for a
    side with one factor 3, 5 or 7 and 1.75 for a side with more (ties to the
    smaller side).  None beyond 8192."""
    best = None
    N = max(16, int(m))
    while N <= 8192:
        if supported_side(N):
            if rule == "smallest":
                return N
            w = 1.0 if N & (N - 1) == 0 else (1.2 if _odd_factors(N)[1] == 1 else 1.75)
            if best is None or N * w < best[0]:
                best = (N * w, N)
            if N & (N - 1) == 0:
                break
        N += 1
    return None if best is None else best[1]
