"""Direct O(p^2) masked covariance product.

Test infrastructure only (see ``oracle/__init__``).

With gridded data A is the identity with unobserved rows removed (Sec. 2),
so the unit-variance covariance of the observations is
    K = A Sigma A^T + eta I,   eta = tau^2 / sigma^2,
and (K v)_a = sum_{b observed} C(s_a - s_b) v_b + eta v_a.  The paper's fast
route (circulant embedding + FFT, Sec. 3 and 3.2) reaches this exactly up to
rounding; this module is the plain sum.
"""
import numpy as np

from .geometry import lag_table, observed_cells


def _lags(grid, theta):
    n1, n2, dx1, dx2 = grid
    return lag_table(n1, n2, dx1, dx2, theta)


def masked_matvec(grid, mask, theta, v, eta=None, rows=None, table=None):
    """(K v) for compact vectors v (p,) or (p, m).

    ``rows`` optionally restricts the output to those compact indices (each
    still a full O(p) sum), so large grids can be checked on a sample.
    ``eta`` defaults to tau2 / sigma2 of ``theta``.
    """
    n1, n2 = grid[0], grid[1]
    if eta is None:
        eta = theta["tau2"] / theta["sigma2"]
    T = _lags(grid, theta) if table is None else table
    r, c = observed_cells(mask)
    v = np.asarray(v, dtype=np.float64)
    out_idx = np.arange(r.size) if rows is None else np.asarray(rows)
    out = np.empty((out_idx.size,) + v.shape[1:])
    for k, a in enumerate(out_idx):
        row = T[r[a] - r + n1 - 1, c[a] - c + n2 - 1]
        out[k] = row @ v + eta * v[a]
    return out


def full_matvec(grid, theta, v, table=None):
    """Sigma v for a full-grid vector v (n1*n2,) (no nugget): the unmasked
    product used by the Golub-Kahan recurrences (Algorithm 1) and by the
    kriging mean Sigma A^T w."""
    n1, n2 = grid[0], grid[1]
    T = _lags(grid, theta) if table is None else table
    ii, jj = np.divmod(np.arange(n1 * n2), n2)
    v = np.asarray(v, dtype=np.float64)
    out = np.empty_like(v)
    for a in range(n1 * n2):
        out[a] = T[ii[a] - ii + n1 - 1, jj[a] - jj + n2 - 1] @ v
    return out
