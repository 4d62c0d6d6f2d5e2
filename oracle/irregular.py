"""Irregularly spaced observations (Sec. 2): the latent field lives on the
grid and each observation is a convex combination of the grid values near
it, y = X beta + A x + eps.

Test infrastructure only (see ``oracle/__init__``).

The mapping matrix (Sec. 2): with d_ij = max(|s_i1 - s*_j1| / Delta_1,
|s_i2 - s*_j2| / Delta_2) between observation i and grid point j and the
Wendland function w(d) = (1 - d)_+^4 (1 + 4 d),
    A_ij = w(d_ij) / sum_k w(d_ik).
Coordinates (reading): locations are given in grid units, (u1, u2) =
(s1 / Delta_1, s2 / Delta_2) with grid point (row a, column b) at (a, b),
so d_ij = max(|u_i1 - a_j|, |u_i2 - b_j|) exactly.  Everything else is the
gridded model with A in place of the selection: K = A Sigma A^T + eta I,
and the likelihood and kriging of ``oracle.dense`` carry over.
"""
import numpy as np
from scipy.linalg import cho_factor, cho_solve
from scipy.sparse import csr_matrix

from . import philox
from .dense import assemble, full_correlation
from .geometry import lag_table
from .sampler import circulant_field


def wendland(d):
    d = np.asarray(d, dtype=np.float64)
    t = np.clip(1.0 - d, 0.0, None)
    return t ** 4 * (1.0 + 4.0 * d)


def mapping_matrix(grid, locs):
    """Dense A (p x n) by the definition: the weight of every grid point,
    normalised per observation."""
    n1, n2 = grid[0], grid[1]
    locs = np.asarray(locs, dtype=np.float64).reshape(-1, 2)
    ii, jj = np.divmod(np.arange(n1 * n2), n2)
    d = np.maximum(np.abs(locs[:, :1] - ii[None, :]), np.abs(locs[:, 1:] - jj[None, :]))
    W = wendland(d)
    return W / W.sum(axis=1, keepdims=True)


def covariance(grid, A, theta):
    """K = A Sigma A^T + eta I (unit variance)."""
    S = full_correlation(grid, theta)
    return A @ S @ A.T + (theta["tau2"] / theta["sigma2"]) * np.eye(A.shape[0])


def loglik(grid, locs, theta, y):
    """Exact marginal log-likelihood pieces (zero mean), as ``dense.loglik``."""
    A = mapping_matrix(grid, locs)
    K = covariance(grid, A, theta)
    L = np.linalg.cholesky(K)
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    z = np.linalg.solve(L, np.asarray(y, dtype=np.float64))
    return assemble(A.shape[0], logdet, float(z @ z), theta["sigma2"])


def krige_cells(grid, locs, theta, y, targets):
    """Kriging of the latent field at grid cells (ids): with c_t = A Sigma e_t,
        E[x_t | y] = c_t^T K^{-1} y,  var x_t = sigma2 (1 - c_t^T K^{-1} c_t),
        var y_t = var x_t + tau2."""
    A = mapping_matrix(grid, locs)
    S = full_correlation(grid, theta)
    K = A @ S @ A.T + (theta["tau2"] / theta["sigma2"]) * np.eye(A.shape[0])
    cf = cho_factor(K, lower=True)
    C = A @ S[:, np.asarray(targets, dtype=np.int64)]
    mean = C.T @ cho_solve(cf, np.asarray(y, dtype=np.float64))
    var_x = theta["sigma2"] * (1.0 - np.sum(C * cho_solve(cf, C), axis=0))
    return mean, var_x, var_x + theta["tau2"]


def matvec(grid, locs, theta, V):
    """K v for the columns of V by the dense definition."""
    A = mapping_matrix(grid, locs)
    return covariance(grid, A, theta) @ np.asarray(V, dtype=np.float64)


def mapping_sparse(grid, locs):
    """The same A as ``mapping_matrix`` in sparse form: w vanishes beyond
    distance 1, so only the corners of each observation's cell can carry
    weight; the definition is evaluated there."""
    n1, n2 = grid[0], grid[1]
    locs = np.asarray(locs, dtype=np.float64).reshape(-1, 2)
    p = locs.shape[0]
    rows, cols, vals = [], [], []
    for i, (u1, u2) in enumerate(locs):
        a0, b0 = min(int(np.floor(u1)), n1 - 1), min(int(np.floor(u2)), n2 - 1)
        cand = [(a, b) for a in (a0, a0 + 1) for b in (b0, b0 + 1) if a < n1 and b < n2]
        w = np.array([wendland(max(abs(u1 - a), abs(u2 - b))) for a, b in cand])
        w = w / w.sum()
        for (a, b), wv in zip(cand, w):
            if wv > 0:
                rows.append(i)
                cols.append(a * n2 + b)
                vals.append(wv)
    return csr_matrix((vals, (rows, cols)), shape=(p, n1 * n2))


def matvec_rows(grid, locs, theta, v, rows):
    """Selected entries of K v = A Sigma A^T v + eta v for one vector v,
    computed from the definition: u = A^T v on the grid, then for each
    needed cell the direct sum of Sigma's row against u."""
    n1, n2, dx1, dx2 = grid
    A = mapping_sparse(grid, locs)
    u = A.T @ np.asarray(v, dtype=np.float64)
    T = lag_table(n1, n2, dx1, dx2, theta)
    ii, jj = np.divmod(np.arange(n1 * n2), n2)
    out = np.empty(len(rows))
    for k, r in enumerate(rows):
        row = A.getrow(r)
        acc = 0.0
        for c, w in zip(row.indices, row.data):
            a, b = divmod(int(c), n2)
            acc += w * float(T[a - ii + n1 - 1, b - jj + n2 - 1] @ u)
        out[k] = acc + (theta["tau2"] / theta["sigma2"]) * v[r]
    return out


def bootstrap_variance(grid, locs, theta, targets, B, N1, N2, seed):
    """eq. bootstrap_uq with irregular observations: y_b = A x_b + tau eps_b
    with eps at observation index j (Philox stream b, domain NOISE); the
    prediction target's simulated observation as in ``oracle.bootstrap``."""
    n1, n2 = grid[0], grid[1]
    A = mapping_matrix(grid, locs)
    p = A.shape[0]
    targets = np.asarray(targets, dtype=np.int64)
    tau = np.sqrt(theta["tau2"])
    sx = np.zeros(targets.size)
    sy = np.zeros(targets.size)
    for b in range(B):
        x, _ = circulant_field(grid, theta, N1, N2, seed, stream=b)
        xf = x.ravel()
        yb = A @ xf + tau * philox.normals(np.arange(p), b, seed, philox.DOMAIN_NOISE)
        xhat, _, _ = krige_cells(grid, locs, theta, yb, targets)
        yt = xf[targets] + tau * philox.normals(targets, b, seed, philox.DOMAIN_TARGET)
        sx += (xf[targets] - xhat) ** 2
        sy += (yt - xhat) ** 2
    return sx / B, sy / B
