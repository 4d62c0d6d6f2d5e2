"""Dense Gaussian log-likelihood and kriging by Cholesky factorisation.

Test infrastructure only (see ``oracle/__init__``).

Model (Sec. 2, observation model): y = A x + eps, x ~ N(0, sigma^2 Sigma),
eps ~ N(0, tau^2 I); zero mean (no covariates).  The observations are
therefore y ~ N(0, sigma^2 K) with K = A Sigma A^T + eta I, eta = tau^2/sigma^2.

Log-likelihood (reading of the profile-likelihood objective of Sec. 3.1 and
3.4 for the marginal model; x integrated out, sigma^2 profiled):
    l(sigma^2)  = -1/2 [ p log(2 pi sigma^2) + log det K + Q / sigma^2 ],
    Q           = y^T K^{-1} y,
    sigma2_hat  = Q / p,
    l_p         = -1/2 [ p (log 2 pi + log sigma2_hat + 1) + log det K ].

Kriging (posterior of x given y, the closed form of eq. act_xhat restricted
to one cell t; c_t = correlation between t and every observed cell):
    E[x_t | y]  = c_t^T K^{-1} y
    var x_t     = sigma^2 (1 - c_t^T K^{-1} c_t)
    var y_t     = var x_t + tau^2
"""
import numpy as np
from scipy.linalg import cho_factor, cho_solve, solve_triangular

from .geometry import lag_table, observed_cells


def covariance(grid, mask, theta, table=None):
    """Dense unit-variance observed covariance K = A Sigma A^T + eta I."""
    n1, n2, dx1, dx2 = grid
    T = lag_table(n1, n2, dx1, dx2, theta) if table is None else table
    r, c = observed_cells(mask)
    K = T[r[:, None] - r[None, :] + n1 - 1, c[:, None] - c[None, :] + n2 - 1]
    K = K + (theta["tau2"] / theta["sigma2"]) * np.eye(r.size)
    return K


def full_correlation(grid, theta):
    """Dense n x n correlation Sigma over every cell (row-major ids)."""
    n1, n2, dx1, dx2 = grid
    T = lag_table(n1, n2, dx1, dx2, theta)
    ii, jj = np.divmod(np.arange(n1 * n2), n2)
    return T[ii[:, None] - ii[None, :] + n1 - 1, jj[:, None] - jj[None, :] + n2 - 1]


def loglik(grid, mask, theta, y_obs):
    """Exact marginal log-likelihood pieces at theta (sigma2, tau2 as given).

    Returns dict: logdet (log det K), quad (Q), loglik (l at theta's sigma2),
    sigma2_hat, loglik_profiled (l_p), p.
    """
    K = covariance(grid, mask, theta)
    p = K.shape[0]
    L = np.linalg.cholesky(K)
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    z = solve_triangular(L, np.asarray(y_obs, dtype=np.float64), lower=True)
    Q = float(z @ z)
    return assemble(p, logdet, Q, theta["sigma2"])


def assemble(p, logdet, Q, sigma2):
    """Likelihood assembly from (p, log det K, Q) -- the formulas in the
    module docstring."""
    ll = -0.5 * (p * np.log(2.0 * np.pi * sigma2) + logdet + Q / sigma2)
    s2 = Q / p
    llp = -0.5 * (p * (np.log(2.0 * np.pi) + np.log(s2) + 1.0) + logdet)
    return dict(logdet=float(logdet), quad=float(Q), loglik=float(ll),
                sigma2_hat=float(s2), loglik_profiled=float(llp), p=int(p))


def cross_correlation(grid, mask, theta, targets):
    """c_t for each target cell id: (p, T) correlations between observed cells
    and the targets (no nugget)."""
    n1, n2, dx1, dx2 = grid
    T = lag_table(n1, n2, dx1, dx2, theta)
    r, c = observed_cells(mask)
    ti, tj = np.divmod(np.asarray(targets, dtype=np.int64), n2)
    return T[r[:, None] - ti[None, :] + n1 - 1, c[:, None] - tj[None, :] + n2 - 1]


def krige(grid, mask, theta, y_obs, targets):
    """Dense simple-kriging mean and variances at target cell ids."""
    K = covariance(grid, mask, theta)
    cf = cho_factor(K, lower=True)
    C = cross_correlation(grid, mask, theta, targets)
    w = cho_solve(cf, np.asarray(y_obs, dtype=np.float64))
    mean = C.T @ w
    KC = cho_solve(cf, C)
    var_x = theta["sigma2"] * (1.0 - np.sum(C * KC, axis=0))
    var_y = var_x + theta["tau2"]
    return mean, var_x, var_y


def posterior_mean_all(grid, mask, theta, y_obs):
    """x_hat on every cell: Sigma A^T K^{-1} y (eq. act_xhat with X beta = 0,
    rewritten with the push-through identity)."""
    K = covariance(grid, mask, theta)
    w = np.linalg.solve(K, np.asarray(y_obs, dtype=np.float64))
    S = full_correlation(grid, theta)
    obs = np.flatnonzero(np.asarray(mask).ravel())
    return S[:, obs] @ w
