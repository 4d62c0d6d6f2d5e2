"""Dense Gaussian log-likelihood and kriging by Cholesky factorisation.

Test infrastructure only (see ``oracle/__init__``).

Model (Sec. 2, eq. obs_mod): y = X beta + A x + eps, x ~ N(0, sigma^2 Sigma),
eps ~ N(0, tau^2 I).  The observations are therefore y ~ N(X beta, sigma^2 K)
with K = A Sigma A^T + eta I, eta = tau^2/sigma^2.  The functions without
covariates take beta = 0 (X empty); the ``*_covariates`` functions below
estimate beta.

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


# ---- covariates (eq. obs_mod with X beta) --------------------------------------------


def gls(K, X, y):
    """Generalised least squares for y ~ N(X beta, sigma^2 K): the beta that
    maximises the likelihood at fixed covariance parameters solves the
    normal equations X^T K^{-1} (y - X beta) = 0 (the beta-gradient of the
    appendix's profile likelihood, set to zero, in the marginal form), so

        beta_hat = (X^T K^{-1} X)^{-1} X^T K^{-1} y,
        Q        = (y - X beta_hat)^T K^{-1} (y - X beta_hat).

    Returns beta_hat, G = X^T K^{-1} X and Q."""
    X = np.asarray(X, dtype=np.float64).reshape(K.shape[0], -1)
    y = np.asarray(y, dtype=np.float64)
    cf = cho_factor(K, lower=True)
    KX = cho_solve(cf, X)
    G = X.T @ KX
    g = KX.T @ y
    beta = np.linalg.solve(G, g) if X.shape[1] else np.zeros(0)
    r = y - X @ beta
    Q = float(r @ cho_solve(cf, r))
    return beta, G, Q


def loglik_covariates(grid, mask, theta, y_obs, X_obs, reml=False):
    """Log-likelihood with the mean X beta profiled at beta_hat (``gls``).

    X_obs: (p, q) covariates at the observed cells, increasing cell id.

    Maximum likelihood (reml=False): the formulas of ``loglik`` with
    Q = (y - X beta_hat)^T K^{-1} (y - X beta_hat).

    Restricted likelihood (reml=True; not in the paper, the standard
    alternative for the covariance parameters): the likelihood of the error
    contrasts L y, L with orthonormal rows spanning the complement of X's
    columns, which is (m = p - q)
        l_R   = -1/2 [ m log(2 pi sigma^2) + log det K + log det(X^T K^{-1} X)
                       - log det(X^T X) + Q / sigma^2 ],
        sigma2_hat = Q / m,
        l_R,p = -1/2 [ m (log 2 pi + log sigma2_hat + 1) + log det K
                       + log det(X^T K^{-1} X) - log det(X^T X) ].

    Also returns beta, beta_se = sqrt(diag(sigma2_hat (X^T K^{-1} X)^{-1}))
    and logdet_xkx = log det(X^T K^{-1} X).
    """
    K = covariance(grid, mask, theta)
    X = np.asarray(X_obs, dtype=np.float64).reshape(K.shape[0], -1)
    p, q = X.shape
    L = np.linalg.cholesky(K)
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    beta, G, Q = gls(K, X, y_obs)
    ld_xkx = float(np.linalg.slogdet(G)[1]) if q else 0.0
    ld_xx = float(np.linalg.slogdet(X.T @ X)[1]) if q else 0.0
    if not reml:
        out = assemble(p, logdet, Q, theta["sigma2"])
    else:
        m = p - q
        s2 = Q / m
        extra = logdet + ld_xkx - ld_xx
        out = dict(logdet=float(logdet), quad=float(Q),
                   loglik=float(-0.5 * (m * np.log(2.0 * np.pi * theta["sigma2"]) + extra + Q / theta["sigma2"])),
                   sigma2_hat=float(s2),
                   loglik_profiled=float(-0.5 * (m * (np.log(2.0 * np.pi) + np.log(s2) + 1.0) + extra)),
                   p=int(p))
    cov = out["sigma2_hat"] * np.linalg.inv(G) if q else np.zeros((0, 0))
    out.update(beta=beta, beta_se=np.sqrt(np.diag(cov)), logdet_xkx=ld_xkx)
    return out


def krige_covariates(grid, mask, theta, y_obs, X_obs, X_targets, targets):
    """Kriging with the mean at its GLS estimate (plug-in: beta treated as
    known at beta_hat, as the bootstrap of Sec. 3.5 does):
        mean_t = X_t beta_hat + c_t^T K^{-1} (y - X beta_hat),
    and the variances of ``krige`` (they do not involve the mean).
    X_targets: (T, q) covariates at the targets."""
    K = covariance(grid, mask, theta)
    X = np.asarray(X_obs, dtype=np.float64).reshape(K.shape[0], -1)
    beta, _, _ = gls(K, X, y_obs)
    r = np.asarray(y_obs, dtype=np.float64) - X @ beta
    mean, var_x, var_y = krige(grid, mask, theta, r, targets)
    Xt = np.asarray(X_targets, dtype=np.float64).reshape(len(targets), -1)
    return Xt @ beta + mean, var_x, var_y, beta
