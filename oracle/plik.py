"""The paper's own objective: the profile log-likelihood of the latent model
(Sec. 3.1, eq. exact_plik), its approximation (Sec. 3.4, eq. prof_lik) with
the block-circulant log-determinant of Sec. 3.3 and the genGK quadratic
terms of Sec. 3.2, the approximate gradient of the appendix (eq.
approx_grad) and the trust-region fit with a rank-one Hessian (Sec. 3.4).

Test infrastructure only (see ``oracle/__init__``).

Notation: Sigma is the unit-variance correlation over all n cells, A selects
the p observed cells, b = y - X beta, sigma2 and tau2 are the variances
(lambda^2 = 1/sigma2, lambda_e^2 = 1/tau2 in the appendix).  The objectives
are written as the paper writes them, up to the constants it drops (no 2 pi
terms).
"""
import numpy as np

from .dense import full_correlation
from .geometry import embedding_lags, lag_table, spectrum
from .gengk import gengk, projected_solve


def _selection(mask):
    obs = np.flatnonzero(np.asarray(mask).ravel())
    A = np.zeros((obs.size, np.asarray(mask).size))
    A[np.arange(obs.size), obs] = 1.0
    return obs, A


def full_correlation_drange(grid, theta):
    """Dense d Sigma / d rho over every cell (BTTB like Sigma)."""
    n1, n2, dx1, dx2 = grid
    T = lag_table(n1, n2, dx1, dx2, theta, drange=True)
    ii, jj = np.divmod(np.arange(n1 * n2), n2)
    return T[ii[:, None] - ii[None, :] + n1 - 1, jj[:, None] - jj[None, :] + n2 - 1]


def _residual_data(y_obs, X_obs, beta):
    b = np.asarray(y_obs, dtype=np.float64).copy()
    if X_obs is not None and np.size(X_obs):
        b = b - np.asarray(X_obs, dtype=np.float64).reshape(b.size, -1) @ np.asarray(beta, dtype=np.float64)
    return b


def exact_plik(grid, mask, theta, y_obs, X_obs=None, beta=None, A=None):
    """eq. exact_plik, densely: x_hat of eq. act_xhat,
        x_hat = (Sigma^{-1}/sigma2 + A^T A/tau2)^{-1} A^T b / tau2,
        psi   = b - A x_hat,
        pl    = -(p/2) log tau2 - psi^T psi / (2 tau2) - (n/2) log sigma2
                - (1/2) log det Sigma - x_hat^T Sigma^{-1} x_hat / (2 sigma2).
    Also the exact gradient of eq. anal_grad with respect to (beta,
    lambda^2, rho, lambda_e^2), with dL = trace(Sigma^{-1} d Sigma).  A
    given (p x n) replaces the selection of the masked cells."""
    n1, n2 = grid[0], grid[1]
    n = n1 * n2
    s2, t2 = theta["sigma2"], theta["tau2"]
    S = full_correlation(grid, theta)
    if A is None:
        _, A = _selection(mask)
    p = A.shape[0]
    b = _residual_data(y_obs, X_obs, beta)
    Si = np.linalg.inv(S)
    Gam = np.linalg.inv(Si / s2 + A.T @ A / t2)
    x = Gam @ (A.T @ b) / t2
    psi = b - A @ x
    w = Si @ x  # Sigma^{-1} x_hat
    qx = float(x @ w)
    ld = float(np.linalg.slogdet(S)[1])
    pl = -0.5 * p * np.log(t2) - psi @ psi / (2 * t2) - 0.5 * n * np.log(s2) - 0.5 * ld - qx / (2 * s2)
    dS = full_correlation_drange(grid, theta)
    dL = float(np.trace(Si @ dS))
    grad = dict(lam2=0.5 * n * s2 - 0.5 * qx,
                rho=-0.5 * dL + 0.5 * float(w @ dS @ w) / s2,
                lame2=0.5 * p * t2 - 0.5 * float(psi @ psi))
    if X_obs is not None and np.size(X_obs):
        grad["beta"] = np.asarray(X_obs, dtype=np.float64).reshape(p, -1).T @ psi / t2
    return dict(pl=float(pl), x=x, psi=psi, quad_x=qx, logdet=ld, dL=dL, grad=grad)


def quadrant_lambdas(grid, theta, drange=False):
    """Sec. 3.3: eigenvalues of the (2 n1 - 1) x (2 n2 - 1) block circulant
    built from the lags |h1| < n1, |h2| < n2 (exactly the product's
    embedding at that size), at the frequencies p < n1, q < n2 only (the
    formula's index range, taken literally).  The DFT is real (the lag grid
    is even).  With drange, the same for d Sigma / d rho."""
    n1, n2, dx1, dx2 = grid
    c = embedding_lags(2 * n1 - 1, 2 * n2 - 1, dx1, dx2, theta, drange=drange)
    return spectrum(c)[:n1, :n2]


def quadrant_logdet(grid, theta):
    """log det-hat Sigma of Sec. 3.3: sum of the logs of the quadrant
    eigenvalues (ValueError if one is not positive)."""
    lam = quadrant_lambdas(grid, theta)
    if not np.all(lam > 0):
        raise ValueError("a quadrant eigenvalue is not positive")
    return float(np.sum(np.log(lam)))


def quadrant_dlogdet(grid, theta):
    """dL-hat of the appendix: trace(D1^{-1} D2) with D1, D2 the quadrant
    eigenvalues of Sigma and of d Sigma / d rho (eq. circ_diag,
    eq. trace_approx)."""
    return float(np.sum(quadrant_lambdas(grid, theta, drange=True) / quadrant_lambdas(grid, theta)))


def approx_plik(grid, mask, theta, y_obs, k, X_obs=None, beta=None, reorth=True, A=None):
    """eq. prof_lik with x_k* and z_k from k steps of Algorithm 1
    (``oracle.gengk``) and the quadrant log-determinant:
        pl~ = -(p/2) log tau2 - psi*^T psi* / (2 tau2) - (n/2) log sigma2
              - (1/2) logdet-hat Sigma - ||z_k||^2 / (2 sigma2),
    psi* = b - A x_k*, and the approximate gradient of eq. approx_grad:
        d/d beta        lambda_e^2 X^T psi*
        d/d lambda^2    n / (2 lambda^2) - ||z_k||^2 / 2
        d/d rho         -dL-hat / 2 + (lambda^2 / 2) z^T V^T dSigma V z
        d/d lambda_e^2  p / (2 lambda_e^2) - psi*^T psi* / 2.
    A given (p x n) replaces the selection of the masked cells."""
    n1, n2 = grid[0], grid[1]
    n = n1 * n2
    s2, t2 = theta["sigma2"], theta["tau2"]
    S = full_correlation(grid, theta)
    if A is None:
        _, A = _selection(mask)
    p = A.shape[0]
    b = _residual_data(y_obs, X_obs, beta)
    beta1, U, V, B, _, _ = gengk(A, S, b, t2, k, reorth=reorth)
    z, J = projected_solve(B, beta1, s2)
    w = V @ z
    x = S @ w
    psi = b - A @ x
    ld = quadrant_logdet(grid, theta)
    dL = quadrant_dlogdet(grid, theta)
    zz = float(z @ z)
    pp = float(psi @ psi)
    pl = -0.5 * p * np.log(t2) - pp / (2 * t2) - 0.5 * n * np.log(s2) - 0.5 * ld - zz / (2 * s2)
    dS = full_correlation_drange(grid, theta)
    grad = dict(lam2=0.5 * n * s2 - 0.5 * zz,
                rho=-0.5 * dL + 0.5 * float(w @ dS @ w) / s2,
                lame2=0.5 * p * t2 - 0.5 * pp)
    if X_obs is not None and np.size(X_obs):
        grad["beta"] = np.asarray(X_obs, dtype=np.float64).reshape(p, -1).T @ psi / t2
    return dict(pl=float(pl), x=x, psi=psi, z=z, zz=zz, psi2=pp, logdet=ld, dL=dL, grad=grad, J=J)


def log_gradient(theta, grad):
    """Gradient of pl~ in the fit's coordinates (log sigma2, log tau2,
    log rho, beta) from the appendix's (lambda^2, lambda_e^2, rho, beta):
    d/d log sigma2 = -lambda^2 d/d lambda^2, d/d log tau2 = -lambda_e^2
    d/d lambda_e^2, d/d log rho = rho d/d rho."""
    g = [-grad["lam2"] / theta["sigma2"], -grad["lame2"] / theta["tau2"], theta["range"] * grad["rho"]]
    return np.concatenate([g, np.asarray(grad.get("beta", []), dtype=np.float64)])


def trust_region_fit(f_and_grad, x0, delta0=0.5, gtol=1e-6, xtol=1e-8, maxiter=200):
    """Maximise f with the trust-region method of Sec. 3.4: the model of -f
    at x is m(s) = -f - g^T s + (g^T s)^2 / 2 (gradient g of f; the rank-one
    Hessian g g^T, the outer product of the score).  The model depends on s
    only through t = g^T s and is least at t = 1, so the step is the
    shortest s with g^T s = 1, s = g / ||g||^2, cut back to the trust radius
    along g.  The radius shrinks by 4 when the actual gain is under a quarter
    of the model's, and doubles when it exceeds three quarters at the
    boundary; steps with positive gain are taken.
    Returns (x, f(x), iterations)."""
    x = np.asarray(x0, dtype=np.float64)
    fx, g = f_and_grad(x)
    delta = delta0
    it = 0
    for it in range(1, maxiter + 1):
        gn = float(np.linalg.norm(g))
        if gn <= gtol:
            break
        if 1.0 / gn <= delta:
            s, boundary = g / gn ** 2, False
        else:
            s, boundary = delta * g / gn, True
        t = float(g @ s)
        pred = t - 0.5 * t * t  # model gain in f
        fn, gnew = f_and_grad(x + s)
        ratio = (fn - fx) / pred if pred > 0 else -1.0
        if ratio < 0.25:
            delta *= 0.25
        elif ratio > 0.75 and boundary:
            delta *= 2.0
        if ratio > 0:
            x, fx, g = x + s, fn, gnew
        if delta < xtol:
            break
    return x, fx, it
