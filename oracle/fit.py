"""Profile-likelihood maximisation over (range, nugget ratio).

Test infrastructure only (see ``oracle/__init__``).

Sec. 3.4 maximises the profile likelihood over log-transformed parameters
with a generic optimiser.  Here the objective is the exact dense l_p (sigma^2
profiled, see ``oracle.dense``) over (log rho, log eta) with nu and the
anisotropy fixed; scipy's Nelder-Mead is the optimiser.
"""
import numpy as np
from scipy.optimize import minimize

from .dense import loglik


def profile_objective(grid, mask, y_obs, base, log_rho, log_eta):
    th = dict(base)
    th["range"] = float(np.exp(log_rho))
    th["sigma2"] = 1.0
    th["tau2"] = float(np.exp(log_eta))
    return loglik(grid, mask, th, y_obs)["loglik_profiled"]


def fit(grid, mask, y_obs, base, x0, xatol=1e-4, fatol=1e-8, maxiter=400):
    """Returns (rho_hat, eta_hat, l_p at the optimum)."""
    f = lambda t: -profile_objective(grid, mask, y_obs, base, t[0], t[1])
    res = minimize(f, np.asarray(x0, dtype=np.float64), method="Nelder-Mead",
                   options=dict(xatol=xatol, fatol=fatol, maxiter=maxiter))
    return float(np.exp(res.x[0])), float(np.exp(res.x[1])), float(-res.fun)
