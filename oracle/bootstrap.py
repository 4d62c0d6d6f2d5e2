"""Parametric bootstrap prediction variance (Sec. 3.5, eq. bootstrap_uq).

Test infrastructure only (see ``oracle/__init__``).

For b = 1..B at the fitted theta: draw x_b ~ N(0, sigma^2 Sigma) on the grid,
form y_b = A x_b + eps_b, krige x_hat_b from y_b with theta known, and
estimate
    var x(s_i) ~ (1/B) sum_b (x_b(s_i) - x_hat_b(s_i))^2
    var y(s_i) ~ (1/B) sum_b (y_b(s_i) - y_hat_b(s_i))^2
at each prediction cell.  Noise draws (readings): eps_b at observed cell id
uses the Philox normal stream b of domain NOISE; the simulated observation
at a prediction cell uses stream b of domain TARGET; fields use stream b of
domain FIELD on the torus.
"""
import numpy as np

from . import philox
from .dense import krige
from .fit import fit
from .sampler import circulant_field


def bootstrap_variance(grid, mask, theta, targets, B, N1, N2, seed):
    n1, n2 = grid[0], grid[1]
    mask = np.asarray(mask).astype(bool)
    obs = np.flatnonzero(mask.ravel())
    targets = np.asarray(targets, dtype=np.int64)
    tau = np.sqrt(theta["tau2"])
    sx = np.zeros(targets.size)
    sy = np.zeros(targets.size)
    for b in range(B):
        x, _ = circulant_field(grid, theta, N1, N2, seed, stream=b)
        xf = x.ravel()
        yb = xf[obs] + tau * philox.normals(obs, b, seed, philox.DOMAIN_NOISE)
        xhat, _, _ = krige(grid, mask, theta, yb, targets)
        yt = xf[targets] + tau * philox.normals(targets, b, seed, philox.DOMAIN_TARGET)
        sx += (xf[targets] - xhat) ** 2
        sy += (yt - xhat) ** 2
    return sx / B, sy / B


def bootstrap_data(grid, mask, theta, b, N1, N2, seed):
    """Simulated observations of draw b, the y_b of ``bootstrap_variance``:
    x_b on the torus (Philox stream b, domain FIELD) at the observed cells
    plus tau eps_b (stream b, domain NOISE, cell id as index)."""
    obs = np.flatnonzero(np.asarray(mask).astype(bool).ravel())
    x, _ = circulant_field(grid, theta, N1, N2, seed, stream=b)
    return x.ravel()[obs] + np.sqrt(theta["tau2"]) * philox.normals(obs, b, seed, philox.DOMAIN_NOISE)


def bootstrap_theta(grid, mask, theta_hat, B, N1, N2, seed, xatol=1e-4):
    """The extension Sec. 3.5 mentions: estimate the covariance parameters
    again on every simulated data set of the parametric bootstrap.  Draw b
    uses the y_b above; each is fitted from theta_hat by ``oracle.fit`` over
    (log range, log nugget ratio).  Returns (B, 2) estimates (range, eta)."""
    out = np.empty((B, 2))
    x0 = [np.log(theta_hat["range"]), np.log(theta_hat["tau2"] / theta_hat["sigma2"])]
    for b in range(B):
        yb = bootstrap_data(grid, mask, theta_hat, b, N1, N2, seed)
        rho, eta, _ = fit(grid, mask, yb, theta_hat, x0, xatol=xatol)
        out[b] = (rho, eta)
    return out
