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
