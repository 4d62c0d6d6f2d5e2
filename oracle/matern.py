"""Matern correlation and the anisotropic lag distance.

Test infrastructure only (see ``oracle/__init__``).

Sec. 2 (Latent Gaussian Model) defines the correlation between two sites at
Euclidean distance d as

    Sigma_ij = 2^(1-nu) / Gamma(nu) * (sqrt(2 nu) d / rho)^nu * K_nu(sqrt(2 nu) d / rho)

with K_nu the modified Bessel function of the second kind, range rho and
smoothness nu.  The same section allows a geometrically anisotropic
covariance (stretching along axes).  The rotated form used here (reading):
with u = (cos phi, sin phi) in (x = column, y = row) coordinates, the
distance is d = sqrt((h.u)^2 + (r * h.u_perp)^2), r >= 1; rho is the range
along u and rho / r across it.  r = 1 is the isotropic case.
"""
import numpy as np
from scipy.special import gamma as _gamma, kv as _kv


def matern(d, rho, nu):
    """Matern correlation at distances d (array, >= 0), range rho, smoothness nu.

    Written straight from the Sec. 2 formula with scipy's K_nu; the value at
    d = 0 is the limit 1.
    """
    d = np.asarray(d, dtype=np.float64)
    x = np.sqrt(2.0 * nu) * d / rho
    out = np.ones_like(x)
    pos = x > 0
    xp = x[pos]
    with np.errstate(under="ignore", invalid="ignore"):
        val = 2.0 ** (1.0 - nu) / _gamma(nu) * xp ** nu * _kv(nu, xp)
    val = np.where(np.isfinite(val), val, 0.0)
    out[pos] = val
    return out


def matern_half_integer(d, rho, nu):
    """Closed forms of the Matern correlation for nu = 1/2, 3/2, 5/2.

    These follow from the elementary form of K_{m+1/2}; they are a pin for
    ``matern`` (not used by it).
    """
    d = np.asarray(d, dtype=np.float64)
    if nu == 0.5:
        return np.exp(-d / rho)
    if nu == 1.5:
        t = np.sqrt(3.0) * d / rho
        return (1.0 + t) * np.exp(-t)
    if nu == 2.5:
        t = np.sqrt(5.0) * d / rho
        return (1.0 + t + t * t / 3.0) * np.exp(-t)
    raise ValueError("closed form only for nu in {0.5, 1.5, 2.5}")


def matern_drange(d, rho, nu):
    """Derivative of the Matern correlation with respect to the range rho
    (the d Sigma(rho) of the appendix's gradient).  With x = sqrt(2 nu) d / rho,
    d/dx [x^nu K_nu(x)] = -x^nu K_{nu-1}(x) (DLMF 10.29.4) and dx/drho = -x/rho,
    so  dM/drho = 2^(1-nu) / Gamma(nu) * x^(nu+1) K_{nu-1}(x) / rho,  0 at d = 0."""
    d = np.asarray(d, dtype=np.float64)
    x = np.sqrt(2.0 * nu) * d / rho
    out = np.zeros_like(x)
    pos = x > 0
    xp = x[pos]
    with np.errstate(under="ignore", invalid="ignore", over="ignore"):
        val = 2.0 ** (1.0 - nu) / _gamma(nu) * xp ** (nu + 1.0) * _kv(nu - 1.0, xp) / rho
    out[pos] = np.where(np.isfinite(val), val, 0.0)
    return out


def matern_drange_half_integer(d, rho, nu):
    """Closed forms of d/drho of the Matern correlation for nu = 1/2, 3/2,
    5/2, by differentiating ``matern_half_integer`` (a pin for
    ``matern_drange``)."""
    d = np.asarray(d, dtype=np.float64)
    if nu == 0.5:
        t = d / rho
        return t * np.exp(-t) / rho
    if nu == 1.5:
        u = np.sqrt(3.0) * d / rho
        return u * u * np.exp(-u) / rho
    if nu == 2.5:
        u = np.sqrt(5.0) * d / rho
        return u * u * (1.0 + u) * np.exp(-u) / (3.0 * rho)
    raise ValueError("closed form only for nu in {0.5, 1.5, 2.5}")


def aniso_distance(dx, dy, ratio=1.0, angle=0.0):
    """Distance of displacement (dx along columns, dy along rows) under the
    rotated geometric anisotropy (reading of the Sec. 2 remark): components
    along u = (cos angle, sin angle) and, scaled by ``ratio``, across it."""
    dx = np.asarray(dx, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    ca, sa = np.cos(angle), np.sin(angle)
    a = dx * ca + dy * sa
    b = -dx * sa + dy * ca
    return np.sqrt(a * a + (ratio * b) ** 2)


def correlation(dx, dy, theta, drange=False):
    """Unit-variance Matern correlation for displacement (dx, dy) given a
    parameter dict with keys range, nu, aniso_ratio, aniso_angle (its
    derivative with respect to the range when drange)."""
    d = aniso_distance(dx, dy, theta.get("aniso_ratio", 1.0), theta.get("aniso_angle", 0.0))
    return (matern_drange if drange else matern)(d, theta["range"], theta["nu"])
