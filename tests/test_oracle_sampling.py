"""Pins for the samplers, the parametric bootstrap and the profile fit."""
import numpy as np
import pytest

from oracle import bootstrap, dense, fit, sampler
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta


def test_circulant_sampler_covariance_is_exact():
    # The sampler is linear in the white noise: x = L xi.  L L^T must equal
    # sigma^2 Sigma on the grid (brute force over unit noise vectors).
    n1, n2, N1, N2 = 4, 5, 16, 16
    g = grid(n1, n2)
    th = theta(0.2, 1.5, sigma2=2.0, ratio=1.5, angle=0.6)
    lam = sampler.torus_spectrum(g, th, N1, N2)
    assert lam.min() > -1e-10 * lam.max()
    lam = np.maximum(lam, 0)
    cols = []
    for e in range(N1 * N2):
        xi = np.zeros(N1 * N2)
        xi[e] = 1.0
        cols.append(sampler.circulant_sqrt_apply(lam, xi.reshape(N1, N2))[:n1, :n2].ravel())
    L = np.sqrt(th["sigma2"]) * np.array(cols).T
    np.testing.assert_allclose(L @ L.T, th["sigma2"] * dense.full_correlation(g, th), atol=1e-12)


def test_circulant_field_reports_non_psd():
    g = grid(16, 16)
    th = theta(0.5, 2.5)
    with pytest.raises(ValueError):
        sampler.circulant_field(g, th, 32, 32, seed=1)


def test_cholesky_field_empirical_covariance():
    g = grid(3, 3)
    th = theta(0.4, 0.5, sigma2=1.5, tau2=0.2)
    xs, ys = [], []
    for s in range(3000):
        x, y = sampler.cholesky_field(g, th, seed=77, stream=s)
        xs.append(x.ravel())
        ys.append(y.ravel())
    xs, ys = np.array(xs), np.array(ys)
    S = th["sigma2"] * dense.full_correlation(g, th)
    # 3000 draws: entrywise standard error about sqrt(2/3000) * 1.5 ~ 0.04
    np.testing.assert_allclose(np.cov(xs.T), S, atol=0.15)
    np.testing.assert_allclose(np.cov(ys.T), S + th["tau2"] * np.eye(9), atol=0.15)


def test_bootstrap_variance_is_unbiased_for_kriging_variance():
    n1 = n2 = 8
    g = grid(n1, n2)
    th = theta(0.15, 0.5, sigma2=1.0, tau2=0.1)
    mask = synth.uniform_mask(n1, n2, 0.3, seed=4)
    targets = np.flatnonzero(mask.ravel() == 0)
    B = 60
    vx, vy = bootstrap.bootstrap_variance(g, mask, th, targets, B, 32, 32, seed=21)
    y0 = np.zeros(int(mask.sum()))
    _, ex, ey = dense.krige(g, mask, th, y0, targets)
    # each bootstrap value is ex * chi2_B / B; the mean ratio over T targets
    # has standard deviation about sqrt(2 / (B T)) (targets correlated: loosen)
    T = targets.size
    tol = 4 * np.sqrt(2.0 / B) / np.sqrt(T) * 3
    assert abs(np.mean(vx / ex) - 1) < tol
    assert abs(np.mean(vy / ey) - 1) < tol


def test_profile_fit_is_stationary_and_beats_neighbours():
    n1 = n2 = 12
    g = grid(n1, n2)
    th = theta(0.15, 0.5, sigma2=1.0, tau2=0.5)
    x, y = sampler.cholesky_field(g, th, seed=8)
    mask = synth.uniform_mask(n1, n2, 0.2, seed=6)
    yo = y.ravel()[mask.ravel().astype(bool)]
    rho, eta, best = fit.fit(g, mask, yo, th, x0=[np.log(0.1), np.log(0.2)])
    f = lambda a, b: fit.profile_objective(g, mask, yo, th, a, b)
    lr, le = np.log(rho), np.log(eta)
    h = 1e-3
    gr = (f(lr + h, le) - f(lr - h, le)) / (2 * h)
    ge = (f(lr, le + h) - f(lr, le - h)) / (2 * h)
    assert abs(gr) < 1e-2 and abs(ge) < 1e-2
    for dr, de in [(0.1, 0), (-0.1, 0), (0, 0.1), (0, -0.1)]:
        assert f(lr + dr, le + de) < best


def test_psd_torus_doubles_until_psd():
    g = grid(16, 16)
    th = theta(0.5, 2.5)
    N = sampler.psd_torus(g, th, 32, 32, cap=1024)
    assert N is not None and N[0] > 32
    lam = sampler.torus_spectrum(g, th, *N)
    assert lam.min() >= -1e-10 * lam.max()
    half = sampler.torus_spectrum(g, th, N[0] // 2, N[1] // 2)
    assert half.min() < -1e-10 * half.max()


def test_bootstrap_data_are_the_variance_bootstraps_draws():
    # the parameter bootstrap refits exactly the data sets the prediction
    # variance bootstrap simulates (same fields and noise): checked by
    # rebuilding draw b from the sampler and the Philox normals directly
    from oracle import bootstrap, philox, sampler
    from paper_2012_13133_amd import synth
    n1, n2 = 10, 9
    g = (n1, n2, 1.0 / n1, 1.0 / n2)
    th = dict(range=0.2, nu=0.5, sigma2=1.3, tau2=0.2, aniso_ratio=1.0, aniso_angle=0.0)
    mask = synth.uniform_mask(n1, n2, 0.25, seed=3)
    obs = np.flatnonzero(mask.ravel())
    N1, N2 = sampler.psd_torus(g, th, 32, 32)
    for b in (0, 3):
        x, _ = sampler.circulant_field(g, th, N1, N2, seed=17, stream=b)
        ref = x.ravel()[obs] + np.sqrt(0.2) * philox.normals(obs, b, 17, philox.DOMAIN_NOISE)
        np.testing.assert_array_equal(bootstrap.bootstrap_data(g, mask, th, b, N1, N2, 17), ref)
