"""Pins for the dense log-likelihood and kriging oracle."""
import numpy as np
import pytest
from scipy import stats

from oracle import dense
from oracle.geometry import observed_cells
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta


def test_loglik_matches_scipy_multivariate_normal():
    g = grid(7, 6)
    th = theta(0.2, 1.5, sigma2=1.7, tau2=0.3, ratio=1.5, angle=0.4)
    mask = synth.uniform_mask(7, 6, 0.3, seed=1)
    y = synth.random_vectors(int(mask.sum()), 1, seed=2)[0]
    out = dense.loglik(g, mask, th, y)
    K = dense.covariance(g, mask, th)
    ref = stats.multivariate_normal(mean=np.zeros(K.shape[0]), cov=th["sigma2"] * K).logpdf(y)
    assert abs(out["loglik"] - ref) < 1e-10 * abs(ref)
    # the profiled value is l at sigma2_hat = Q / p, and it is the maximum over sigma2
    th2 = dict(th, sigma2=out["sigma2_hat"], tau2=out["sigma2_hat"] * th["tau2"] / th["sigma2"])
    ref2 = stats.multivariate_normal(mean=np.zeros(K.shape[0]), cov=out["sigma2_hat"] * K).logpdf(y)
    assert abs(out["loglik_profiled"] - ref2) < 1e-10 * abs(ref2)
    for f in (0.9, 1.1):
        s = f * out["sigma2_hat"]
        assert stats.multivariate_normal(mean=np.zeros(K.shape[0]), cov=s * K).logpdf(y) < ref2
    assert dense.loglik(g, mask, th2, y)["loglik_profiled"] == pytest.approx(out["loglik_profiled"], rel=1e-12)


def test_nugget_only_closed_form():
    g = grid(5, 5)
    eta = 0.37
    th = theta(1e-6, 0.5, sigma2=1.0, tau2=eta)
    mask = synth.uniform_mask(5, 5, 0.2, seed=3)
    p = int(mask.sum())
    y = synth.random_vectors(p, 1, seed=4)[0]
    out = dense.loglik(g, mask, th, y)
    assert out["logdet"] == pytest.approx(p * np.log1p(eta), rel=1e-14)
    assert out["quad"] == pytest.approx(y @ y / (1 + eta), rel=1e-14)


def test_ar1_closed_form_logdet_and_quadratic():
    n = 30
    rho = 0.2
    g = grid(1, n)
    th = theta(rho, 0.5, sigma2=1.0, tau2=0.0)
    phi = np.exp(-(1.0 / n) / rho)
    y = synth.random_vectors(n, 1, seed=5)[0]
    out = dense.loglik(g, np.ones((1, n)), th, y)
    assert out["logdet"] == pytest.approx((n - 1) * np.log(1 - phi ** 2), rel=1e-12)
    q = y[0] ** 2 + np.sum((y[1:] - phi * y[:-1]) ** 2) / (1 - phi ** 2)
    assert out["quad"] == pytest.approx(q, rel=1e-12)


def _precision_form(g, mask, th, y):
    """Posterior mean/variance through eq. act_xhat's precision form
    (Sigma^-1/sigma^2 + A^T A / tau^2)^-1, a different route from K^-1."""
    n1, n2 = g[0], g[1]
    S = dense.full_correlation(g, th)
    obs = np.flatnonzero(mask.ravel())
    A = np.zeros((obs.size, n1 * n2))
    A[np.arange(obs.size), obs] = 1.0
    P = np.linalg.inv(S) / th["sigma2"] + A.T @ A / th["tau2"]
    G = np.linalg.inv(P)
    return G @ (A.T @ y) / th["tau2"], np.diag(G)


@pytest.mark.parametrize("th", [theta(0.15, 0.5, sigma2=1.3, tau2=0.2),
                                theta(0.3, 1.5, sigma2=0.8, tau2=0.05, ratio=2.0, angle=0.5)])
def test_kriging_matches_precision_form(th):
    g = grid(6, 6)
    mask = synth.uniform_mask(6, 6, 0.3, seed=6)
    y = synth.random_vectors(int(mask.sum()), 1, seed=7)[0]
    targets = np.arange(36)
    mean, vx, vy = dense.krige(g, mask, th, y, targets)
    mref, vref = _precision_form(g, mask, th, y)
    np.testing.assert_allclose(mean, mref, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(vx, vref, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(vy, vref + th["tau2"], rtol=1e-9)
    np.testing.assert_allclose(dense.posterior_mean_all(g, mask, th, y), mref, rtol=1e-9, atol=1e-10)


def test_kriging_limits():
    g = grid(8, 8)
    mask = synth.uniform_mask(8, 8, 0.3, seed=9)
    y = synth.random_vectors(int(mask.sum()), 1, seed=10)[0]
    r, c = observed_cells(mask)
    # tiny nugget: prediction at an observed cell reproduces the datum, variance -> 0
    th = theta(0.2, 1.5, sigma2=1.0, tau2=1e-10)
    ids = r[:5] * 8 + c[:5]
    mean, vx, _ = dense.krige(g, mask, th, y, ids)
    np.testing.assert_allclose(mean, y[:5], atol=1e-6)
    assert np.all(np.abs(vx) < 1e-6)
    # range far below the spacing: no information at a missing cell
    th = theta(1e-4, 0.5, sigma2=2.0, tau2=0.1)
    miss = np.flatnonzero(mask.ravel() == 0)[:5]
    mean, vx, vy = dense.krige(g, mask, th, y, miss)
    np.testing.assert_allclose(mean, 0.0, atol=1e-30)
    np.testing.assert_allclose(vx, 2.0, rtol=1e-15)
    np.testing.assert_allclose(vy, 2.1, rtol=1e-15)
