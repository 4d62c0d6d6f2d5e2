"""Pins for the covariate (GLS) part of the dense oracle: each pin uses a
route other than the GLS formulas themselves -- numerical maximisation over
beta of the zero-mean likelihood, ordinary least squares from numpy where K
is a multiple of I, scipy's normal density of the error contrasts, and
invariances a dropped term or a wrong sign breaks."""
import numpy as np
import pytest
from scipy import linalg, optimize, stats

from oracle import dense
from oracle.geometry import observed_cells
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta


def _case(n1=7, n2=6, q=3, seed=1, th=None):
    g = grid(n1, n2)
    th = th or theta(0.2, 1.5, sigma2=1.7, tau2=0.3, ratio=1.5, angle=0.4)
    mask = synth.uniform_mask(n1, n2, 0.3, seed=seed)
    obs = np.flatnonzero(mask.ravel())
    X = synth.covariates(n1, n2, q, seed=seed + 1).reshape(q, -1).T[obs]
    rng = np.random.default_rng(seed + 2)
    y = X @ rng.normal(3.0, 2.0, q) + synth.random_vectors(obs.size, 1, seed=seed + 3)[0]
    return g, th, mask, X, y


def test_gls_is_the_maximum_over_beta_of_the_zero_mean_likelihood():
    g, th, mask, X, y = _case()
    out = dense.loglik_covariates(g, mask, th, y, X)
    f = lambda b: -dense.loglik(g, mask, th, y - X @ b)["loglik"]
    res = optimize.minimize(f, np.zeros(X.shape[1]), method="BFGS", options=dict(gtol=1e-10))
    assert np.allclose(res.x, out["beta"], rtol=0, atol=1e-6)
    assert -res.fun == pytest.approx(out["loglik"], rel=1e-12)
    # and the profiled value is the maximum over sigma2 as well
    s2 = out["sigma2_hat"]
    th2 = dict(th, sigma2=s2, tau2=s2 * th["tau2"] / th["sigma2"])
    assert dense.loglik(g, mask, th2, y - X @ out["beta"])["loglik"] == pytest.approx(
        out["loglik_profiled"], rel=1e-12)


def test_shift_of_the_data_along_the_covariates():
    g, th, mask, X, y = _case(seed=5)
    b = np.array([40.0, -3.0, 7.5])
    a = dense.loglik_covariates(g, mask, th, y, X)
    s = dense.loglik_covariates(g, mask, th, y + X @ b, X)
    assert s["quad"] == pytest.approx(a["quad"], rel=1e-9)
    assert np.allclose(s["beta"] - b, a["beta"], rtol=0, atol=1e-9)
    for r in (False, True):
        assert dense.loglik_covariates(g, mask, th, y + X @ b, X, reml=r)["loglik_profiled"] == pytest.approx(
            dense.loglik_covariates(g, mask, th, y, X, reml=r)["loglik_profiled"], rel=1e-11)


def test_uncorrelated_case_is_ordinary_least_squares():
    # range far below the spacing: K = (1 + eta) I
    eta = 0.4
    g, th, mask, X, y = _case(seed=9, th=theta(1e-6, 0.5, sigma2=1.0, tau2=eta))
    out = dense.loglik_covariates(g, mask, th, y, X)
    b, rss, _, _ = np.linalg.lstsq(X, y, rcond=None)
    p = y.size
    assert np.allclose(out["beta"], b, rtol=1e-12, atol=1e-12)
    assert out["quad"] == pytest.approx(rss[0] / (1 + eta), rel=1e-12)
    se = np.sqrt(np.diag(out["sigma2_hat"] * (1 + eta) * np.linalg.inv(X.T @ X)))
    assert np.allclose(out["beta_se"], se, rtol=1e-12)
    assert out["logdet_xkx"] == pytest.approx(np.linalg.slogdet(X.T @ X)[1] - 3 * np.log1p(eta), rel=1e-12)


def test_reml_is_the_likelihood_of_error_contrasts():
    g, th, mask, X, y = _case(seed=13)
    out = dense.loglik_covariates(g, mask, th, y, X, reml=True)
    K = dense.covariance(g, mask, th)
    L = linalg.null_space(X.T).T  # orthonormal rows, L X = 0
    m = L.shape[0]
    assert m == y.size - X.shape[1]
    Ky = L @ K @ L.T
    ref = stats.multivariate_normal(mean=np.zeros(m), cov=th["sigma2"] * Ky).logpdf(L @ y)
    assert out["loglik"] == pytest.approx(ref, rel=1e-11)
    s2 = float((L @ y) @ np.linalg.solve(Ky, L @ y)) / m
    assert out["sigma2_hat"] == pytest.approx(s2, rel=1e-11)
    ref_p = stats.multivariate_normal(mean=np.zeros(m), cov=s2 * Ky).logpdf(L @ y)
    assert out["loglik_profiled"] == pytest.approx(ref_p, rel=1e-11)


def test_reparametrised_covariates():
    g, th, mask, X, y = _case(seed=17)
    M = np.array([[2.0, 0.3, -1.0], [0.0, 1.5, 0.2], [0.4, 0.0, 0.7]])
    for r in (False, True):
        a = dense.loglik_covariates(g, mask, th, y, X, reml=r)
        b = dense.loglik_covariates(g, mask, th, y, X @ M, reml=r)
        assert b["loglik"] == pytest.approx(a["loglik"], rel=1e-11)
        assert b["loglik_profiled"] == pytest.approx(a["loglik_profiled"], rel=1e-11)
        assert np.allclose(M @ b["beta"], a["beta"], rtol=0, atol=1e-9)


def test_no_covariates_is_the_zero_mean_model():
    g, th, mask, X, y = _case(seed=21)
    a = dense.loglik_covariates(g, mask, th, y, np.zeros((y.size, 0)))
    b = dense.loglik(g, mask, th, y)
    for k in ("loglik", "loglik_profiled", "quad", "logdet", "sigma2_hat"):
        assert a[k] == pytest.approx(b[k], rel=1e-14)


def test_kriging_reproduces_an_exact_mean_surface():
    n1, n2 = 8, 7
    g, th, mask, _, _ = _case(n1, n2, seed=25)
    Xall = synth.covariates(n1, n2, 3, seed=26).reshape(3, -1).T
    obs = np.flatnonzero(mask.ravel())
    tg = np.flatnonzero(mask.ravel() == 0)
    b = np.array([44.49, -2.0, 1.25])
    mean, _, _, beta = dense.krige_covariates(g, mask, th, Xall[obs] @ b, Xall[obs], Xall[tg], tg)
    assert np.allclose(beta, b, rtol=1e-12)
    assert np.allclose(mean, Xall[tg] @ b, rtol=1e-12)


def test_kriging_interpolates_observed_cells_without_nugget():
    # eta = 0: predicting an observed cell returns its datum, covariates or not
    n1, n2 = 8, 7
    th = theta(0.3, 0.5, sigma2=2.0, tau2=0.0)
    g, _, mask, X, y = _case(n1, n2, seed=29, th=th)
    obs = np.flatnonzero(mask.ravel())
    pick = obs[[0, 5, 17]]
    Xall = synth.covariates(n1, n2, 3, seed=30).reshape(3, -1).T
    mean, var_x, _, _ = dense.krige_covariates(g, mask, th, y, Xall[obs], Xall[pick], pick)
    assert np.allclose(mean, y[[0, 5, 17]], rtol=1e-9, atol=1e-9)
    assert np.allclose(var_x, 0.0, atol=1e-9)
