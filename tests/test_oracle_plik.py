"""Pins for the paper's own objective (oracle.plik), the range derivative of
the Matern correlation and the low-rank posterior variance: each against a
route other than the formula itself -- closed forms, finite differences, the
marginal likelihood (pinned to scipy elsewhere), a geometric series, the
dense posterior covariance and kriging variances."""
import numpy as np
import pytest

from oracle import dense, gengk, matern, plik, sampler
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta


def _case(n1=8, n2=7, th=None, frac=0.3, seed=1, q=0):
    g = grid(n1, n2)
    th = th or theta(0.25, 1.5, sigma2=1.7, tau2=0.3, ratio=1.5, angle=0.4)
    mask = synth.uniform_mask(n1, n2, frac, seed=seed)
    obs = np.flatnonzero(mask.ravel())
    _, y = sampler.cholesky_field(g, th, seed=seed + 1)
    yo = y.ravel()[obs]
    X = synth.covariates(n1, n2, q, seed=seed + 2).reshape(q, -1).T[obs] if q else None
    return g, th, mask, obs, yo, X


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_matern_range_derivative_closed_forms(nu):
    d = np.linspace(0.0, 0.7, 57)
    np.testing.assert_allclose(matern.matern_drange(d, 0.2, nu), matern.matern_drange_half_integer(d, 0.2, nu),
                               rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("nu", [0.7, 1.0, 1.5, 3.2])
def test_matern_range_derivative_finite_difference(nu):
    d = np.linspace(0.01, 0.6, 40)
    h = 1e-6
    fd = (matern.matern(d, 0.2 + h, nu) - matern.matern(d, 0.2 - h, nu)) / (2 * h)
    np.testing.assert_allclose(matern.matern_drange(d, 0.2, nu), fd, rtol=1e-7, atol=1e-10)


@pytest.mark.parametrize("q", [0, 2])
def test_exact_plik_is_the_marginal_likelihood_plus_the_dropped_terms(q):
    # x integrated out exactly: l_marginal = pl - 1/2 log det(Sigma^-1/sigma2 + A^T A/tau2) - (p/2) log 2 pi
    g, th, mask, obs, yo, X = _case(q=q)
    beta = np.array([1.5, -0.7])[:q]
    r = plik.exact_plik(g, mask, th, yo, X, beta)
    S = dense.full_correlation(g, th)
    A = np.zeros((obs.size, S.shape[0]))
    A[np.arange(obs.size), obs] = 1.0
    H = np.linalg.inv(S) / th["sigma2"] + A.T @ A / th["tau2"]
    b = yo - (X @ beta if q else 0.0)
    marg = dense.loglik(g, mask, th, b)["loglik"]
    want = marg + 0.5 * np.linalg.slogdet(H)[1] + 0.5 * obs.size * np.log(2 * np.pi)
    assert r["pl"] == pytest.approx(want, rel=1e-11)


def test_exact_gradient_matches_finite_differences():
    g, th, mask, obs, yo, X = _case(q=2)
    beta = np.array([0.4, -1.1])
    r = plik.exact_plik(g, mask, th, yo, X, beta)
    gr = r["grad"]

    def pl(**kw):
        t = dict(th)
        b = beta.copy()
        if "lam2" in kw:
            t["sigma2"] = 1.0 / kw["lam2"]
        if "lame2" in kw:
            t["tau2"] = 1.0 / kw["lame2"]
        if "rho" in kw:
            t["range"] = kw["rho"]
        if "beta" in kw:
            b = kw["beta"]
        return plik.exact_plik(g, mask, t, yo, X, b)["pl"]

    for key, x0 in (("lam2", 1 / th["sigma2"]), ("lame2", 1 / th["tau2"]), ("rho", th["range"])):
        h = 1e-5 * x0
        fd = (pl(**{key: x0 + h}) - pl(**{key: x0 - h})) / (2 * h)
        assert gr[key] == pytest.approx(fd, rel=1e-6, abs=1e-8), key
    for j in range(2):
        e = np.zeros(2)
        e[j] = 1e-5
        fd = (pl(beta=beta + e) - pl(beta=beta - e)) / 2e-5
        assert gr["beta"][j] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_quadrant_logdet_white_noise_and_ar1_geometric_series():
    # no correlation between distinct cells: every eigenvalue is 1
    g = grid(6, 5)
    assert plik.quadrant_logdet(g, theta(1e-6, 0.5)) == pytest.approx(0.0, abs=1e-12)
    # one row, exponential: c(l) = phi^|l|, the (2n-1)-point DFT at k < n is
    # 1 + 2 Re sum_{l=1}^{n-1} (phi w)^l, w = exp(-2 pi i k / (2n-1))
    n = 40
    g1 = (1, n, 1.0, 1.0 / n)
    th = theta(0.07, 0.5)
    phi = np.exp(-(1.0 / n) / 0.07)
    M = 2 * n - 1
    k = np.arange(n)
    a = phi * np.exp(-2j * np.pi * k / M)
    lam = 1.0 + 2.0 * np.real(a * (1 - a ** (n - 1)) / (1 - a))
    np.testing.assert_allclose(plik.quadrant_lambdas(g1, th)[0], lam, rtol=1e-12)
    assert plik.quadrant_logdet(g1, th) == pytest.approx(np.sum(np.log(lam)), rel=1e-12)


@pytest.mark.parametrize("th", [theta(0.2, 0.5), theta(0.15, 1.5, ratio=2.0, angle=0.5), theta(0.1, 1.0)])
def test_quadrant_dlogdet_is_the_range_derivative(th):
    g = grid(9, 11)
    h = 1e-6 * th["range"]
    fd = (plik.quadrant_logdet(g, dict(th, range=th["range"] + h)) -
          plik.quadrant_logdet(g, dict(th, range=th["range"] - h))) / (2 * h)
    assert plik.quadrant_dlogdet(g, th) == pytest.approx(fd, rel=1e-6)


def test_approx_plik_at_full_krylov_space_is_exact():
    # k = p: x_k* = x_hat, ||z||^2 = x_hat^T Sigma^-1 x_hat, and every genGK
    # term of the approximate gradient equals the exact one
    g, th, mask, obs, yo, X = _case(q=2, th=theta(0.25, 0.5, sigma2=1.3, tau2=0.4))
    beta = np.array([0.2, 0.9])
    ex = plik.exact_plik(g, mask, th, yo, X, beta)
    ap = plik.approx_plik(g, mask, th, yo, obs.size, X, beta)
    assert np.linalg.norm(ap["x"] - ex["x"]) <= 1e-9 * np.linalg.norm(ex["x"])
    assert ap["zz"] == pytest.approx(ex["quad_x"], rel=1e-9)
    assert ap["psi2"] == pytest.approx(float(ex["psi"] @ ex["psi"]), rel=1e-9)
    for key in ("lam2", "lame2"):
        assert ap["grad"][key] == pytest.approx(ex["grad"][key], rel=1e-8)
    # rho: the same up to the log-determinant term (quadrant vs exact trace)
    assert ap["grad"]["rho"] + 0.5 * ap["dL"] == pytest.approx(ex["grad"]["rho"] + 0.5 * ex["dL"], rel=1e-8)
    np.testing.assert_allclose(ap["grad"]["beta"], ex["grad"]["beta"], rtol=1e-8)
    # and the objective differs only by the log-determinant approximation
    assert ap["pl"] + 0.5 * ap["logdet"] == pytest.approx(ex["pl"] + 0.5 * ex["logdet"], rel=1e-10)


def test_trust_region_fit_finds_the_maximum_of_a_concave_function():
    a = np.array([0.3, -1.2, 2.0])
    M = np.array([[2.0, 0.3, 0.0], [0.3, 1.0, -0.2], [0.0, -0.2, 0.5]])

    def fg(x):
        d = x - a
        return -0.5 * d @ M @ d, -M @ d

    x, f, it = plik.trust_region_fit(fg, np.zeros(3), gtol=1e-9, maxiter=5000)
    assert np.linalg.norm(x - a) <= 1e-6 and it < 5000


def test_trust_region_fit_on_a_likelihood_with_a_closed_form_maximum():
    # the marginal log-likelihood in log sigma2 (everything else fixed) is
    # largest at sigma2_hat = Q / p
    g, th, mask, obs, yo, _ = _case(n1=10, n2=10, th=theta(0.2, 0.5, sigma2=1.0, tau2=0.2))
    ref = dense.loglik(g, mask, th, yo)
    eta = th["tau2"] / th["sigma2"]

    def fg(x):
        s2 = float(np.exp(x[0]))
        r = dense.loglik(g, mask, dict(th, sigma2=s2, tau2=eta * s2), yo)
        return r["loglik"], np.array([-0.5 * obs.size + 0.5 * r["quad"] / s2])

    x, f, it = plik.trust_region_fit(fg, np.log([5.0]), gtol=1e-9, maxiter=5000)
    assert float(np.exp(x[0])) == pytest.approx(ref["sigma2_hat"], rel=1e-7)
    assert f == pytest.approx(ref["loglik_profiled"], rel=1e-12)


def test_exact_plik_has_no_interior_maximum_in_the_range():
    # a property of the paper's objective (not of the code): with the
    # variances fixed, -1/2 log det Sigma(rho) grows without bound as Sigma
    # approaches a rank-one matrix, so pl keeps increasing with the range
    g, th, mask, obs, yo, _ = _case(n1=10, n2=10, th=theta(0.2, 0.5, sigma2=1.0, tau2=0.2))
    vals = [plik.exact_plik(g, mask, dict(th, range=r), yo)["pl"] for r in (0.1, 0.3, 1.0, 3.0)]
    assert np.all(np.diff(vals) > 0)


def test_low_rank_posterior_variance_exact_at_full_rank_and_decreasing():
    g, th, mask, obs, yo, _ = _case(n1=8, n2=8, th=theta(0.2, 1.5, sigma2=1.7, tau2=0.3))
    S = dense.full_correlation(g, th)
    A = np.zeros((obs.size, S.shape[0]))
    A[np.arange(obs.size), obs] = 1.0
    # exact: the kriging variance at every cell (Woodbury route)
    _, vx, _ = dense.krige(g, mask, th, yo, np.arange(64))
    full = gengk.posterior_variance(A, S, yo, th["sigma2"], th["tau2"], obs.size)
    np.testing.assert_allclose(full, vx, rtol=1e-9, atol=1e-12)
    prev = None
    for k in (3, 8, 16, 30):
        v = gengk.posterior_variance(A, S, yo, th["sigma2"], th["tau2"], k)
        assert np.all(v >= vx - 1e-10)  # never below the exact variance
        if prev is not None:
            assert np.all(v <= prev + 1e-10)  # a larger Krylov space only lowers it
        prev = v
