"""GPU: degenerate and boundary cases of the likelihood path against closed
forms and the dense oracle -- one observation, the smallest grid, every cell
observed, a covariate count one below the observations, a zero nugget."""
import numpy as np
import pytest

from oracle import dense
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_2012_13133_amd.kryging")


@pytest.mark.parametrize("precision", [0, 1])
def test_one_observation_closed_form(precision):
    # K = 1 + eta: log det = log(1 + eta), Q = y^2 / (1 + eta); the Lanczos
    # recurrence breaks down after one step with the exact quadrature
    n1, n2 = 6, 5
    mask = np.zeros((n1, n2), dtype=np.uint8)
    mask[2, 3] = 1
    y = np.zeros((n1, n2))
    y[2, 3] = 1.7
    eta = 0.4
    th = K.theta(sigma2=2.0, tau2=2.0 * eta, range=0.2, nu=1.5)
    with K.Problem(n1, n2, mask, y) as P:
        r = K.kry_loglik(P.h, th, K.kry_opts_default(num_probes=3, precision=precision))
    # FP32 form: the product (1 + eta) v is rounded to FP32 before the FP64 coefficients
    tol = 1e-12 if precision == 0 else 1e-6
    assert r["p"] == 1 and r["lanczos_steps_used"] == 1
    assert r["logdet"] == pytest.approx(np.log1p(eta), rel=tol)
    assert r["quad"] == pytest.approx(1.7 ** 2 / (1 + eta), rel=1e-12 if precision == 0 else 1e-8)
    ll = -0.5 * (np.log(2 * np.pi * 2.0) + np.log1p(eta) + 1.7 ** 2 / (1 + eta) / 2.0)
    assert r["loglik"] == pytest.approx(ll, rel=tol)


def test_smallest_grid_fully_observed_matches_dense():
    n1 = n2 = 2
    g = grid(n1, n2)
    th = theta(0.7, 0.5, sigma2=1.3, tau2=0.2)
    mask = np.ones((2, 2), dtype=np.uint8)
    y = np.array([[0.3, -1.2], [0.8, 2.0]])
    ref = dense.loglik(g, mask, th, y.ravel())
    with K.Problem(n1, n2, mask, y) as P:
        # four probes of dimension four, four Lanczos steps: the quadrature is exact per probe
        r = K.kry_loglik(P.h, K.theta_from_dict(th), K.kry_opts_default(lanczos_steps=4, num_probes=4, reorth=1,
                                                                           cg_rtol=1e-12))
        mean, vx, _ = K.kry_krige(P.h, K.theta_from_dict(th), K.kry_opts_default(cg_rtol=1e-12), np.array([0, 3]))
    assert r["quad"] == pytest.approx(ref["quad"], rel=1e-10)
    Kd = dense.covariance(g, mask, th)
    from oracle import lanczos, philox
    from oracle.geometry import observed_cells
    rr, cc = observed_cells(mask)
    hut, _ = lanczos.exact_hutchinson(Kd, philox.probe_matrix(rr, cc, 4, 303))
    assert r["logdet"] == pytest.approx(hut, rel=1e-10)
    m_ref, v_ref, _ = dense.krige(g, mask, th, y.ravel(), np.array([0, 3]))
    np.testing.assert_allclose(mean, m_ref, rtol=1e-10)
    np.testing.assert_allclose(vx, v_ref, rtol=1e-9)


def test_covariates_one_below_the_observation_count():
    # q = p - 1: the REML contrast space is one-dimensional
    n1, n2 = 4, 3
    g = grid(n1, n2)
    th = theta(0.3, 0.5, sigma2=1.0, tau2=0.3)
    mask = synth.uniform_mask(n1, n2, 0.5, seed=3)  # 6 observed
    obs = np.flatnonzero(mask.ravel())
    q = obs.size - 1
    X = synth.covariates(n1, n2, q, seed=4).reshape(q, -1)
    y = synth.random_vectors(n1 * n2, 1, seed=5)[0]
    ref = dense.loglik_covariates(g, mask, th, y[obs], X[:, obs].T, reml=True)
    with K.Problem(n1, n2, mask, y) as P:
        K.kry_problem_set_covariates(P.h, X)
        r = K.kry_loglik(P.h, K.theta_from_dict(th), K.kry_opts_default(lanczos_steps=6, num_probes=4, reorth=1,
                                                                           cg_rtol=1e-12, reml=1))
    assert r["ncov"] == q
    assert r["quad"] == pytest.approx(ref["quad"], rel=1e-8)
    assert r["sigma2_hat"] == pytest.approx(ref["quad"] / 1.0, rel=1e-8)
    np.testing.assert_allclose(r["beta"], ref["beta"], rtol=1e-7, atol=1e-9)


def test_zero_nugget_quadratic_form():
    # eta = 0: K = Sigma_oo, still positive definite for the exponential kernel
    n1, n2 = 10, 9
    g = grid(n1, n2)
    th = theta(0.2, 0.5, sigma2=1.0, tau2=0.0)
    mask = synth.uniform_mask(n1, n2, 0.3, seed=6)
    obs = np.flatnonzero(mask.ravel())
    y = synth.random_vectors(n1 * n2, 1, seed=7)[0]
    ref = dense.loglik(g, mask, th, y[obs])
    with K.Problem(n1, n2, mask, y) as P:
        for prec in (0, 1):
            r = K.kry_loglik(P.h, K.theta_from_dict(th), K.kry_opts_default(precision=prec, cg_rtol=1e-11,
                                                                               lanczos_steps=10))
            assert r["quad"] == pytest.approx(ref["quad"], rel=1e-7), prec
