"""Pins for the oracle's Lanczos quadrature, CG and genGK (Algorithm 1)."""
import numpy as np
import pytest

from oracle import cg as ocg
from oracle import dense, gengk, lanczos, philox
from oracle.geometry import observed_cells
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta


def _problem(n1=6, n2=6, th=None, frac=0.25, seed=1):
    th = th or theta(0.2, 1.5, tau2=0.1)
    g = grid(n1, n2)
    mask = synth.uniform_mask(n1, n2, frac, seed=seed)
    K = dense.covariance(g, mask, th)
    return g, mask, th, K


def test_slq_with_m_equal_p_is_exact_hutchinson():
    g, mask, th, K = _problem()
    p = K.shape[0]
    r, c = observed_cells(mask)
    Z = philox.probe_matrix(r, c, 6, seed=11)
    est, _, vals, steps = lanczos.slq_logdet(lambda v: K @ v, Z, m=p, reorth=True)
    ref, per = lanczos.exact_hutchinson(K, Z)
    np.testing.assert_allclose(vals, per, rtol=1e-10)
    assert est == pytest.approx(ref, rel=1e-10)


def test_slq_with_unit_probes_is_exact_logdet():
    g, mask, th, K = _problem(5, 5)
    p = K.shape[0]
    est, _, _, _ = lanczos.slq_logdet(lambda v: K @ v, np.eye(p), m=p, reorth=True, coloured=True)
    assert est == pytest.approx(np.linalg.slogdet(K)[1], rel=1e-10)
    # coloured probes whose period covers the grid are unit vectors up to sign
    r, c = observed_cells(mask)
    Z = philox.probe_matrix(r, c, 0, seed=3, colour_period=5)
    est2, _, _, _ = lanczos.slq_logdet(lambda v: K @ v, Z, m=p, reorth=True, coloured=True)
    assert est2 == pytest.approx(np.linalg.slogdet(K)[1], rel=1e-10)


def test_nugget_only_breaks_down_after_one_step_and_is_exact():
    eta = 0.25
    g, mask, th, K = _problem(th=theta(1e-6, 0.5, tau2=eta))
    p = K.shape[0]
    r, c = observed_cells(mask)
    Z = philox.probe_matrix(r, c, 4, seed=2)
    est, se, vals, steps = lanczos.slq_logdet(lambda v: K @ v, Z, m=20, reorth=False)
    assert np.all(steps == 1)
    np.testing.assert_allclose(vals, p * np.log1p(eta), rtol=1e-14)
    assert se == 0.0


def test_ritz_values_inside_spectrum():
    g, mask, th, K = _problem(th=theta(0.3, 2.5, tau2=0.05))
    w = np.linalg.eigvalsh(K)
    a, b = lanczos.lanczos(lambda v: K @ v, np.ones(K.shape[0]), 10, reorth=True)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    ev = np.linalg.eigvalsh(T)
    assert ev.min() >= w.min() - 1e-12 and ev.max() <= w.max() + 1e-12


def test_cg_matches_direct_solve():
    g, mask, th, K = _problem(8, 8, th=theta(0.1, 0.5, tau2=0.2))
    b = synth.random_vectors(K.shape[0], 1, seed=4)[0]
    x, it, rel = ocg.cg(lambda v: K @ v, b, rtol=1e-12)
    np.testing.assert_allclose(x, np.linalg.solve(K, b), rtol=1e-9, atol=1e-11)
    assert rel <= 1e-12 and it <= K.shape[0]


def _gk_setup(n1=5, n2=5, th=None, seed=3):
    th = th or theta(0.25, 0.5, sigma2=1.5, tau2=0.2)
    g = grid(n1, n2)
    mask = synth.uniform_mask(n1, n2, 0.3, seed=seed)
    S = dense.full_correlation(g, th)
    obs = np.flatnonzero(mask.ravel())
    A = np.zeros((obs.size, n1 * n2))
    A[np.arange(obs.size), obs] = 1.0
    b = synth.random_vectors(obs.size, 1, seed=seed + 1)[0]
    return g, mask, th, S, A, b


def test_gengk_invariants():
    g, mask, th, S, A, b = _gk_setup()
    k = 8
    beta1, U, V, B, al, be = gengk.gengk(A, S, b, th["tau2"], k, reorth=True)
    np.testing.assert_allclose(A @ S @ V, U @ B, atol=1e-12)
    np.testing.assert_allclose(U.T @ U, th["tau2"] * np.eye(k + 1), atol=1e-12)
    np.testing.assert_allclose(V.T @ S @ V, np.eye(k), atol=1e-12)


def test_gengk_full_steps_reproduce_dense_solution():
    g, mask, th, S, A, b = _gk_setup(th=theta(0.3, 1.5, sigma2=1.2, tau2=0.15))
    p = A.shape[0]
    x, J, z = gengk.gengk_solve(A, S, b, th["sigma2"], th["tau2"], k=p, reorth=True)
    # eq. act_xhat in its precision form
    P = np.linalg.inv(S) / th["sigma2"] + A.T @ A / th["tau2"]
    xhat = np.linalg.solve(P, A.T @ b / th["tau2"])
    np.testing.assert_allclose(x, xhat, rtol=1e-9, atol=1e-10)
    # minimum value = b^T (sigma^2 A Sigma A^T + tau^2 I)^-1 b
    Jref = b @ np.linalg.solve(th["sigma2"] * A @ S @ A.T + th["tau2"] * np.eye(p), b)
    assert J == pytest.approx(Jref, rel=1e-10)
    # the quadratic term x^T Sigma^-1 x equals ||z||^2
    assert z @ z == pytest.approx(xhat @ np.linalg.solve(S, xhat), rel=1e-8)
    # sigma^2 J is the marginal quadratic form y^T K^-1 y of the dense oracle
    out = dense.loglik(g, mask, th, b)
    assert th["sigma2"] * J == pytest.approx(out["quad"], rel=1e-10)


def test_adaptive_slq_stopping_rule():
    g, mask, th, K = _problem(8, 8)
    p = K.shape[0]
    r, c = observed_cells(mask)
    Z = philox.probe_matrix(r, c, 5, seed=21)
    mv = lambda v: K @ v  # noqa: E731
    hut, _ = lanczos.exact_hutchinson(K, Z)
    # a loose tolerance stops at the first check (10 steps), equal to m = 10
    est, _, vals, m = lanczos.slq_logdet_adaptive(mv, Z, max_steps=p, rtol=10.0)
    ref, _, rvals, _ = lanczos.slq_logdet(mv, Z, m=10, reorth=True)
    assert m == 10 and est == ref and np.array_equal(vals, rvals)
    # rtol = 0 stops only once every recurrence has ended: exact Hutchinson
    est0, _, _, m0 = lanczos.slq_logdet_adaptive(mv, Z, max_steps=p, rtol=0.0)
    assert est0 == pytest.approx(hut, rel=1e-10)
    # a tight tolerance converges well before p steps, close to the exact value
    est1, _, _, m1 = lanczos.slq_logdet_adaptive(mv, Z, max_steps=p, rtol=1e-9)
    assert m1 < p and abs(est1 - hut) <= 1e-7 * abs(hut)
    # a nugget-only covariance ends every recurrence after one step, before
    # any check: the steps run (one) are used, and the value is exact
    eta = 0.3
    _, _, _, Kn = _problem(8, 8, th=theta(1e-6, 0.5, tau2=eta))
    estn, _, _, mn = lanczos.slq_logdet_adaptive(lambda v: Kn @ v, Z, max_steps=40, rtol=1e-12)
    assert mn == 1 and estn == pytest.approx(p * np.log1p(eta), rel=1e-14)


def test_adaptive_check_schedule():
    # every 5 steps to 100, then 10, 15, 20, ... apart (5 floor(j / 50))
    got = lanczos.check_steps(260)
    want = list(range(5, 101, 5)) + [110, 120, 130, 140, 150, 165, 180, 195, 210, 230, 250]
    assert got == want
    assert lanczos.check_steps(4) == []
    # at the 1024-step cap: 46 checks instead of 204
    assert len(lanczos.check_steps(1024)) == 46
