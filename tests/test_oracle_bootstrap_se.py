"""Pins for the parametric bootstrap's data and refits (Sec. 3.5) and for the
standard error the stochastic trace estimate reports (Sec. 3.3).

Each check rests on something other than the oracle's own expressions: the
covariance of the simulated observations (Gaussian model of Sec. 2), the
optimality conditions of the refitted estimates, and the closed-form variance
of Hutchinson's estimator with Rademacher signs.
"""
import numpy as np

from oracle import bootstrap, dense, fit, lanczos, philox, sampler
from oracle.geometry import observed_cells
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta


def test_bootstrap_data_have_the_model_covariance():
    # y_b = A x_b + eps_b with x_b ~ N(0, sigma^2 Sigma) and eps_b ~ N(0, tau^2 I)
    # independent: over many draws, mean 0 and covariance sigma^2 Sigma_oo + tau^2 I.
    # Draws b and b + 1 must be independent (no stream reused across draws).
    n1, n2 = 5, 4
    g = grid(n1, n2)
    th = theta(0.3, 1.5, sigma2=1.3, tau2=0.3)
    mask = synth.uniform_mask(n1, n2, 0.3, seed=5)
    N1, N2 = sampler.psd_torus(g, th, 16, 16)
    B = 4000
    Y = np.array([bootstrap.bootstrap_data(g, mask, th, b, N1, N2, seed=91) for b in range(B)])
    p = Y.shape[1]
    K = th["sigma2"] * (dense.covariance(g, mask, dict(th, sigma2=1.0, tau2=0.0))) + th["tau2"] * np.eye(p)
    d = np.sqrt(np.diag(K))
    # entrywise standard error of a sample covariance: sqrt((K_ij^2 + K_ii K_jj) / B)
    se = np.sqrt((K ** 2 + np.outer(d, d) ** 2) / B)
    emp = Y.T @ Y / B
    assert np.max(np.abs(emp - K) / se) < 5.0
    assert np.max(np.abs(Y.mean(axis=0)) / (d / np.sqrt(B))) < 5.0
    cross = Y[:-1].T @ Y[1:] / (B - 1)
    assert np.max(np.abs(cross) / (np.outer(d, d) / np.sqrt(B - 1))) < 5.0
    # the noise variance (not its square root, not tau^4) sits on the diagonal
    # only: at zero correlation range the observations are white with
    # variance sigma^2 + tau^2
    th0 = theta(1e-6, 0.5, sigma2=1.3, tau2=0.3)
    Y0 = np.array([bootstrap.bootstrap_data(g, mask, th0, b, 16, 16, seed=92) for b in range(B)])
    v = Y0.var(axis=0)
    assert np.all(np.abs(v - 1.6) < 5 * 1.6 * np.sqrt(2.0 / B))


def test_bootstrap_theta_rows_are_the_refits_of_their_own_draws():
    # Each row b is (range, nugget ratio), in that order, maximising the exact
    # profile likelihood of draw b: stationary in (log range, log eta), better
    # than its four neighbours at +-0.1, and better on draw b than any other
    # row is (a refit of the wrong draw, or swapped columns, fails this).
    n1 = n2 = 12
    g = grid(n1, n2)
    # a smooth kernel, so that the nugget is identified and every optimum is
    # interior (with nu = 1/2 a short range can stand in for the nugget)
    th = theta(0.2, 1.5, sigma2=1.0, tau2=0.2)
    mask = synth.uniform_mask(n1, n2, 0.2, seed=6)
    N1, N2 = sampler.psd_torus(g, th, 32, 32)
    B = 3
    est = bootstrap.bootstrap_theta(g, mask, th, B, N1, N2, seed=33)
    assert est.shape == (B, 2)
    ys = [bootstrap.bootstrap_data(g, mask, th, b, N1, N2, seed=33) for b in range(B)]
    for b in range(B):
        f = lambda a, e, y=ys[b]: fit.profile_objective(g, mask, y, th, a, e)  # noqa: E731
        lr, le = np.log(est[b, 0]), np.log(est[b, 1])
        best = f(lr, le)
        h = 1e-3
        gr = (f(lr + h, le) - f(lr - h, le)) / (2 * h)
        ge = (f(lr, le + h) - f(lr, le - h)) / (2 * h)
        assert abs(gr) < 1e-2 and abs(ge) < 1e-2
        for dr, de in [(0.1, 0), (-0.1, 0), (0, 0.1), (0, -0.1)]:
            assert f(lr + dr, le + de) < best
        for o in range(B):
            if o != b:
                assert f(np.log(est[o, 0]), np.log(est[o, 1])) < best
        # swapped columns are not an optimum
        assert f(le, lr) < best
    # the draws differ, and so do their estimates
    assert len({tuple(np.round(r, 6)) for r in est}) == B


def _torus_problem(n=6, rho=0.25, eta=0.4):
    # all cells of an n x n torus observed, exponential correlation of the
    # wrapped distance plus a nugget: a block-circulant K, so every lattice
    # colour class (period dividing n) is a translate of every other
    ii, jj = np.divmod(np.arange(n * n), n)
    di = np.abs(ii[:, None] - ii[None, :])
    dj = np.abs(jj[:, None] - jj[None, :])
    di = np.minimum(di, n - di) / n
    dj = np.minimum(dj, n - dj) / n
    K = np.exp(-np.hypot(di, dj) / rho) + eta * np.eye(n * n)
    w, V = np.linalg.eigh(K)
    assert w.min() > 0
    return K, (V * np.log(w)) @ V.T, ii, jj


def test_rademacher_standard_error_matches_the_closed_form_variance():
    # z^T A z with Rademacher z has variance 2 sum_{i != j} A_ij^2, so with N
    # probes N * se^2 (se = sd / sqrt(N), sample sd) is unbiased for it, and
    # the estimates themselves spread by sqrt(that / N).
    K, A, ii, jj = _torus_problem()
    var1 = 2.0 * (np.sum(A * A) - np.sum(np.diag(A) ** 2))
    N, S = 10, 600
    ests, n_se2 = [], []
    for s in range(S):
        Z = philox.probe_matrix(ii, jj, N, seed=1000 + s)
        est, per = lanczos.exact_hutchinson(K, Z)
        e2, se = lanczos.combine(per, coloured=False)
        assert e2 == est
        ests.append(est)
        n_se2.append(N * se * se)
    # relative Monte-Carlo error of the mean of S * N squared deviations ~ sqrt(2 / (S (N - 1)))
    assert abs(np.mean(n_se2) / var1 - 1) < 0.1
    assert abs(np.var(ests, ddof=1) / (var1 / N) - 1) < 0.2
    # the mean itself is unbiased for tr log K
    tr = np.trace(A)
    assert abs(np.mean(ests) - tr) < 5 * np.sqrt(var1 / N / S)


def test_coloured_standard_error_matches_the_closed_form_variance():
    # Coloured probes: the estimate is the sum over the c^2 colour classes of
    # z_k^T A z_k, independent across classes, variance
    # sum_k 2 sum_{i != j in class k} A_ij^2.  On a torus the classes are
    # translates of each other, so the reported se^2 = N * sample variance is
    # unbiased for that.
    n, c = 6, 3
    K, A, ii, jj = _torus_problem(n)
    colour = (ii % c) + c * (jj % c)
    var_sum = 0.0
    for k in range(c * c):
        sub = A[np.ix_(colour == k, colour == k)]
        var_sum += 2.0 * (np.sum(sub * sub) - np.sum(np.diag(sub) ** 2))
    S = 800
    ests, se2 = [], []
    for s in range(S):
        Z = philox.probe_matrix(ii, jj, 0, seed=5000 + s, colour_period=c)
        est, per = lanczos.exact_hutchinson(K, Z, coloured=True)
        e2, se = lanczos.combine(per, coloured=True)
        assert e2 == est
        ests.append(est)
        se2.append(se * se)
    assert abs(np.mean(se2) / var_sum - 1) < 0.1
    assert abs(np.var(ests, ddof=1) / var_sum - 1) < 0.2
    assert abs(np.mean(ests) - np.trace(A)) < 5 * np.sqrt(var_sum / S)


def test_slq_standard_error_describes_the_spread_over_seeds():
    # The full route (Lanczos, Gauss quadrature, combine) on a 16 x 16 grid
    # with 30 % missing: over 200 probe seeds the estimates spread as the
    # reported standard errors say (within 20 %).
    n = 16
    g = grid(n, n)
    th = theta(0.1, 0.5, tau2=0.2)
    mask = synth.uniform_mask(n, n, 0.3, seed=2)
    K = dense.covariance(g, mask, th)
    r, c = observed_cells(mask)
    mv = lambda v: K @ v  # noqa: E731
    ests, ses = [], []
    for s in range(200):
        Z = philox.probe_matrix(r, c, 8, seed=700 + s)
        est, se, _, _ = lanczos.slq_logdet(mv, Z, m=25, reorth=True)
        ests.append(est)
        ses.append(se)
    ratio = np.std(ests, ddof=1) / np.sqrt(np.mean(np.square(ses)))
    assert 0.8 < ratio < 1.2
