"""GPU parity: Lanczos, quadrature, SLQ log-determinant, likelihood, CG,
genGK, kriging, sampling, bootstrap, fit and the batched form."""
import numpy as np
import pytest

from oracle import bootstrap, dense, direct, fit, gengk, lanczos, philox, sampler
from oracle.geometry import observed_cells
from paper_2012_13133_amd import synth
from tests.gpu_util import normwise, rows_rel
from tests.oracle_cases import grid, theta

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_2012_13133_amd.kryging")

CONFIG1 = theta(0.1, 0.5, sigma2=1.0, tau2=0.1)


def _problem(n1, n2, th, frac=0.3, seed=1, data_seed=202, cholesky=True):
    g = grid(n1, n2)
    mask = synth.uniform_mask(n1, n2, frac, seed=seed) if frac > 0 else np.ones((n1, n2), dtype=np.uint8)
    if cholesky:
        _, y = sampler.cholesky_field(g, th, seed=data_seed)
    else:
        y = synth.random_vectors(n1 * n2, 1, seed=data_seed)[0].reshape(n1, n2)
    yo = y.ravel()[mask.ravel().astype(bool)]
    return g, mask, y, yo


@pytest.mark.parametrize("reorth", [0, 1])
@pytest.mark.parametrize("case", [(32, 32, 0.0, CONFIG1), (20, 24, 0.3, theta(0.15, 1.5, tau2=0.2, ratio=2, angle=0.5))])
def test_lanczos_coefficients_match_oracle(reorth, case):
    n1, n2, frac, th = case
    g, mask, y, yo = _problem(n1, n2, th, frac)
    Kd = dense.covariance(g, mask, th)
    m = 30
    opts = K.kry_opts_default(lanczos_steps=m, num_probes=4, seed=77, reorth=reorth)
    with K.Problem(n1, n2, mask, y) as P:
        a, b, s = K.kry_lanczos(P.h, K.theta_from_dict(th), opts)
    r, c = observed_cells(mask)
    Z = philox.probe_matrix(r, c, 4, 77)
    rng = np.random.default_rng(0)
    w = np.linalg.eigvalsh(Kd)
    for k in range(4):
        ra, rb = lanczos.lanczos(lambda v: Kd @ v, Z[:, k], m, reorth=bool(reorth))
        assert s[k] == len(ra)
        # Once Ritz values converge the coefficients are ill-conditioned: a
        # rounding-level perturbation of the oracle's own products moves them
        # by O(1).  Compare element-wise on the prefix the oracle shows to be
        # stable, and the spectrum of T over all steps.
        pa, _ = lanczos.lanczos(lambda v: Kd @ v * (1 + 1e-15 * rng.standard_normal(v.size)), Z[:, k], m,
                                reorth=bool(reorth))
        unstable = np.flatnonzero(np.abs(pa - ra) > 1e-10 * np.abs(ra))
        stable = int(unstable[0]) if unstable.size else len(ra)
        assert stable >= 12
        np.testing.assert_allclose(a[k, :stable], ra[:stable], rtol=1e-9)
        np.testing.assert_allclose(b[k, : stable - 1], rb[: stable - 1], rtol=1e-9)
        T = np.diag(a[k, : s[k]]) + np.diag(b[k, : s[k] - 1], 1) + np.diag(b[k, : s[k] - 1], -1)
        ev = np.linalg.eigvalsh(T)
        assert ev.min() >= w.min() * (1 - 1e-9) and ev.max() <= w.max() * (1 + 1e-9)
        # extreme Ritz values converge first and are well conditioned
        Tr = np.diag(ra) + np.diag(rb, 1) + np.diag(rb, -1)
        assert abs(ev.max() - np.linalg.eigvalsh(Tr).max()) <= 1e-9 * w.max()


def test_gauss_quadrature_matches_oracle():
    rng = np.random.default_rng(3)
    nprobe, m = 6, 40
    steps = np.array([40, 1, 17, 40, 0, 5], dtype=np.int32)
    alpha = rng.uniform(1.0, 5.0, size=(nprobe, m))
    beta = rng.uniform(0.05, 0.9, size=(nprobe, m))
    zn = rng.uniform(10, 100, size=nprobe)
    got = K.kry_gauss_quadrature(alpha, beta, steps, zn)
    for k in range(nprobe):
        s = steps[k]
        ref = 0.0 if s == 0 else lanczos.quadrature(alpha[k, :s], beta[k, : s - 1], zn[k])
        assert abs(got[k] - ref) <= 1e-12 * max(abs(ref), 1.0)


def test_gauss_quadrature_at_the_step_cap():
    # tridiagonals of up to the 1024-step cap (the adaptive rule's ceiling),
    # with a ragged mix of lengths across 70 probes (more than one wavefront)
    rng = np.random.default_rng(4)
    nprobe, m = 70, 1024
    steps = rng.integers(1, m + 1, size=nprobe).astype(np.int32)
    steps[:3] = [m, m - 1, 1]
    alpha = rng.uniform(2.0, 5.0, size=(nprobe, m))  # diagonally dominant: positive definite
    beta = rng.uniform(0.05, 0.9, size=(nprobe, m))
    zn = rng.uniform(10, 100, size=nprobe)
    got = K.kry_gauss_quadrature(alpha, beta, steps, zn)
    for k in range(nprobe):
        s = steps[k]
        ref = lanczos.quadrature(alpha[k, :s], beta[k, : s - 1], zn[k])
        assert abs(got[k] - ref) <= 1e-11 * max(abs(ref), 1.0), (k, s, got[k], ref)


def test_slq_logdet_matches_oracle_and_exact_hutchinson():
    g, mask, y, yo = _problem(32, 32, CONFIG1, 0.0)
    Kd = dense.covariance(g, mask, CONFIG1)
    r, c = observed_cells(mask)
    opts = K.kry_opts_default(lanczos_steps=50, num_probes=10, seed=303)
    with K.Problem(32, 32, mask, y) as P:
        ld, se, per = K.kry_logdet(P.h, K.theta_from_dict(CONFIG1), opts)
    Z = philox.probe_matrix(r, c, 10, 303)
    est, ose, vals, _ = lanczos.slq_logdet(lambda v: Kd @ v, Z, 50, reorth=False)
    np.testing.assert_allclose(per, vals, rtol=1e-9)
    assert abs(ld - est) <= 1e-9 * abs(est) and abs(se - ose) <= 1e-6 * ose
    hut, _ = lanczos.exact_hutchinson(Kd, Z)
    assert abs(ld - hut) <= 1e-6 * abs(hut)


def test_slq_exact_when_m_equals_p_and_nugget_only():
    n1, n2 = 8, 8
    th = theta(0.2, 1.5, tau2=0.1)
    g, mask, y, yo = _problem(n1, n2, th, 0.25)
    Kd = dense.covariance(g, mask, th)
    p = Kd.shape[0]
    r, c = observed_cells(mask)
    opts = K.kry_opts_default(lanczos_steps=p, num_probes=3, seed=5, reorth=1)
    with K.Problem(n1, n2, mask, y) as P:
        ld, _, per = K.kry_logdet(P.h, K.theta_from_dict(th), opts)
        # nugget only: range far below the spacing
        th0 = theta(1e-6, 0.5, tau2=0.37)
        ld0, se0, per0 = K.kry_logdet(P.h, K.theta_from_dict(th0), K.kry_opts_default(lanczos_steps=20, num_probes=4))
        _, _, s0 = K.kry_lanczos(P.h, K.theta_from_dict(th0), K.kry_opts_default(lanczos_steps=20, num_probes=4))
    hut, hper = lanczos.exact_hutchinson(Kd, philox.probe_matrix(r, c, 3, 5))
    np.testing.assert_allclose(per, hper, rtol=1e-10)
    np.testing.assert_allclose(per0, p * np.log1p(0.37), rtol=1e-13)
    assert np.all(s0 == 1) and se0 <= 1e-13 * abs(ld0)


def _config1_loglik_case():
    g, mask, y, yo = _problem(32, 32, CONFIG1, 0.0)
    return g, mask, y, dense.loglik(g, mask, CONFIG1, yo)


@pytest.mark.parametrize("precision", [0, 1])
def test_config1_loglik_within_1e3_of_dense(precision):
    g, mask, y, ref = _config1_loglik_case()
    opts = K.kry_opts_default(lanczos_steps=30, probe_kind=K.KRY_PROBE_COLOURED, colour_period=6,
                              precision=precision)
    with K.Problem(32, 32, mask, y) as P:
        r = K.kry_loglik(P.h, K.theta_from_dict(CONFIG1), opts)
        plain = K.kry_loglik(P.h, K.theta_from_dict(CONFIG1), K.kry_opts_default(precision=precision))
    assert abs(r["loglik"] - ref["loglik"]) <= 1e-3 * abs(ref["loglik"])
    assert abs(r["loglik_profiled"] - ref["loglik_profiled"]) <= 1e-3 * abs(ref["loglik_profiled"])
    assert abs(r["quad"] - ref["quad"]) <= 1e-7 * ref["quad"]
    assert r["p"] == 1024 and r["cg_relres"] <= 1e-8
    # the literal 10-Rademacher-probe run: error within 4 reported standard errors
    assert abs(plain["logdet"] - ref["logdet"]) <= 4 * plain["logdet_se"] + 1e-9


def test_cg_solve_fp64_and_mixed():
    n1, n2 = 40, 40
    th = theta(0.05, 1.5, tau2=0.2)
    g, mask, y, yo = _problem(n1, n2, th, 0.3, cholesky=False)
    Kd = dense.covariance(g, mask, th)
    B = synth.random_vectors(Kd.shape[0], 3, seed=8)
    ref = np.linalg.solve(Kd, B.T).T
    with K.Problem(n1, n2, mask, y) as P:
        for prec in (0, 1):
            x, it, rr = K.kry_solve(P.h, K.theta_from_dict(th), K.kry_opts_default(precision=prec, cg_rtol=1e-10), B)
            true_res = max(normwise(Kd @ x[i], B[i]) for i in range(3))
            assert true_res <= 2e-10, (prec, true_res)
            assert rows_rel(x, ref) <= 1e-8


def test_mixed_refinement_reports_the_residual_of_the_returned_solution():
    # a tolerance below the FP64 rounding floor keeps the refinement running
    # to its cap of corrections: the residual reported must still be the one
    # of the X returned, b - K x with the library's own FP64 product
    n1, n2 = 24, 24
    th = theta(0.1, 1.5, tau2=0.05)
    g, mask, y, yo = _problem(n1, n2, th, 0.3, cholesky=False)
    with K.Problem(n1, n2, mask, y) as P:
        B = synth.random_vectors(P.p, 3, seed=9)
        t = K.theta_from_dict(th)
        x, it, rr = K.kry_solve(P.h, t, K.kry_opts_default(precision=1, cg_rtol=1e-300), B, allow_noconv=True)
        kx = K.kry_matvec(P.h, t, x, K.KRY_FP64)
        for i in range(3):
            true = np.linalg.norm(B[i] - kx[i]) / np.linalg.norm(B[i])
            assert rr[i] == pytest.approx(true, rel=1e-6), (i, rr[i], true)
            assert rr[i] < 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_gengk_matches_algorithm1_oracle(precision):
    n1, n2 = 12, 12
    th = theta(0.2, 0.5, sigma2=1.0, tau2=0.25)
    g, mask, y, yo = _problem(n1, n2, th, 0.3)
    S = dense.full_correlation(g, th)
    obs = np.flatnonzero(mask.ravel())
    A = np.zeros((obs.size, n1 * n2))
    A[np.arange(obs.size), obs] = 1.0
    eta = th["tau2"] / th["sigma2"]
    k = 15
    with K.Problem(n1, n2, mask, y) as P:
        a, b, z, x, J = K.kry_gengk(P.h, K.theta_from_dict(th),
                                    K.kry_opts_default(gk_steps=k, reorth=1, precision=precision), n=n1 * n2)
        kf = obs.size
        af, bf, zf, xf, Jf = K.kry_gengk(P.h, K.theta_from_dict(th), K.kry_opts_default(gk_steps=kf, reorth=1),
                                         n=n1 * n2)
    beta1, U, V, B, al, be = gengk.gengk(A, S, yo, eta, k, reorth=True)
    zr, Jr = gengk.projected_solve(B, beta1, 1.0)
    tol = 1e-9 if precision == 0 else 1e-3
    np.testing.assert_allclose(a[:k], al, rtol=tol)
    np.testing.assert_allclose(b[: k + 1], be, rtol=tol)
    np.testing.assert_allclose(z, zr, rtol=tol * 10, atol=tol * np.abs(zr).max())
    assert abs(J - Jr) <= tol * Jr
    # k = p: the quadratic form and x_k* are exact (eq. act_xhat)
    ref = dense.loglik(g, mask, th, yo)
    assert abs(Jf - ref["quad"]) <= 1e-9 * ref["quad"]
    assert normwise(xf, dense.posterior_mean_all(g, mask, th, yo)) <= 1e-9


def test_kriging_exact_config1():
    g, mask_all, y, _ = _problem(32, 32, CONFIG1, 0.0)
    mask, held = synth.held_out_cells(mask_all, 100, seed=404)
    yo = y.ravel()[mask.ravel().astype(bool)]
    mean_ref, vx_ref, vy_ref = dense.krige(g, mask, CONFIG1, yo, held)
    with K.Problem(32, 32, mask, y) as P:
        for prec in (0, 1):
            mean, vx, vy = K.kry_krige(P.h, K.theta_from_dict(CONFIG1), K.kry_opts_default(precision=prec), held)
            assert np.abs(mean - mean_ref).max() <= 1e-6 * np.abs(mean_ref).max()
            np.testing.assert_allclose(vx, vx_ref, rtol=1e-6)
            np.testing.assert_allclose(vy, vy_ref, rtol=1e-6)


def test_sampler_matches_oracle_and_psd_torus():
    n1, n2 = 24, 20
    th = theta(0.15, 1.0, sigma2=2.0, tau2=0.1, ratio=2.0, angle=np.pi / 6)
    g = grid(n1, n2)
    with K.Problem(n1, n2, np.ones((n1, n2))) as P:
        N = K.kry_psd_torus(P.h, K.theta_from_dict(th))
        f, mm = K.kry_sample(P.h, K.theta_from_dict(th), N[0], N[1], 999, 3, 2, n1, n2)
    assert N == sampler.psd_torus(g, th, P.N1, P.N2)
    for i in range(2):
        ref, _ = sampler.circulant_field(g, th, N[0], N[1], seed=999, stream=3 + i)
        assert normwise(f[i], ref) <= 1e-12


def test_bootstrap_matches_oracle():
    n1, n2 = 16, 16
    th = theta(0.15, 0.5, sigma2=1.0, tau2=0.1)
    g, mask, y, yo = _problem(n1, n2, th, 0.3)
    targets = np.flatnonzero(mask.ravel() == 0)
    B = 6
    opts = K.kry_opts_default(seed=4242, cg_rtol=1e-12)
    with K.Problem(n1, n2, mask, y) as P:
        N = K.kry_psd_torus(P.h, K.theta_from_dict(th))
        mean, vx, vy = K.kry_krige(P.h, K.theta_from_dict(th), opts, None, ntargets=targets.size, bootstrap_B=B)
    rx, ry = bootstrap.bootstrap_variance(g, mask, th, targets, B, N[0], N[1], seed=4242)
    np.testing.assert_allclose(vx, rx, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(vy, ry, rtol=1e-7, atol=1e-12)
    mref, _, _ = dense.krige(g, mask, th, yo, targets)
    assert np.abs(mean - mref).max() <= 1e-6 * np.abs(mref).max()


def test_fit_reaches_dense_optimum():
    n1 = n2 = 16
    th = theta(0.15, 0.5, sigma2=1.0, tau2=0.3)
    g, mask, y, yo = _problem(n1, n2, th, 0.2, data_seed=8)
    rho_o, eta_o, best = fit.fit(g, mask, yo, th, x0=[np.log(0.1), np.log(0.2)])
    opts = K.kry_opts_default(lanczos_steps=80, probe_kind=K.KRY_PROBE_COLOURED, colour_period=16, cg_rtol=1e-10)
    init = K.theta(sigma2=1.0, tau2=0.2, range=0.1, nu=0.5)
    with K.Problem(n1, n2, mask, y) as P:
        est, at = K.kry_fit(P.h, init, 3, opts, xtol=1e-4, maxiter=300)
    # colour period 16 covers the grid: the log-det is exact, so the optimum is the dense one
    assert abs(np.log(est.range) - np.log(rho_o)) < 5e-3
    assert abs(np.log(est.tau2 / est.sigma2) - np.log(eta_o)) < 5e-3
    assert abs(at["loglik_profiled"] - best) < 1e-6 * abs(best)


@pytest.mark.parametrize("probes", [6, 5])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_points(precision, probes):
    # an odd probe count leaves the second vector slot of the last column
    # workgroup unused in FP32: regression case for its spectrum index
    n1, n2 = 24, 24
    g, mask, y, yo = _problem(n1, n2, CONFIG1, 0.3)
    thetas = [theta(0.05, 0.5, tau2=0.2), theta(0.1, 1.5, tau2=0.05), theta(0.2, 2.5, tau2=0.5)]
    opts = K.kry_opts_default(lanczos_steps=25, num_probes=probes, precision=precision)
    with K.Problem(n1, n2, mask, y) as P:
        batch = K.kry_loglik_batch(P.h, [K.theta_from_dict(t) for t in thetas], opts)
        single = [K.kry_loglik(P.h, K.theta_from_dict(t), opts) for t in thetas]
    for b, s, t in zip(batch, single, thetas):
        assert b["logdet"] == s["logdet"] and b["quad"] == s["quad"] and b["cg_iters"] == s["cg_iters"]
        ref = dense.loglik(g, mask, t, yo)
        assert abs(b["quad"] - ref["quad"]) <= 1e-7 * ref["quad"]


def test_error_paths():
    n1, n2 = 8, 8
    mask = np.ones((n1, n2))
    y = np.zeros((n1, n2))
    ctx = K.kry_ctx_create()
    try:
        with pytest.raises(K.KryError) as e:
            K.kry_problem_create(ctx, n1, n2, np.zeros((n1, n2)))
        assert e.value.status == K.KRY_EINVAL
        bad = y.copy()
        bad[3, 3] = np.nan
        with pytest.raises(K.KryError) as e:
            K.kry_problem_create(ctx, n1, n2, mask, bad)
        assert e.value.status == K.KRY_EINVAL
        h = K.kry_problem_create(ctx, n1, n2, mask, synth.random_vectors(64, 1, seed=1)[0])
        try:
            for bad_th in (K.theta(nu=0.0), K.theta(range=-1.0), K.theta(tau2=-0.1), K.theta(aniso_ratio=0.5)):
                with pytest.raises(K.KryError) as e:
                    K.kry_loglik(h, bad_th, K.kry_opts_default())
                assert e.value.status == K.KRY_EINVAL
            with pytest.raises(K.KryError) as e:
                K.kry_loglik(h, K.theta(range=0.3, nu=2.5, tau2=1e-3), K.kry_opts_default(cg_maxit=1))
            assert e.value.status == K.KRY_ENOCONV
            r = K.kry_loglik(h, K.theta(range=0.3, nu=2.5, tau2=1e-3), K.kry_opts_default(cg_maxit=1),
                             allow_noconv=True)
            assert r["cg_iters"] == 1 and r["cg_relres"] > 1e-8
            with pytest.raises(K.KryError) as e:
                K.kry_sample(h, K.theta(range=2.0, nu=2.5), 16, 16, 1, 0, 1, n1, n2)
            assert e.value.status == K.KRY_ENOTPSD
        finally:
            K.kry_problem_destroy(h)
    finally:
        K.kry_ctx_destroy(ctx)
    # a budget that holds the context's tables (about 1.4 MB) but not a
    # 512 x 512 problem
    small = K.kry_ctx_create(0, 3 << 20)
    try:
        with pytest.raises(K.KryError) as e:
            K.kry_problem_create(small, 512, 512, np.ones((512, 512)))
        assert e.value.status == K.KRY_ENOMEM
    finally:
        K.kry_ctx_destroy(small)


def _shift_case():
    n1, n2 = 24, 24
    g, mask, y, yo = _problem(n1, n2, CONFIG1, 0.3)
    thetas = [theta(r, 1.5, tau2=e) for r in (0.05, 0.15) for e in (0.02, 0.2, 1.0)]
    thetas.append(theta(0.1, 0.5, tau2=0.3))  # a group of one
    return n1, n2, g, mask, y, yo, thetas


@pytest.mark.parametrize("precision", [0, 1])
def test_shift_share_matches_oracle(precision):
    # one Lanczos recurrence on Sigma_oo per group and probe, quadrature of
    # T + eta I per point, and one multi-shift CG per group: the oracle runs
    # Lanczos on each K = Sigma_oo + eta I and solves each K densely
    n1, n2, g, mask, y, yo, thetas = _shift_case()
    r, c = observed_cells(mask)
    m, npr = 40, 6
    opts = K.kry_opts_default(lanczos_steps=m, num_probes=npr, reorth=1, cg_rtol=1e-10, shift_share=1,
                              precision=precision)
    with K.Problem(n1, n2, mask, y) as P:
        res = K.kry_loglik_batch(P.h, [K.theta_from_dict(t) for t in thetas], opts)
    Z = philox.probe_matrix(r, c, npr, opts.seed)
    for got, t in zip(res, thetas):
        Kd = dense.covariance(g, mask, t)
        est, _, _, _ = lanczos.slq_logdet(lambda v: Kd @ v, Z, m, reorth=True)
        tol = 1e-9 if precision == 0 else 1e-5
        assert abs(got["logdet"] - est) <= tol * abs(est), (t, got["logdet"], est)
        ref = dense.loglik(g, mask, t, yo)
        # the quadratic form runs in FP64 in both forms
        assert abs(got["quad"] - ref["quad"]) <= 1e-8 * ref["quad"]
        assert got["cg_relres"] <= 1e-10 and got["cg_iters"] > 0


@pytest.mark.parametrize("precision", [0, 1])
def test_shift_share_same_alone_and_in_mix(precision):
    n1, n2, g, mask, y, yo, thetas = _shift_case()
    opts = K.kry_opts_default(lanczos_steps=20, num_probes=5, shift_share=1, precision=precision)
    with K.Problem(n1, n2, mask, y) as P:
        mix = K.kry_loglik_batch(P.h, [K.theta_from_dict(t) for t in thetas], opts)
        # reversed order changes every group's position and its packing
        rev = K.kry_loglik_batch(P.h, [K.theta_from_dict(t) for t in thetas[::-1]], opts)[::-1]
        alone = [K.kry_loglik(P.h, K.theta_from_dict(t), opts) for t in thetas]
    for a, b, s in zip(mix, rev, alone):
        for k in ("logdet", "quad", "cg_iters", "cg_relres", "lanczos_steps_used"):
            assert a[k] == s[k] and b[k] == s[k], k


def test_shift_share_even_spectra_on_a_power_of_two_embedding():
    # 32 x 32 grid, 64 x 64 embedding (power-of-two column kernels): the
    # multi-shift CG reads half of each spectrum when every group's covariance
    # is even (isotropic or grid-aligned), the whole of it otherwise, and takes
    # p . w from the spectrum of p inside the product; a point's result does
    # not depend on the other points of the call
    n1, n2 = 32, 32
    g, mask, y, yo = _problem(n1, n2, CONFIG1, 0.3)
    sets = [[theta(r, 1.5, tau2=e) for r in (0.05, 0.15) for e in (0.02, 0.3)],
            [theta(0.1, 0.5, tau2=e, ratio=2.0, angle=0.0) for e in (0.05, 0.5)],
            [theta(0.1, 0.5, tau2=0.1), theta(0.1, 0.5, tau2=0.1, ratio=2.0, angle=0.7)]]
    opts = K.kry_opts_default(lanczos_steps=10, num_probes=2, cg_rtol=1e-10, shift_share=1)
    with K.Problem(n1, n2, mask, y) as P:
        assert K.kry_problem_info(P.h)[1] == 64
        for thetas in sets:
            ths = [K.theta_from_dict(t) for t in thetas]
            res = K.kry_loglik_batch(P.h, ths, opts)
            rev = K.kry_loglik_batch(P.h, ths[::-1], opts)[::-1]
            for got, back, th, t in zip(res, rev, ths, thetas):
                ref = dense.loglik(g, mask, t, yo)
                assert abs(got["quad"] - ref["quad"]) <= 1e-8 * ref["quad"], t
                assert got["cg_relres"] <= 1e-10
                alone = K.kry_loglik(P.h, th, opts)
                for k in ("quad", "cg_iters", "cg_relres"):
                    assert got[k] == alone[k] and back[k] == alone[k], (k, t)


@pytest.mark.parametrize("shape, N1", [((2048, 48), 4096), ((4096, 12), 8192)])
def test_shift_share_long_power_of_two_columns(shape, N1):
    # 4096- and 8192-point columns: eight and sixteen wavefronts per column
    # write the spectral p . Ap partials; the shared form's quadratic forms
    # against the unshared FP64 CG's (a dot of p with the product)
    n1, n2 = shape
    mask = synth.uniform_mask(n1, n2, 0.3, seed=21)
    y = synth.random_vectors(n1 * n2, 1, seed=22)[0].reshape(n1, n2)
    ths = [K.theta_from_dict(theta(0.05, 1.5, tau2=e)) for e in (0.05, 0.5)]
    base = dict(lanczos_steps=5, num_probes=2, cg_rtol=1e-11)
    with K.Problem(n1, n2, mask, y) as P:
        assert K.kry_problem_info(P.h)[1] == N1
        sh = K.kry_loglik_batch(P.h, ths, K.kry_opts_default(shift_share=1, **base))
        un = K.kry_loglik_batch(P.h, ths, K.kry_opts_default(**base))
    for a, b in zip(sh, un):
        assert a["cg_relres"] <= 1e-11 and b["cg_relres"] <= 1e-11
        assert abs(a["quad"] - b["quad"]) <= 1e-8 * abs(b["quad"])


def test_shift_share_with_more_shifts_than_a_block():
    # 300 shifts (30 ranges x 10 nuggets): more than one thread each in a
    # reduction block, so the scalar step takes its looped form; the same
    # points in batches of 150 take the one-pass form
    n1, n2 = 20, 16
    g, mask, y, yo = _problem(n1, n2, CONFIG1, 0.3)
    thetas = [theta(float(r), 1.5, tau2=float(e)) for r in np.geomspace(0.03, 0.2, 30)
              for e in np.geomspace(0.01, 1.0, 10)]
    opts = K.kry_opts_default(lanczos_steps=8, num_probes=2, cg_rtol=1e-10, shift_share=1)
    with K.Problem(n1, n2, mask, y) as P:
        ths = [K.theta_from_dict(t) for t in thetas]
        whole = K.kry_loglik_batch(P.h, ths, opts)
        parts = K.kry_loglik_batch(P.h, ths[:150], opts) + K.kry_loglik_batch(P.h, ths[150:], opts)
    for k in range(0, 300, 7):
        ref = dense.loglik(g, mask, thetas[k], yo)
        assert abs(whole[k]["quad"] - ref["quad"]) <= 1e-8 * ref["quad"], thetas[k]
    for a, b in zip(whole, parts):
        assert a["cg_relres"] <= 1e-10 and b["cg_relres"] <= 1e-10
        assert abs(a["cg_iters"] - b["cg_iters"]) <= 1
        assert abs(a["quad"] - b["quad"]) <= 1e-11 * abs(b["quad"])


def test_shift_share_zero_nugget_and_unshared_agreement():
    # a zero nugget makes the point its group's base system; the shared and
    # unshared forms agree to rounding of the two recurrences
    n1, n2 = 20, 20
    th = theta(0.05, 0.5, tau2=0.0)
    g, mask, y, yo = _problem(n1, n2, th, 0.3, cholesky=False)
    thetas = [th, theta(0.05, 0.5, tau2=0.1)]
    base = dict(lanczos_steps=30, num_probes=4, reorth=1, cg_rtol=1e-10)
    with K.Problem(n1, n2, mask, y) as P:
        sh = K.kry_loglik_batch(P.h, [K.theta_from_dict(t) for t in thetas], K.kry_opts_default(shift_share=1, **base))
        un = K.kry_loglik_batch(P.h, [K.theta_from_dict(t) for t in thetas], K.kry_opts_default(**base))
    for a, b, t in zip(sh, un, thetas):
        ref = dense.loglik(g, mask, t, yo)
        assert abs(a["quad"] - ref["quad"]) <= 1e-8 * ref["quad"]
        assert abs(a["logdet"] - b["logdet"]) <= 1e-8 * abs(b["logdet"])


@pytest.mark.parametrize("precision", [0, 1])
def test_loglik_multi_matches_single_problems(precision):
    # grids of different sizes: three share a 64 x 64 embedding, two a 32 x 32
    # one; each problem's result must match its own single-problem run
    shapes = [(20, 20), (12, 12), (24, 30), (17, 32), (9, 14)]
    thetas = [theta(0.1, 0.5, tau2=0.2), theta(0.15, 1.5, tau2=0.05), theta(0.08, 2.5, tau2=0.3),
              dict(theta(0.2, 1.0, tau2=0.1), aniso_ratio=2.0, aniso_angle=0.5), theta(0.3, 0.5, tau2=0.5)]
    opts = K.kry_opts_default(lanczos_steps=25, num_probes=5, reorth=1, cg_rtol=1e-10, precision=precision)
    ctx = K.kry_ctx_create()
    hs = []
    try:
        for i, ((n1, n2), t) in enumerate(zip(shapes, thetas)):
            mask = synth.uniform_mask(n1, n2, 0.15 + 0.1 * i, seed=40 + i)
            y = synth.random_vectors(n1 * n2, 1, seed=50 + i)[0]
            hs.append(K.kry_problem_create(ctx, n1, n2, mask, y))
        th = [K.theta_from_dict(t) for t in thetas]
        multi = K.kry_loglik_multi(hs, th, opts)
        single = [K.kry_loglik(h, t, opts) for h, t in zip(hs, th)]
        # reversed order: a problem's result does not depend on its neighbours
        rev = K.kry_loglik_multi(hs[::-1], th[::-1], opts)[::-1]
    finally:
        for h in hs:
            K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)
    tol_ld = 1e-10 if precision == 0 else 1e-5
    for m, s, r in zip(multi, single, rev):
        assert m["p"] == s["p"]
        assert abs(m["logdet"] - s["logdet"]) <= tol_ld * abs(s["logdet"])
        assert abs(m["quad"] - s["quad"]) <= 1e-8 * s["quad"]
        assert m["logdet"] == r["logdet"] and m["quad"] == r["quad"]
        assert m["cg_relres"] <= 1e-10


def test_loglik_multi_errors():
    ctx = K.kry_ctx_create()
    h = K.kry_problem_create(ctx, 8, 8, np.ones((8, 8)), np.zeros((8, 8)))
    try:
        with pytest.raises(K.KryError):
            K.kry_loglik_multi([h], [K.theta(sigma2=1.0, tau2=0.1, range=0.1, nu=0.5)],
                               K.kry_opts_default(shift_share=1))
        with pytest.raises(K.KryError):
            K.kry_loglik_multi([h], [K.theta(sigma2=1.0, tau2=0.1, range=0.1, nu=0.5)],
                               K.kry_opts_default(solver=K.KRY_SOLVER_GENGK))
    finally:
        K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)


@pytest.mark.parametrize("precision", [0, 1])
def test_adaptive_lanczos_matches_oracle_rule(precision):
    # the adaptive mode stops where every probe's quadrature value settled
    # over 5 steps (checks from step 10); the oracle applies the same rule
    n1, n2 = 24, 24
    th = theta(0.15, 1.5, tau2=0.05)
    g, mask, y, yo = _problem(n1, n2, th, 0.3)
    Kd = dense.covariance(g, mask, th)
    r, c = observed_cells(mask)
    opts = K.kry_opts_default(num_probes=6, reorth=1, lanczos_rtol=1e-6, lanczos_max_steps=120,
                              precision=precision, cg_rtol=1e-10)
    Z = philox.probe_matrix(r, c, 6, opts.seed)
    est, _, vals, m = lanczos.slq_logdet_adaptive(lambda v: Kd @ v, Z, 120, 1e-6, reorth=True)
    assert 10 <= m < 120
    with K.Problem(n1, n2, mask, y) as P:
        ld, _, per = K.kry_logdet(P.h, K.theta_from_dict(th), opts)
        res = K.kry_loglik(P.h, K.theta_from_dict(th), opts)
    tol = 1e-9 if precision == 0 else 1e-5
    assert abs(ld - est) <= tol * abs(est)
    np.testing.assert_allclose(per, vals, rtol=tol * 10)
    assert res["lanczos_steps_used"] == m and res["logdet"] == ld


@pytest.mark.parametrize("share", [0, 1])
def test_adaptive_lanczos_same_alone_and_in_mix(share):
    n1, n2, g, mask, y, yo, thetas = _shift_case()
    opts = K.kry_opts_default(num_probes=5, reorth=1, lanczos_rtol=1e-5, lanczos_max_steps=100, shift_share=share)
    with K.Problem(n1, n2, mask, y) as P:
        mix = K.kry_loglik_batch(P.h, [K.theta_from_dict(t) for t in thetas], opts)
        alone = [K.kry_loglik(P.h, K.theta_from_dict(t), opts) for t in thetas]
    for a, s in zip(mix, alone):
        for k in ("logdet", "quad", "lanczos_steps_used"):
            assert a[k] == s[k], k
    assert len({a["lanczos_steps_used"] for a in mix}) > 1  # points settle at different steps


@pytest.mark.parametrize("precision", [0, 1])
def test_reorth_past_the_fused_basis_sizes(precision):
    # 80 steps with full reorthogonalisation: the first update and the second
    # dots share one basis sweep up to 64 (FP32) or 32 (FP64) basis vectors,
    # separate sweeps after that; both stretches must follow the oracle
    n1, n2 = 24, 24
    th = theta(0.15, 1.5, tau2=0.05)
    g, mask, y, yo = _problem(n1, n2, th, 0.3)
    Kd = dense.covariance(g, mask, th)
    r, c = observed_cells(mask)
    m, npr = 80, 4
    opts = K.kry_opts_default(lanczos_steps=m, num_probes=npr, reorth=1, precision=precision)
    with K.Problem(n1, n2, mask, y) as P:
        _, _, steps = K.kry_lanczos(P.h, K.theta_from_dict(th), opts)
        ld, _, per = K.kry_logdet(P.h, K.theta_from_dict(th), opts)
    assert list(steps) == [m] * npr
    Z = philox.probe_matrix(r, c, npr, opts.seed)
    est, _, vals, _ = lanczos.slq_logdet(lambda v: Kd @ v, Z, m, reorth=True)
    tol = 1e-9 if precision == 0 else 1e-5
    assert abs(ld - est) <= tol * abs(est), (ld, est)
    np.testing.assert_allclose(per, vals, rtol=tol * 10)
