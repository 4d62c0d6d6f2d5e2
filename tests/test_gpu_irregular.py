"""GPU parity for irregularly spaced observations (the Wendland mapping of
Sec. 2): the product, the likelihood in every form, kriging at grid cells,
the bootstrap, genGK and the paper's objective, at small sizes against the
dense oracle and at the paper's third-study size on sampled rows."""
import numpy as np
import pytest

from oracle import dense, gengk, irregular, lanczos, plik, sampler
from oracle.philox import probe_matrix
from paper_2012_13133_amd import synth
from tests.gpu_util import normwise
from tests.oracle_cases import grid, theta

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_2012_13133_amd.kryging")

TH = theta(0.15, 1.5, sigma2=1.4, tau2=0.25, ratio=1.5, angle=0.3)


def _case(n1=24, n2=20, p=300, th=TH, seed=1):
    g = grid(n1, n2)
    locs = synth.irregular_locations(g, p, seed=seed)
    A = irregular.mapping_matrix(g, locs)
    x, _ = sampler.cholesky_field(g, th, seed=seed + 1)
    rng = np.random.default_rng(seed + 2)
    y = A @ x.ravel() + np.sqrt(th["tau2"]) * rng.standard_normal(p)
    return g, locs, A, y


def test_product_matches_oracle():
    g, locs, A, y = _case()
    V = synth.random_vectors(300, 3, seed=5)
    ref = irregular.matvec(g, locs, TH, V.T).T
    with K.IrregularProblem(24, 20, locs, y) as P:
        got64 = K.kry_matvec(P.h, K.theta_from_dict(TH), V, K.KRY_FP64)
        got32 = K.kry_matvec(P.h, K.theta_from_dict(TH), V, K.KRY_FP32)
    for i in range(3):
        assert normwise(got64[i], ref[i]) <= 1e-12
        assert normwise(got32[i], ref[i]) <= 1e-5


def test_caller_order_is_kept_at_every_entry_point():
    # the library stores observations by nearest cell: the same observations
    # given in cell order and in a shuffled order give the same results, in
    # the caller's order
    g, locs, A, y = _case(seed=21)
    near = np.minimum(np.floor(locs[:, 0] + 0.5), 23) * 20 + np.minimum(np.floor(locs[:, 1] + 0.5), 19)
    srt = np.argsort(near, kind="stable")
    perm = np.random.default_rng(3).permutation(300)
    V = synth.random_vectors(300, 2, seed=6)
    th = K.theta_from_dict(TH)
    opts = K.kry_opts_default(lanczos_steps=30, num_probes=4, reorth=1, cg_rtol=1e-11)
    out = {}
    for name, o in (("sorted", srt), ("shuffled", perm)):
        with K.IrregularProblem(24, 20, locs[o], y[o]) as P:
            inv = np.argsort(o)
            out[name] = dict(
                mv=K.kry_matvec(P.h, th, V[:, o], K.KRY_FP64)[:, inv],
                x=K.kry_solve(P.h, th, opts, V[:, o])[0][:, inv],
                ll=K.kry_loglik(P.h, th, opts),
                pr=K.kry_probes(P.h, opts),
                kr=K.kry_krige(P.h, th, opts, np.array([0, 77, 479])))
    a, b = out["sorted"], out["shuffled"]
    for i in range(2):
        assert normwise(b["mv"][i], a["mv"][i]) <= 1e-13
        assert normwise(b["x"][i], a["x"][i]) <= 1e-9
    assert b["ll"]["quad"] == pytest.approx(a["ll"]["quad"], rel=1e-10)
    # probes are drawn by the caller's index
    Z = probe_matrix(np.zeros(300, dtype=np.int64), np.zeros(300, dtype=np.int64), 4, opts.seed).T
    np.testing.assert_array_equal(a["pr"], Z)
    np.testing.assert_array_equal(b["pr"], Z)
    for u, v in zip(a["kr"], b["kr"]):
        np.testing.assert_allclose(v, u, rtol=1e-8)


def test_on_grid_locations_equal_the_masked_problem():
    n1, n2 = 20, 18
    mask = synth.uniform_mask(n1, n2, 0.3, seed=7)
    obs = np.flatnonzero(mask.ravel())
    a, b = np.divmod(obs, n2)
    locs = np.stack([a, b], axis=1).astype(np.float64)
    yfull = synth.random_vectors(n1 * n2, 1, seed=8)[0]
    opts = K.kry_opts_default(lanczos_steps=25, num_probes=6, reorth=1, cg_rtol=1e-11)
    th = K.theta_from_dict(TH)
    with K.Problem(n1, n2, mask, yfull) as Pm, K.IrregularProblem(n1, n2, locs, yfull[obs]) as Pi:
        rm = K.kry_loglik(Pm.h, th, opts)
        ri = K.kry_loglik(Pi.h, th, opts)
        km = K.kry_krige(Pm.h, th, opts, np.array([0, 50, 123]))
        ki = K.kry_krige(Pi.h, th, opts, np.array([0, 50, 123]))
    assert ri["logdet"] == pytest.approx(rm["logdet"], rel=1e-10)
    assert ri["quad"] == pytest.approx(rm["quad"], rel=1e-9)
    for u, v in zip(km, ki):
        np.testing.assert_allclose(v, u, rtol=1e-8)


@pytest.mark.parametrize("precision", [0, 1])
def test_loglik_matches_oracle(precision):
    g, locs, A, y = _case(seed=11)
    ref = irregular.loglik(g, locs, TH, y)
    Kd = irregular.covariance(g, A, TH)
    with K.IrregularProblem(24, 20, locs, y) as P:
        opts = K.kry_opts_default(lanczos_steps=60, num_probes=8, reorth=1, precision=precision, cg_rtol=1e-11)
        r = K.kry_loglik(P.h, K.theta_from_dict(TH), opts)
        _, _, per = K.kry_logdet(P.h, K.theta_from_dict(TH), opts)
        # shift-shared batch over nuggets against the plain form
        pts = [dict(TH, tau2=e) for e in (0.05, 0.25, 1.0)]
        sh = K.kry_loglik_batch(P.h, [K.theta_from_dict(t) for t in pts],
                                K.kry_opts_default(lanczos_steps=60, num_probes=8, reorth=1, precision=precision,
                                                   cg_rtol=1e-11, shift_share=1))
    assert abs(r["quad"] - ref["quad"]) <= 1e-8 * ref["quad"]
    # per-probe quadrature against the oracle's SLQ with the same probes and steps
    Z = probe_matrix(np.zeros(300, dtype=np.int64), np.zeros(300, dtype=np.int64), 8, opts.seed)
    _, _, vals, _ = lanczos.slq_logdet(lambda u: Kd @ u, Z, 60, reorth=True)
    np.testing.assert_allclose(per, vals, rtol=1e-9 if precision == 0 else 1e-5)
    # eight probes: the estimate is within its reported Monte-Carlo error of the exact log-det
    assert abs(r["logdet"] - ref["logdet"]) <= 4 * r["logdet_se"]
    for k, t in enumerate(pts):
        rr = irregular.loglik(g, locs, t, y)
        assert abs(sh[k]["quad"] - rr["quad"]) <= 1e-8 * rr["quad"]


@pytest.mark.parametrize("precision", [0, 1])
def test_kriging_at_cells_and_bootstrap_match_oracle(precision):
    g, locs, A, y = _case(seed=21)
    tg = np.arange(0, 480, 7)
    mean_ref, vx_ref, vy_ref = irregular.krige_cells(g, locs, TH, y, tg)
    with K.IrregularProblem(24, 20, locs, y) as P:
        th = K.theta_from_dict(TH)
        mean, vx, vy = K.kry_krige(P.h, th, K.kry_opts_default(precision=precision, cg_rtol=1e-11), tg)
        N = K.kry_psd_torus(P.h, th)
        _, bx, by = K.kry_krige(P.h, th, K.kry_opts_default(precision=precision, cg_rtol=1e-11, seed=77), tg,
                                bootstrap_B=6)
        full = K.kry_krige(P.h, th, K.kry_opts_default(cg_rtol=1e-10), None, ntargets=480, want_var=False)[0]
    assert np.abs(mean - mean_ref).max() <= 1e-7 * np.abs(mean_ref).max()
    np.testing.assert_allclose(vx, vx_ref, rtol=1e-7)
    np.testing.assert_allclose(vy, vy_ref, rtol=1e-7)
    bx_ref, by_ref = irregular.bootstrap_variance(g, locs, TH, tg, 6, N[0], N[1], 77)
    np.testing.assert_allclose(bx, bx_ref, rtol=1e-6)
    np.testing.assert_allclose(by, by_ref, rtol=1e-6)
    m_all, _, _ = irregular.krige_cells(g, locs, TH, y, np.arange(480))
    assert np.abs(full - m_all).max() <= 1e-7 * np.abs(m_all).max()


def test_gengk_plik_and_posterior_variance_match_oracle():
    n1, n2 = 12, 12
    th = theta(0.2, 0.5, sigma2=1.0, tau2=0.3)
    g, locs, A, y = _case(n1, n2, 90, th, seed=31)
    S = dense.full_correlation(g, th)
    with K.IrregularProblem(n1, n2, locs, y) as P:
        t = K.theta_from_dict(th)
        k = 90
        _, _, _, _, J = K.kry_gengk(P.h, t, K.kry_opts_default(gk_steps=k, reorth=1))
        r = K.kry_plik(P.h, t, K.kry_opts_default(gk_steps=20, reorth=1))
        vx, _, _ = K.kry_posterior_variance(P.h, t, K.kry_opts_default(gk_steps=k, reorth=1), n1 * n2)
    assert J == pytest.approx(irregular.loglik(g, locs, th, y)["quad"], rel=1e-9)
    ref = plik.approx_plik(g, None, th, y, 20, A=A)
    assert r["pl"] == pytest.approx(ref["pl"], rel=1e-9)
    assert r["psi2"] == pytest.approx(ref["psi2"], rel=1e-9)
    assert r["grad_range"] == pytest.approx(ref["grad"]["rho"], rel=1e-8)
    _, v_ref, _ = irregular.krige_cells(g, locs, th, y, np.arange(n1 * n2))
    np.testing.assert_allclose(vx, v_ref, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(gengk.posterior_variance(A, S, y, th["sigma2"], th["tau2"], k), v_ref, rtol=1e-8,
                               atol=1e-10)


def test_covariates_per_observation_and_errors():
    g, locs, A, y = _case(seed=41)
    X = np.stack([np.ones(300), locs[:, 1] / 20.0])
    yy = y + X.T @ np.array([44.49, 2.0])
    with K.IrregularProblem(24, 20, locs, yy) as P:
        K.kry_problem_set_covariates(P.h, X)
        r = K.kry_loglik(P.h, K.theta_from_dict(TH), K.kry_opts_default(cg_rtol=1e-11, lanczos_steps=10))
        Kd = irregular.covariance(g, A, TH)
        beta, _, Q = dense.gls(Kd, X.T, yy)
        assert r["quad"] == pytest.approx(Q, rel=1e-8)
        np.testing.assert_allclose(r["beta"], beta, rtol=1e-8)
        with pytest.raises(K.KryError) as e:
            K.kry_krige(P.h, K.theta_from_dict(TH), K.kry_opts_default(), np.array([3]))
        assert e.value.status == K.KRY_ENOTIMPL
        with pytest.raises(K.KryError):
            K.kry_loglik_multi([P.h], [K.theta_from_dict(TH)], K.kry_opts_default())
    ctx = K.kry_ctx_create()
    try:
        with pytest.raises(K.KryError) as e:
            K.kry_problem_create_irregular(ctx, 8, 8, np.array([[7.5, 2.0]]))  # beyond the last row
        assert e.value.status == K.KRY_EINVAL
    finally:
        K.kry_ctx_destroy(ctx)


def test_paper_third_study_size_sampled_rows_and_precisions():
    # 40,000 irregular observations on a 400 x 400 latent grid (the third study)
    n = 400
    g = grid(n, n)
    locs = synth.irregular_locations(g, 40000, seed=51)
    th = theta(0.1, 0.5, sigma2=3.0, tau2=0.5)
    rng = np.random.default_rng(52)
    v = rng.standard_normal(40000)
    rows = np.sort(rng.choice(40000, size=12, replace=False))
    ref = irregular.matvec_rows(g, locs, th, v, rows)
    with K.IrregularProblem(n, n, locs, rng.standard_normal(40000)) as P:
        t = K.theta_from_dict(th)
        got64 = K.kry_matvec(P.h, t, v[None, :], K.KRY_FP64)[0]
        got32 = K.kry_matvec(P.h, t, v[None, :], K.KRY_FP32)[0]
        base = dict(lanczos_steps=30, num_probes=4, reorth=1, cg_rtol=1e-8, cg_maxit=100000)
        r64 = K.kry_loglik(P.h, t, K.kry_opts_default(precision=K.KRY_FP64, **base))
        r32 = K.kry_loglik(P.h, t, K.kry_opts_default(precision=K.KRY_FP32, **base))
    scale = np.sqrt(np.mean(got64 ** 2))
    assert np.abs(got64[rows] - ref).max() <= 1e-12 * scale
    assert np.abs(got32[rows] - ref).max() <= 1e-5 * scale
    assert abs(r32["quad"] - r64["quad"]) <= 1e-6 * r64["quad"]
    assert abs(r32["loglik"] - r64["loglik"]) <= 1e-3 * abs(r64["loglik"])


def test_server_requests_on_an_irregular_problem():
    g, locs, A, y = _case(seed=61)
    ctx = K.kry_ctx_create()
    h = K.kry_problem_create_irregular(ctx, 24, 20, locs, y)
    try:
        opts = K.kry_opts_default(lanczos_steps=20, num_probes=4, cg_rtol=1e-10)
        pts = [K.theta(sigma2=1.4, tau2=e, range=0.15, nu=1.5) for e in (0.1, 0.25, 0.6)]
        alone = [K.kry_loglik(h, t, opts) for t in pts]
        tg = np.array([5, 77, 300])
        kr = K.kry_krige(h, pts[1], opts, tg)
        srv = K.kry_server_create(ctx, slots=2, max_batch=8)
        try:
            pend = [K.kry_server_submit(srv, K.KRY_REQ_LOGLIK, h, t, opts) for t in pts]
            pk = K.kry_server_submit(srv, K.KRY_REQ_KRIGE, h, pts[1], opts, targets=tg, variances=True)
            res = [K.kry_server_wait(srv, pd) for pd in pend]
            rk = K.kry_server_wait(srv, pk)
        finally:
            K.kry_server_destroy(srv)
        for r, a in zip(res, alone):
            d = r.loglik.as_dict()
            assert r.status == 0 and d["quad"] == a["quad"] and d["logdet"] == a["logdet"]
        assert rk.status == 0
        np.testing.assert_array_equal(pk.outputs["mean_x"], kr[0])
        np.testing.assert_array_equal(pk.outputs["var_x"], kr[1])
    finally:
        K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)
