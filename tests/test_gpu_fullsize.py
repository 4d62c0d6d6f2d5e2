"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (32 vectors per product), on outputs the oracle computes one
row at a time, plus properties that hold at any size."""
import numpy as np
import pytest

from oracle import direct, sampler
from oracle.geometry import lag_table
from paper_2012_13133_amd import synth
from tests.oracle_cases import theta

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_2012_13133_amd.kryging")

CASES = {
    # metric shape: 1024^2, 30 % uniform missing, nu 1.5, range 0.05, nugget ratio 0.2
    "1024": (1024, theta(0.05, 1.5, sigma2=1.0, tau2=0.2), lambda n: synth.uniform_mask(n, n, 0.3, seed=101)),
    # large anisotropic shape: 2048^2, 40 % blob missing, nu 1, ratio 2 at 30 degrees, nugget ratio 0.1
    "2048": (2048, theta(0.05, 1.0, sigma2=1.0, tau2=0.1, ratio=2.0, angle=np.pi / 6),
             lambda n: synth.blob_mask(n, n, 0.4, seed=102)),
    # grids whose smallest embedding (the smallest-side rule) takes mixed
    # radices (600^2: 1200 = 2^4 3 5^2; 700^2: 1440 = 2^5 3^2 5; 880^2:
    # 1792 = 2^8 7)
    "600": (600, theta(0.04, 2.5, sigma2=1.0, tau2=0.2), lambda n: synth.uniform_mask(n, n, 0.3, seed=103)),
    "700": (700, theta(0.06, 0.5, sigma2=1.0, tau2=0.2, ratio=1.5, angle=0.3),
            lambda n: synth.blob_mask(n, n, 0.25, seed=104, rmin=5, rmax=40)),
    "880": (880, theta(0.03, 1.5, sigma2=1.0, tau2=0.1), lambda n: synth.uniform_mask(n, n, 0.2, seed=105)),
}
EMBEDDING = {"1024": 2048, "2048": 4096, "600": 1200, "700": 1440, "880": 1792}


@pytest.mark.parametrize("case", ["1024", "2048", "600", "700", "880"])
def test_masked_product_sampled_rows(case):
    n, th, mk = CASES[case]
    mask = mk(n)
    g = (n, n, 1.0 / n, 1.0 / n)
    p = int(mask.sum())
    rng = np.random.default_rng(7)
    v = rng.standard_normal((32, p))
    rows = np.sort(rng.choice(p, size=24, replace=False))
    T = lag_table(n, n, 1.0 / n, 1.0 / n, th)
    pick = [0, 13, 31]
    ref = direct.masked_matvec(g, mask, th, v[pick].T, rows=rows, table=T)  # (24, 3)
    with K.Problem(n, n, mask, embedding=K.KRY_EMBED_SMALLEST) as P:
        assert (P.N1, P.N2) == (EMBEDDING[case],) * 2
        got64 = K.kry_matvec(P.h, K.theta_from_dict(th), v, K.KRY_FP64)
        got32 = K.kry_matvec(P.h, K.theta_from_dict(th), v, K.KRY_FP32)
        if case in ("600", "700", "880"):
            # one and two vectors per column workgroup, both tile heights: bit for bit
            for cv in (1, 2):
                for rs in (1, 2):
                    for prec, ref_got in ((K.KRY_FP64, got64), (K.KRY_FP32, got32)):
                        K.kry_set_tuning(P.ctx, P.N1, P.N2, prec, cv, rs, 1, 0, 0)
                        np.testing.assert_array_equal(K.kry_matvec(P.h, K.theta_from_dict(th), v, prec), ref_got)
                        K.kry_set_tuning(P.ctx, P.N1, P.N2, prec)
    for got, tol in ((got64, 1e-12), (got32, 1e-5)):
        for j, vi in enumerate(pick):
            scale = np.sqrt(np.mean(got[vi] ** 2))
            assert np.abs(got[vi][rows] - ref[:, j]).max() <= tol * scale, (case, tol)
    # properties at full size: symmetry and positivity of K
    u, w = v[0], v[1]
    assert abs(u @ got64[1] - w @ got64[0]) <= 1e-11 * np.linalg.norm(u) * np.linalg.norm(got64[1])
    assert np.all(np.einsum("ij,ij->i", v, got64) > 0)


def test_sampler_full_size_matches_oracle():
    n, th, mk = CASES["1024"]
    g = (n, n, 1.0 / n, 1.0 / n)
    with K.Problem(n, n, np.ones((n, n), dtype=np.uint8)) as P:
        N = K.kry_psd_torus(P.h, K.theta_from_dict(th))
        f, _ = K.kry_sample(P.h, K.theta_from_dict(th), N[0], N[1], 202, 0, 1, n, n)
    ref, _ = sampler.circulant_field(g, th, N[0], N[1], seed=202, stream=0)
    # The field uses sqrt(lam): an absolute rounding error d in an eigenvalue
    # near zero becomes d / (2 sqrt(lam)) in sqrt(lam).  On a 2048^2 torus for
    # a smooth kernel the smallest kept eigenvalues are ~1e-9 of the largest,
    # which turns the FFTs' ~1e-16 relative rounding into ~1e-12 relative in
    # the field; the bar is 1e-10 (the small-torus test keeps 1e-12).
    assert np.linalg.norm(f[0] - ref) <= 1e-10 * np.linalg.norm(ref)


def test_loglik_fp32_form_matches_fp64_with_common_probes():
    n, th, mk = CASES["1024"]
    mask = mk(n)
    rng = np.random.default_rng(9)
    y = rng.standard_normal((n, n))
    with K.Problem(n, n, mask, y) as P:
        t = K.theta_from_dict(th)
        r64 = K.kry_loglik(P.h, t, K.kry_opts_default(lanczos_steps=50, num_probes=8, precision=K.KRY_FP64))
        r32 = K.kry_loglik(P.h, t, K.kry_opts_default(lanczos_steps=50, num_probes=8, precision=K.KRY_FP32,
                                                      cg_rtol=1e-6))
    assert abs(r32["loglik"] - r64["loglik"]) <= 1e-3 * abs(r64["loglik"])
    assert abs(r32["quad"] - r64["quad"]) <= 1e-6 * r64["quad"]


def test_masked_product_largest_embedding():
    # the largest grid the library takes: 4096 x 4096 (8192 x 8192 torus)
    n = 4096
    th = theta(0.02, 1.5, sigma2=1.0, tau2=0.2)
    mask = synth.uniform_mask(n, n, 0.3, seed=103)
    g = (n, n, 1.0 / n, 1.0 / n)
    p = int(mask.sum())
    rng = np.random.default_rng(11)
    v = rng.standard_normal((2, p))
    rows = np.sort(rng.choice(p, size=6, replace=False))
    T = lag_table(n, n, 1.0 / n, 1.0 / n, th)
    ref = direct.masked_matvec(g, mask, th, v.T, rows=rows, table=T)
    with K.Problem(n, n, mask) as P:
        assert (P.N1, P.N2) == (8192, 8192)
        got64 = K.kry_matvec(P.h, K.theta_from_dict(th), v, K.KRY_FP64)
        got32 = K.kry_matvec(P.h, K.theta_from_dict(th), v, K.KRY_FP32)
    for got, tol in ((got64, 1e-12), (got32, 1e-5)):
        for j in range(2):
            scale = np.sqrt(np.mean(got[j] ** 2))
            assert np.abs(got[j][rows] - ref[:, j]).max() <= tol * scale, tol


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_range_nugget_grid_fp32_shared_matches_plain_fp64(nu):
    # 512^2 with 30 % missing (the plain-vs-precision workload, every
    # smoothness it names): the FP32 shift-shared batch over a 3 x 3 (range,
    # nugget) grid against the plain FP64 form point by point, same probes
    n = 512
    mask = synth.uniform_mask(n, n, 0.3, seed=104)
    ranges, nuggets = (0.01, 0.05, 0.2), (0.01, 0.1, 1.0)
    thetas = [K.theta(sigma2=1.0, tau2=e, range=r, nu=nu) for r in ranges for e in nuggets]
    base = dict(lanczos_steps=50, num_probes=10, reorth=1, cg_rtol=1e-8, cg_maxit=100000)
    with K.Problem(n, n, mask) as P:
        th0 = K.theta(sigma2=1.0, tau2=0.2, range=0.05, nu=1.5)
        N = K.kry_psd_torus(P.h, th0)
        x, _ = K.kry_sample(P.h, th0, N[0], N[1], 202, 0, 1, n, n)
        y = x[0] + np.sqrt(0.2) * np.random.default_rng(5).standard_normal((n, n))
        K.kry_problem_set_data(P.h, y)
        batch = K.kry_loglik_batch(P.h, thetas, K.kry_opts_default(precision=K.KRY_FP32, shift_share=1, **base))
        for k in (2, 4, 6):  # (0.01, 1), (0.05, 0.1), (0.2, 0.01)
            plain = K.kry_loglik(P.h, thetas[k], K.kry_opts_default(precision=K.KRY_FP64, **base))
            for key in ("loglik", "loglik_profiled"):
                assert abs(batch[k][key] - plain[key]) <= 1e-3 * abs(plain[key]), (k, key)
            assert abs(batch[k]["quad"] - plain["quad"]) <= 1e-7 * plain["quad"]


@pytest.mark.parametrize("shape", [(2520, 20), (20, 2520)])
def test_masked_product_long_run_time_plan_sides(shape):
    # the smallest-side rule puts 2 2520 - 1 on 5040 = 2^4 3^2 5 7: a column
    # (630 threads) or a row (2520 points) of a run-time plan at its largest
    # workgroup classes; sampled rows against the direct sum
    n1, n2 = shape
    th = theta(0.05, 1.5, sigma2=1.0, tau2=0.2, ratio=1.5, angle=0.3)
    mask = synth.uniform_mask(n1, n2, 0.3, seed=106)
    g = (n1, n2, 1.0 / n1, 1.0 / n2)
    p = int(mask.sum())
    rng = np.random.default_rng(8)
    v = rng.standard_normal((4, p))
    rows = np.sort(rng.choice(p, size=24, replace=False))
    T = lag_table(n1, n2, 1.0 / n1, 1.0 / n2, th)
    ref = direct.masked_matvec(g, mask, th, v.T, rows=rows, table=T)  # (24, 4)
    with K.Problem(n1, n2, mask, embedding=K.KRY_EMBED_SMALLEST) as P:
        assert sorted((P.N1, P.N2)) == [48, 5040]
        got64 = K.kry_matvec(P.h, K.theta_from_dict(th), v, K.KRY_FP64)
        got32 = K.kry_matvec(P.h, K.theta_from_dict(th), v, K.KRY_FP32)
    for got, tol in ((got64, 1e-12), (got32, 1e-5)):
        for j in range(4):
            scale = np.sqrt(np.mean(got[j] ** 2))
            assert np.abs(got[j][rows] - ref[:, j]).max() <= tol * scale, (shape, tol)
