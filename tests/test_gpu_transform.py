"""GPU parity: lag grid, spectrum and masked BTTB product against the oracle."""
import numpy as np
import pytest

from oracle import direct
from oracle.geometry import embedding_lags
from paper_2012_13133_amd import synth
from tests.gpu_util import rows_rel
from tests.oracle_cases import grid, theta

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_2012_13133_amd.kryging")

THETAS = [
    theta(0.1, 0.5, tau2=0.1),
    theta(0.05, 1.5, tau2=0.2),
    theta(0.2, 2.5, tau2=0.05),
    theta(0.08, 1.0, tau2=0.1, ratio=2.0, angle=np.pi / 6),
    theta(0.15, 0.7, tau2=0.3, ratio=1.5, angle=2.0),
]


@pytest.mark.parametrize("th", THETAS)
@pytest.mark.parametrize("tor", [(16, 32), (64, 64), (128, 16)])
def test_lag_grid(th, tor):
    n1, n2 = 9, 7
    with K.Problem(n1, n2, np.ones((n1, n2))) as P:
        got = K.kry_lag_grid(P.h, K.theta_from_dict(th), *tor)
    ref = embedding_lags(tor[0], tor[1], 1.0 / n1, 1.0 / n2, th)
    assert np.all(np.abs(got - ref) <= 1e-13 * np.abs(ref) + 1e-15)


@pytest.mark.parametrize("th", THETAS)
@pytest.mark.parametrize("tor", [(16, 16), (64, 32), (256, 512), (48, 80), (96, 160), (1280, 768)])
def test_spectrum(th, tor):
    n1, n2 = 8, 8
    with K.Problem(n1, n2, np.ones((n1, n2))) as P:
        lam, mm = K.kry_spectrum(P.h, K.theta_from_dict(th), *tor)
    c = embedding_lags(tor[0], tor[1], 1.0 / n1, 1.0 / n2, th)
    ref = np.real(np.fft.fft2(c))[:, : tor[1] // 2 + 1].T
    scale = np.abs(ref).max()
    assert np.abs(lam - ref).max() <= 1e-12 * scale
    assert abs(mm[0] - ref.min()) <= 1e-12 * scale and abs(mm[1] - ref.max()) <= 1e-12 * scale


@pytest.mark.parametrize("tor", [(64, 32), (256, 512), (48, 80), (1280, 768), (112, 48)])
def test_spectrum_even_in_k1_for_even_covariances(tor):
    # an isotropic or grid-aligned covariance is even in the row lag, so its
    # spectrum is even in k1: the library's comes out even bit for bit (the
    # products of the multi-shift CG then read half of it); a rotated
    # anisotropy is not even and its spectrum is left as the transform gives it
    n1, n2 = 8, 8
    N1 = tor[0]
    cases = [(THETAS[0], True), (THETAS[2], True), (theta(0.08, 1.0, tau2=0.1, ratio=2.0, angle=0.0), True),
             (THETAS[3], False)]
    with K.Problem(n1, n2, np.ones((n1, n2))) as P:
        for th, even in cases:
            lam, _ = K.kry_spectrum(P.h, K.theta_from_dict(th), *tor)
            c = embedding_lags(tor[0], tor[1], 1.0 / n1, 1.0 / n2, th)
            ref = np.real(np.fft.fft2(c))[:, : tor[1] // 2 + 1].T
            scale = np.abs(ref).max()
            assert np.abs(lam - ref).max() <= 1e-12 * scale
            mirrored = lam[:, (-np.arange(N1)) % N1]
            if even:
                assert np.array_equal(lam, mirrored), th
            else:
                assert np.abs(lam - mirrored).max() > 1e-6 * scale, th


SHAPES = [(2, 2), (3, 5), (7, 9), (16, 16), (32, 32), (33, 47), (64, 50), (100, 3),
          # mixed-radix embeddings by the smallest-side rule: 48 x 64, 80 x 96,
          # 320 x 640, 384 x 768, 48 x 16 (radix 3 or 5), 128 x 112 and 224 x 16
          # above (radix 7), 96 x 144 (3 and 3^2), 240 x 400 (3 5 and 5^2),
          # 784 x 48 (7^2); the fast rule keeps some of them (80 x 96, 320 x 640, ...)
          (20, 30), (40, 41), (150, 300), (190, 380), (24, 3), (45, 68), (113, 200), (392, 20)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("ti", range(len(THETAS)))
@pytest.mark.parametrize("rule", ["fast", "smallest"])
def test_masked_product_fp64_and_fp32(shape, ti, rule):
    th = THETAS[ti]
    n1, n2 = shape
    g = grid(n1, n2)
    mask = synth.uniform_mask(n1, n2, 0.3 if n1 * n2 > 4 else 0.25, seed=11 + ti)
    p = int(mask.sum())
    v = synth.random_vectors(p, 3, seed=5)
    ref = direct.masked_matvec(g, mask, th, v.T).T
    emb = K.KRY_EMBED_FAST if rule == "fast" else K.KRY_EMBED_SMALLEST
    with K.Problem(n1, n2, mask, embedding=emb) as P:
        t = K.theta_from_dict(th)
        got64 = K.kry_matvec(P.h, t, v, K.KRY_FP64)
        got32 = K.kry_matvec(P.h, t, v, K.KRY_FP32)
    assert rows_rel(got64, ref) <= 1e-12
    assert rows_rel(got32, ref) <= 1e-5
    # element by element, against the largest entry of each output vector
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.all(np.abs(got64 - ref) <= 1e-12 * scale)
    assert np.all(np.abs(got32 - ref) <= 1e-5 * scale)


def test_all_missing_but_one_and_fully_observed():
    n1, n2 = 12, 10
    th = THETAS[1]
    g = grid(n1, n2)
    for mask in (np.eye(1, n1 * n2, 37).reshape(n1, n2), np.ones((n1, n2))):
        p = int(mask.sum())
        v = synth.random_vectors(p, 2, seed=3)
        ref = direct.masked_matvec(g, mask, th, v.T).T
        with K.Problem(n1, n2, mask) as P:
            got = K.kry_matvec(P.h, K.theta_from_dict(th), v, K.KRY_FP64)
        assert rows_rel(got, ref) <= 1e-12


def test_full_grid_product():
    n1, n2 = 20, 13
    th = THETAS[3]
    g = grid(n1, n2)
    mask = synth.uniform_mask(n1, n2, 0.4, seed=2)
    w = synth.random_vectors(int(mask.sum()), 2, seed=9)
    X = np.zeros((2, n1 * n2))
    X[:, mask.ravel().astype(bool)] = w
    ref = np.stack([direct.full_matvec(g, th, x) for x in X])
    with K.Problem(n1, n2, mask) as P:
        got = K.kry_cov_apply_full(P.h, K.theta_from_dict(th), w, n1 * n2, K.KRY_FP64)
        got32 = K.kry_cov_apply_full(P.h, K.theta_from_dict(th), w, n1 * n2, K.KRY_FP32)
    assert rows_rel(got, ref) <= 1e-12
    assert rows_rel(got32, ref) <= 1e-5


def test_probes_bit_exact():
    from oracle import philox
    from oracle.geometry import observed_cells
    n1, n2 = 30, 41
    mask = synth.uniform_mask(n1, n2, 0.3, seed=4)
    r, c = observed_cells(mask)
    with K.Problem(n1, n2, mask) as P:
        z = K.kry_probes(P.h, K.kry_opts_default(num_probes=7, seed=12345))
        zc = K.kry_probes(P.h, K.kry_opts_default(probe_kind=K.KRY_PROBE_COLOURED, colour_period=3, seed=99))
    np.testing.assert_array_equal(z, philox.probe_matrix(r, c, 7, 12345).T)
    np.testing.assert_array_equal(zc, philox.probe_matrix(r, c, 0, 99, colour_period=3).T)


@pytest.mark.parametrize("rule", ["fast", "smallest"])
def test_embedding_follows_the_rule(rule):
    # the library's embedding follows the stated rules (restated in
    # oracle.geometry.fast_size): 7 x 13, 20 x 30, 40 x 41, 150 x 300,
    # 600 x 700, 513 x 880, 1100 x 2040
    from oracle.geometry import fast_size
    emb = K.KRY_EMBED_FAST if rule == "fast" else K.KRY_EMBED_SMALLEST
    for n1, n2 in ((7, 13), (20, 30), (40, 41), (150, 300), (600, 700), (513, 880), (1100, 2040)):
        with K.Problem(n1, n2, np.ones((n1, n2)), embedding=emb) as P:
            assert (P.N1, P.N2) == (fast_size(2 * n1 - 1, rule), fast_size(2 * n2 - 1, rule)), (n1, n2)
