"""Pins for the oracle's Matern correlation (Sec. 2) and anisotropic distance."""
import mpmath
import numpy as np
import pytest

from oracle.matern import aniso_distance, matern, matern_half_integer

D = np.array([0.0, 1e-6, 1e-3, 0.01, 0.05, 0.1, 0.37, 1.0, 2.5])


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
@pytest.mark.parametrize("rho", [0.02, 0.1, 0.7])
def test_half_integer_closed_forms(nu, rho):
    a = matern(D, rho, nu)
    b = matern_half_integer(D, rho, nu)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("nu", [0.8, 1.0, 2.0, 3.3])
def test_general_nu_against_mpmath(nu):
    mpmath.mp.dps = 50
    rho = 0.13
    for d in D[1:]:
        x = mpmath.sqrt(2 * mpmath.mpf(nu)) * mpmath.mpf(d) / mpmath.mpf(rho)
        ref = 2 ** (1 - mpmath.mpf(nu)) / mpmath.gamma(nu) * x ** nu * mpmath.besselk(nu, x)
        got = matern(np.array([d]), rho, nu)[0]
        assert abs(got - float(ref)) <= 1e-13 * max(abs(float(ref)), 1e-300)


def test_value_one_at_zero_and_decreasing():
    for nu in (0.5, 1.0, 1.5, 2.5):
        m = matern(np.linspace(0, 1, 200), 0.1, nu)
        assert m[0] == 1.0
        assert np.all(np.diff(m) <= 0)
        assert np.all(m > 0) and m[-1] < 1e-3


def test_aniso_distance_axes_and_symmetry():
    ang = np.pi / 6
    u = np.array([np.cos(ang), np.sin(ang)])
    w = np.array([-np.sin(ang), np.cos(ang)])
    # along the major axis the distance is the Euclidean length
    assert abs(aniso_distance(*(0.3 * u), ratio=2.0, angle=ang) - 0.3) < 1e-15
    # across it, stretched by the ratio
    assert abs(aniso_distance(*(0.3 * w), ratio=2.0, angle=ang) - 0.6) < 1e-15
    rng = np.random.default_rng(0)
    h = rng.standard_normal((2, 50))
    np.testing.assert_allclose(aniso_distance(h[0], h[1], 2.0, ang), aniso_distance(-h[0], -h[1], 2.0, ang))
    np.testing.assert_allclose(aniso_distance(h[0], h[1], 1.0, ang), np.hypot(h[0], h[1]), rtol=1e-15)
