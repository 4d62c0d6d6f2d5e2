"""Pins for the irregular-observation oracle: the Wendland weights' values,
the structure of the mapping matrix (at most the four corners of the
enclosing cell, convex rows), exactness on grid points (the gridded model
with a mask), and interpolation by kriging without nugget."""
import numpy as np
import pytest

from oracle import dense, irregular
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta


def test_wendland_values():
    d = np.array([0.0, 0.25, 0.5, 1.0, 1.5])
    # (1 - d)^4 (1 + 4 d) by hand: 1, 0.75^4 * 2, 0.5^4 * 3, 0, 0
    np.testing.assert_allclose(irregular.wendland(d), [1.0, 0.31640625 * 2.0, 0.1875, 0.0, 0.0], rtol=1e-15)


def test_mapping_rows_are_convex_over_the_enclosing_cell():
    g = grid(9, 7)
    locs = synth.irregular_locations(g, 200, seed=3)
    A = irregular.mapping_matrix(g, locs)
    n1, n2 = g[0], g[1]
    assert np.all(A >= 0)
    np.testing.assert_allclose(A.sum(axis=1), 1.0, rtol=1e-14)
    for i, (s1, s2) in enumerate(locs):
        a0, b0 = int(np.floor(s1)), int(np.floor(s2))
        corners = {(min(a, n1 - 1)) * n2 + min(b, n2 - 1) for a in (a0, a0 + 1) for b in (b0, b0 + 1)}
        nz = set(np.flatnonzero(A[i]).tolist())
        assert nz <= corners and 1 <= len(nz) <= 4


def test_observations_on_grid_points_are_the_masked_model():
    n1, n2 = 8, 7
    g = grid(n1, n2)
    th = theta(0.2, 1.5, sigma2=1.4, tau2=0.3, ratio=1.5, angle=0.3)
    mask = synth.uniform_mask(n1, n2, 0.3, seed=5)
    obs = np.flatnonzero(mask.ravel())
    a, b = np.divmod(obs, n2)
    locs = np.stack([a, b], axis=1).astype(np.float64)
    A = irregular.mapping_matrix(g, locs)
    sel = np.zeros_like(A)
    sel[np.arange(obs.size), obs] = 1.0
    np.testing.assert_array_equal(A, sel)
    y = synth.random_vectors(obs.size, 1, seed=6)[0]
    r = irregular.loglik(g, locs, th, y)
    ref = dense.loglik(g, mask, th, y)
    for k in ("loglik", "logdet", "quad"):
        assert r[k] == pytest.approx(ref[k], rel=1e-12)
    tg = np.array([0, 5, 17, 40])
    m1, v1, _ = irregular.krige_cells(g, locs, th, y, tg)
    m2, v2, _ = dense.krige(g, mask, th, y, tg)
    np.testing.assert_allclose(m1, m2, rtol=1e-12)
    np.testing.assert_allclose(v1, v2, rtol=1e-12)


def test_kriging_interpolates_an_on_grid_observation_without_nugget():
    n1, n2 = 10, 9
    g = grid(n1, n2)
    th = theta(0.3, 0.5, sigma2=2.0, tau2=0.0)
    locs = synth.irregular_locations(g, 30, seed=8)
    locs[4] = (3.0, 5.0)  # on grid point (3, 5)
    y = synth.random_vectors(30, 1, seed=9)[0]
    m, v, _ = irregular.krige_cells(g, locs, th, y, np.array([3 * n2 + 5]))
    # (A Sigma A^T is poorly conditioned without a nugget: 1e-6)
    assert m[0] == pytest.approx(y[4], rel=1e-6)
    assert abs(v[0]) <= 1e-6


def test_sparse_mapping_and_sampled_rows_match_the_dense_definition():
    g = grid(11, 9)
    th = theta(0.2, 1.5, sigma2=1.0, tau2=0.3, ratio=2.0, angle=0.4)
    locs = synth.irregular_locations(g, 120, seed=12)
    locs[7] = (10.0, 8.0)  # the far corner
    Ad = irregular.mapping_matrix(g, locs)
    As = irregular.mapping_sparse(g, locs).toarray()
    np.testing.assert_allclose(As, Ad, rtol=1e-15, atol=1e-300)
    v = synth.random_vectors(120, 1, seed=13)[0]
    rows = np.array([0, 7, 33, 119])
    full = irregular.matvec(g, locs, th, v[:, None])[:, 0]
    np.testing.assert_allclose(irregular.matvec_rows(g, locs, th, v, rows), full[rows], rtol=1e-12)
