"""Pins for the oracle's Philox4x32-10 and the streams built on it."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append([int(t, 16) for t in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat())
def test_known_answer_vectors(row):
    c = [np.array([x], dtype=np.uint64) for x in row[:4]]
    out = philox.philox4x32_10(*c, row[4], row[5])
    assert [int(o[0]) for o in out] == row[6:10]


def test_rademacher_is_balanced_signs():
    z = philox.rademacher(np.arange(200000), 3, seed=12345)
    assert set(np.unique(z)) == {-1.0, 1.0}
    assert abs(z.mean()) < 5 * 1 / np.sqrt(z.size)
    # different probes / seeds give different streams
    z2 = philox.rademacher(np.arange(200000), 4, seed=12345)
    z3 = philox.rademacher(np.arange(200000), 3, seed=12346)
    assert abs(np.mean(z * z2)) < 0.02 and abs(np.mean(z * z3)) < 0.02


def test_normals_are_standard_normal():
    x = philox.normals(np.arange(200000), 7, seed=99, domain=philox.DOMAIN_FIELD)
    assert np.all(np.isfinite(x))
    ks = stats.kstest(x, "norm")
    assert ks.pvalue > 1e-3
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1) < 0.02


def test_coloured_probes_have_unit_diagonal_sum():
    rows, cols = np.divmod(np.arange(12 * 10), 10)
    Z = philox.probe_matrix(rows, cols, 0, seed=5, colour_period=3)
    assert Z.shape == (120, 9)
    np.testing.assert_array_equal(np.sum(Z * Z, axis=1), np.ones(120))
    # each cell belongs to exactly one colour
    assert np.all(np.sum(Z != 0, axis=1) == 1)
