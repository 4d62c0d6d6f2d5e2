"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark: observation masks, plain random vectors, target cells and grid
sides.  Only numpy's seeded generator is used here; nothing in this module
evaluates a covariance, a transform or any other step of the method.

Workload recipes (shapes and structure of the paper's gridded workloads,
Sec. 4 and 5: regular grids on the unit square, randomly held-out or
cloud-covered cells):
* uniform_mask  -- each cell missing independently, exactly round(frac*n)
                   missing cells chosen without replacement;
* blob_mask     -- union of discs (radius uniform in [rmin, rmax] cells,
                   centre uniform) grown until the missing fraction reaches
                   the target, the last disc shrunk by bisection to land
                   within 0.5 % of it (cloud-cover-like contiguous gaps).
"""
import numpy as np


def uniform_mask(n1, n2, missing_frac, seed):
    rng = np.random.default_rng(seed)
    n = n1 * n2
    k = int(round(missing_frac * n))
    mask = np.ones(n, dtype=np.uint8)
    if k > 0:
        mask[rng.choice(n, size=k, replace=False)] = 0
    return mask.reshape(n1, n2)


def _disc(n1, n2, ci, cj, r):
    ii = np.arange(n1)[:, None]
    jj = np.arange(n2)[None, :]
    return (ii - ci) ** 2 + (jj - cj) ** 2 <= r * r


def blob_mask(n1, n2, missing_frac, seed, rmin=10.0, rmax=80.0):
    rng = np.random.default_rng(seed)
    n = n1 * n2
    target = missing_frac * n
    missing = np.zeros((n1, n2), dtype=bool)
    for _ in range(100000):
        if missing.sum() >= target:
            break
        ci, cj = rng.uniform(0, n1), rng.uniform(0, n2)
        r = rng.uniform(rmin, rmax)
        trial = missing | _disc(n1, n2, ci, cj, r)
        if trial.sum() > target * 1.005:
            lo, hi = 0.0, r
            for _ in range(40):
                mid = 0.5 * (lo + hi)
                if (missing | _disc(n1, n2, ci, cj, mid)).sum() > target * 1.005:
                    hi = mid
                else:
                    lo = mid
            trial = missing | _disc(n1, n2, ci, cj, lo)
        missing = trial
    return (~missing).astype(np.uint8)


def random_vectors(p, m, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, p)).astype(dtype)


def held_out_cells(mask, count, seed):
    """Pick `count` observed cells (row-major ids) to hold out; returns the new
    mask and the held-out ids (sorted)."""
    rng = np.random.default_rng(seed)
    obs = np.flatnonzero(np.asarray(mask).ravel())
    pick = np.sort(rng.choice(obs, size=count, replace=False))
    m2 = np.asarray(mask).copy().ravel()
    m2[pick] = 0
    return m2.reshape(np.asarray(mask).shape), pick


def log_uniform_sides(count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(int)


def covariates(n1, n2, q, seed):
    """q covariate columns over every cell, shape (q, n1, n2): an intercept
    (ones), then the column and row coordinates of the cell centres on the
    unit square, then standard normal columns (the paper's experiments use
    the intercept alone; the others give regressions with several columns)."""
    rng = np.random.default_rng(seed)
    out = np.empty((q, n1, n2))
    jj, ii = np.meshgrid((np.arange(n2) + 0.5) / n2, (np.arange(n1) + 0.5) / n1)
    fixed = [np.ones((n1, n2)), jj, ii]
    for c in range(q):
        out[c] = fixed[c] if c < 3 else rng.standard_normal((n1, n2))
    return out


def irregular_locations(grid, count, seed):
    """count observation locations uniform over the grid's extent, in grid
    units (fractional row, fractional column; grid point (a, b) at (a, b)),
    inside [0, n1 - 1] x [0, n2 - 1] (the paper's third study: a fine field
    thinned at random to an irregular sample)."""
    n1, n2 = grid[0], grid[1]
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0, n1 - 1, count), rng.uniform(0, n2 - 1, count)], axis=1)
