"""Helpers for the GPU parity tests."""
import numpy as np


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def rows_rel(got, ref):
    """max over vectors of the normwise relative error of each vector"""
    got = np.atleast_2d(got)
    ref = np.atleast_2d(ref)
    return max(normwise(g, r) for g, r in zip(got, ref))
