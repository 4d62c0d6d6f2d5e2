"""Textbook conjugate gradients (Hestenes-Stiefel) for K w = b.

Test infrastructure only (see ``oracle/__init__``).

The quadratic term y^T K^{-1} y and the kriging weights need K^{-1} applied
to vectors; Sec. 3.2 reduces that to products with the covariance.  CG is
the standard Krylov solver for a symmetric positive definite K.  Stops when
||r|| <= rtol ||b||.
"""
import numpy as np


def cg(matvec, b, rtol=1e-8, maxit=10000):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    bn = float(np.sqrt(b @ b))
    it = 0
    while np.sqrt(rr) > rtol * bn and it < maxit:
        w = matvec(p)
        a = rr / float(p @ w)
        x = x + a * p
        r = r - a * w
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, float(np.sqrt(rr) / bn) if bn > 0 else 0.0
