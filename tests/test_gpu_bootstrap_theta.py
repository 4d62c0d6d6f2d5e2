"""GPU parity for the parametric bootstrap of the parameter estimates: the
same simulated data sets as the oracle, each refitted, and the problem's
data restored afterwards."""
import numpy as np
import pytest

from oracle import bootstrap, sampler
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_2012_13133_amd.kryging")


def test_parameter_bootstrap_matches_oracle_and_restores_the_data():
    n1 = n2 = 16
    g = grid(n1, n2)
    th = theta(0.15, 0.5, sigma2=1.0, tau2=0.3)
    mask = synth.uniform_mask(n1, n2, 0.2, seed=5)
    _, y = sampler.cholesky_field(g, th, seed=6)
    B = 3
    opts = K.kry_opts_default(lanczos_steps=80, probe_kind=K.KRY_PROBE_COLOURED, colour_period=16, cg_rtol=1e-10,
                              seed=91)
    with K.Problem(n1, n2, mask, y) as P:
        t = K.theta_from_dict(th)
        before = K.kry_loglik(P.h, t, opts)
        N = K.kry_psd_torus(P.h, t)
        est, sd = K.kry_bootstrap_theta(P.h, t, opts, B, xtol=1e-4, maxiter=300)
        after = K.kry_loglik(P.h, t, opts)
    assert after["quad"] == before["quad"] and after["logdet"] == before["logdet"]
    ref = bootstrap.bootstrap_theta(g, mask, th, B, N[0], N[1], 91)
    for b in range(B):
        # colour period 16 covers the grid: the log-det is exact, so each optimum is the dense one
        assert abs(np.log(est[b].range) - np.log(ref[b, 0])) < 5e-3, b
        assert abs(np.log(est[b].tau2 / est[b].sigma2) - np.log(ref[b, 1])) < 5e-3, b
    lr = np.log([e.range for e in est])
    assert sd[0] == pytest.approx(np.std(lr, ddof=1), rel=1e-12)
