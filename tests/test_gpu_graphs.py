"""GPU: CG iteration blocks replayed from captured HIP graphs give the same
bits as launching every kernel directly, replay after replay."""
import numpy as np
import pytest

from paper_2012_13133_amd import synth
from tests.oracle_cases import theta

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_2012_13133_amd.kryging")

TH = theta(0.15, 1.5, tau2=0.05)


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_graph_replays_match_direct_launches(precision):
    n1, n2 = 96, 80
    mask = synth.uniform_mask(n1, n2, 0.3, seed=7)
    th = K.theta_from_dict(TH)
    opts = K.kry_opts_default(precision=precision, cg_rtol=1e-10)
    with K.Problem(n1, n2, mask) as P:
        B = synth.random_vectors(P.p, 3, seed=8)
        K.kry_set_graphs(P.ctx, False)
        x0, it0, rr0 = K.kry_solve(P.h, th, opts, B)
        assert min(it0) > 48  # several replayed blocks
        K.kry_set_graphs(P.ctx, True)
        for rep in range(3):
            x, it, rr = K.kry_solve(P.h, th, opts, B)
            assert np.array_equal(x, x0) and list(it) == list(it0) and list(rr) == list(rr0), rep
            K.kry_matvec(P.h, th, B[:1])  # eager work between replays


@pytest.mark.parametrize("precision", [0, 1])
def test_loglik_and_multi_with_and_without_graphs(precision):
    n1, n2 = 64, 72
    mask = synth.uniform_mask(n1, n2, 0.25, seed=9)
    y = synth.random_vectors(n1 * n2, 1, seed=10)[0]
    opts = K.kry_opts_default(lanczos_steps=20, num_probes=4, precision=precision, cg_rtol=1e-9)
    th = K.theta_from_dict(TH)
    ctx = K.kry_ctx_create()
    hs = [K.kry_problem_create(ctx, n1, n2, mask, y), K.kry_problem_create(ctx, 60, 70, mask[:60, :70], y[:4200])]
    try:
        out = {}
        for g in (False, True):
            K.kry_set_graphs(ctx, g)
            out[g] = (K.kry_loglik(hs[0], th, opts), K.kry_loglik_multi(hs, [th, th], opts))
        assert out[True][0] == out[False][0]
        assert out[True][1] == out[False][1]
        assert out[True][0]["cg_iters"] > 32
    finally:
        for h in hs:
            K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)
