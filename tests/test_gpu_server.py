"""GPU: the request server (continuous batching) gives every request the same
result as running it alone, and reports timing."""
import time

import numpy as np
import pytest

from oracle import sampler
from paper_2012_13133_amd import synth
from tests.oracle_cases import grid, theta

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_2012_13133_amd.kryging")

# embeddings: 128 x 128, 128 x 128, 48 x 128 (a radix-3 side)
SHAPES = [(60, 62, 0.3, "uniform"), (64, 64, 0.2, "blob"), (24, 50, 0.5, "uniform")]


def _problems(ctx):
    probs, masks = [], []
    for i, (n1, n2, frac, kind) in enumerate(SHAPES):
        if kind == "uniform":
            mask = synth.uniform_mask(n1, n2, frac, seed=10 + i)
        else:
            mask = synth.blob_mask(n1, n2, frac, seed=10 + i, rmin=3, rmax=10)
        _, y = sampler.cholesky_field(grid(n1, n2), theta(0.1, 1.5, tau2=0.2), seed=20 + i)
        probs.append(K.kry_problem_create(ctx, n1, n2, mask, y))
        masks.append(mask)
    return probs, masks


def _requests(masks, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        pi = int(rng.integers(len(masks)))
        th = K.theta(sigma2=float(rng.uniform(0.5, 2)), tau2=float(rng.uniform(0.05, 0.5)),
                     range=float(np.exp(rng.uniform(np.log(0.03), np.log(0.2)))),
                     nu=float(rng.choice([0.5, 1.5, 2.5])))
        prec = int(rng.integers(2))
        if rng.uniform() < 0.7:
            # a few option sets so that batching has something to merge
            opts = K.kry_opts_default(lanczos_steps=20, num_probes=6, precision=prec, cg_rtol=1e-8)
            reqs.append(("loglik", pi, th, opts, None))
        else:
            miss = np.flatnonzero(masks[pi].ravel() == 0)
            tg = rng.choice(miss, size=min(12, miss.size), replace=False)
            opts = K.kry_opts_default(precision=prec, cg_rtol=1e-9)
            reqs.append(("krige", pi, th, opts, tg))
    return reqs


def test_server_same_alone_and_in_mix():
    ctx = K.kry_ctx_create()
    probs, masks = _problems(ctx)
    try:
        reqs = _requests(masks, 48, seed=1)
        alone = []
        for kind, pi, th, opts, tg in reqs:
            if kind == "loglik":
                alone.append(K.kry_loglik(probs[pi], th, opts))
            else:
                alone.append(K.kry_krige(probs[pi], th, opts, tg))
        srv = K.kry_server_create(ctx, slots=3, max_batch=8)
        try:
            pend = []
            for i, (kind, pi, th, opts, tg) in enumerate(reqs):
                if kind == "loglik":
                    pend.append(K.kry_server_submit(srv, K.KRY_REQ_LOGLIK, probs[pi], th, opts))
                else:
                    pend.append(K.kry_server_submit(srv, K.KRY_REQ_KRIGE, probs[pi], th, opts, tg, variances=True))
                if i % 7 == 6:
                    time.sleep(0.002)  # staggered arrivals
            resp = [K.kry_server_wait(srv, p) for p in pend]
        finally:
            K.kry_server_destroy(srv)
        batches = 0
        for (kind, pi, th, opts, tg), a, p, r in zip(reqs, alone, pend, resp):
            assert r.status == K.KRY_OK
            assert r.t_submit <= r.t_start <= r.t_end
            batches = max(batches, r.batch)
            if kind == "loglik":
                got = r.loglik.as_dict()
                if r.problems == 1:
                    # batched on its own problem: bit-identical
                    for key in ("loglik", "loglik_profiled", "logdet", "logdet_se", "quad", "cg_iters"):
                        assert got[key] == a[key], (key, got[key], a[key])
                else:
                    _close_to_alone(got, a, opts)
            else:
                np.testing.assert_array_equal(p.outputs["mean_x"], a[0])
                np.testing.assert_array_equal(p.outputs["var_x"], a[1])
                np.testing.assert_array_equal(p.outputs["var_y"], a[2])
        assert batches > 1, "no request was batched with another"
        # requests ran concurrently on different slots
        spans = sorted((r.t_start, r.t_end) for r in resp)
        assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    finally:
        for h in probs:
            K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)


def _close_to_alone(got, a, opts):
    # batched with other problems of the same embedding: the Krylov vectors
    # are padded to the largest observed count, which regroups the dot
    # products' partial sums; equal to rounding (FP32 Lanczos amplifies it)
    tol = 1e-9 if opts.precision == K.KRY_FP64 else 1e-4
    for key in ("loglik", "loglik_profiled", "logdet"):
        assert abs(got[key] - a[key]) <= tol * abs(a[key]), (key, got[key], a[key])
    assert abs(got["quad"] - a["quad"]) <= 1e-7 * a["quad"]
    assert got["cg_relres"] <= opts.cg_rtol


def test_server_merges_problems_sharing_an_embedding():
    # problems 0 and 1 share a 128 x 128 embedding; with one slot busy on a
    # kriging request, likelihood requests on both queue up and run together
    ctx = K.kry_ctx_create()
    probs, masks = _problems(ctx)
    try:
        opts = K.kry_opts_default(lanczos_steps=20, num_probes=6, precision=K.KRY_FP64, cg_rtol=1e-8)
        ths = [K.theta(sigma2=1.0, tau2=0.1 + 0.05 * i, range=0.05 + 0.02 * i, nu=1.5) for i in range(6)]
        alone = [K.kry_loglik(probs[i % 2], th, opts) for i, th in enumerate(ths)]
        miss = np.flatnonzero(masks[1].ravel() == 0)
        srv = K.kry_server_create(ctx, slots=1, max_batch=8)
        try:
            first = K.kry_server_submit(srv, K.KRY_REQ_KRIGE, probs[1], ths[0], K.kry_opts_default(cg_rtol=1e-10),
                                        miss[:64], variances=True)
            pend = [K.kry_server_submit(srv, K.KRY_REQ_LOGLIK, probs[i % 2], th, opts) for i, th in enumerate(ths)]
            K.kry_server_wait(srv, first)
            resp = [K.kry_server_wait(srv, p) for p in pend]
        finally:
            K.kry_server_destroy(srv)
        assert max(r.problems for r in resp) == 2
        for r, a in zip(resp, alone):
            assert r.status == K.KRY_OK
            _close_to_alone(r.loglik.as_dict(), a, opts)
    finally:
        for h in probs:
            K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)


def test_server_admission_by_footprint():
    ctx = K.kry_ctx_create()
    probs, masks = _problems(ctx)
    try:
        opts = K.kry_opts_default(lanczos_steps=10, num_probes=4)
        th = K.theta(range=0.1, nu=0.5, tau2=0.2)
        # a budget far below one request's footprint is refused at submit
        srv = K.kry_server_create(ctx, slots=2, hbm_budget_bytes=1 << 10)
        try:
            with pytest.raises(K.KryError) as e:
                K.kry_server_submit(srv, K.KRY_REQ_LOGLIK, probs[1], th, opts)
            assert e.value.status == K.KRY_ENOMEM
        finally:
            K.kry_server_destroy(srv)
        # the reference values first: the problems' own workspaces are then
        # in place, and what the server allocates on top is its slots'
        ref = [K.kry_loglik(probs[i % 3], th, opts)["loglik"] for i in range(6)]
        kopts = K.kry_opts_default(cg_rtol=1e-9)
        tg = [np.flatnonzero(m.ravel() == 0)[:8] for m in masks]
        kref = [K.kry_krige(probs[i], th, kopts, tg[i], want_var=True) for i in range(3)]
        # a budget that fits one request at a time still completes every
        # request, and the slots' device memory (kept between requests) never
        # exceeds it: an idle slot's workspace is released to admit another
        def submit_all(srv):
            pend = [K.kry_server_submit(srv, K.KRY_REQ_LOGLIK, probs[i % 3], th, opts) for i in range(6)]
            pend += [K.kry_server_submit(srv, K.KRY_REQ_KRIGE, probs[i], th, kopts, targets=tg[i], variances=True)
                     for i in range(3)]
            return pend, [K.kry_server_wait(srv, p) for p in pend]

        # every request's admission bound, from an unlimited server
        srv = K.kry_server_create(ctx, slots=3, max_batch=1)
        try:
            _, r0 = submit_all(srv)
        finally:
            K.kry_server_destroy(srv)
        fps = [r.footprint_bytes for r in r0]
        # room for the largest request but not for two of them: slots must
        # give back what they keep for others to start
        budget = max(fps) + min(fps) // 2
        base, _ = K.kry_ctx_memory(ctx, reset_peak=True)
        srv = K.kry_server_create(ctx, slots=3, hbm_budget_bytes=budget, max_batch=1)
        try:
            pend, resp = submit_all(srv)
            assert all(r.status == K.KRY_OK for r in resp)
            assert [r.loglik.loglik for r in resp[:6]] == ref
            for pd, (m, vx, vy) in zip(pend[6:], kref):
                np.testing.assert_array_equal(pd.outputs["mean_x"], m)
                np.testing.assert_array_equal(pd.outputs["var_x"], vx)
            _, peak = K.kry_ctx_memory(ctx)
            assert peak - base <= budget, (peak - base, budget)
        finally:
            K.kry_server_destroy(srv)
    finally:
        for h in probs:
            K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)


def test_server_footprint_bounds_each_request():
    # the admission bound of a request covers the workspace it needs: run
    # each kind alone on a fresh one-slot server, whose workspace then holds
    # exactly what that request allocated
    ctx = K.kry_ctx_create()
    probs, masks = _problems(ctx)
    try:
        th = K.theta(range=0.1, nu=1.5, tau2=0.2)
        cases = [
            ("loglik", K.kry_opts_default(lanczos_steps=12, num_probes=5)),
            ("loglik", K.kry_opts_default(lanczos_steps=12, num_probes=5, precision=1, reorth=1)),
            ("loglik", K.kry_opts_default(lanczos_steps=8, num_probes=3, solver=1, gk_steps=10)),
            ("loglik", K.kry_opts_default(lanczos_steps=8, num_probes=3, probe_kind=K.KRY_PROBE_COLOURED,
                                          colour_period=3, lanczos_rtol=1e-6, lanczos_max_steps=40)),
            ("krige", K.kry_opts_default(cg_rtol=1e-9)),
            ("krige", K.kry_opts_default(cg_rtol=1e-9, precision=1)),
        ]
        for pi in range(3):
            miss = np.flatnonzero(masks[pi].ravel() == 0)
            for kind, opts in cases:
                srv = K.kry_server_create(ctx, slots=1)
                try:
                    if kind == "loglik":
                        pd = K.kry_server_submit(srv, K.KRY_REQ_LOGLIK, probs[pi], th, opts)
                    else:
                        pd = K.kry_server_submit(srv, K.KRY_REQ_KRIGE, probs[pi], th, opts, targets=miss[:20],
                                                 variances=True)
                    r = K.kry_server_wait(srv, pd)
                    assert r.status == K.KRY_OK
                    assert 0 < r.workspace_bytes <= r.footprint_bytes, (pi, kind, r.workspace_bytes,
                                                                        r.footprint_bytes)
                finally:
                    K.kry_server_destroy(srv)
    finally:
        for h in probs:
            K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)


def test_shift_shared_batch_same_on_a_problem_and_through_the_server():
    # The FP32 shift-shared call on a problem and the same points as requests
    # on views with the server's slot workspaces give the same results, bit
    # for bit.
    ctx = K.kry_ctx_create()
    probs, masks = _problems(ctx)
    try:
        pts = [K.theta(sigma2=1.0, tau2=e, range=r, nu=1.5) for r in (0.05, 0.12) for e in (0.03, 0.2, 0.6)]
        opts = K.kry_opts_default(lanczos_steps=25, num_probes=6, precision=K.KRY_FP32, shift_share=1, reorth=1,
                                  cg_rtol=1e-9)
        direct = K.kry_loglik_batch(probs[1], pts, opts)
        srv = K.kry_server_create(ctx, slots=2, max_batch=1)
        try:
            pend = [K.kry_server_submit(srv, K.KRY_REQ_LOGLIK, probs[1], t, opts) for t in pts]
            resp = [K.kry_server_wait(srv, p) for p in pend]
        finally:
            K.kry_server_destroy(srv)
        for d, r in zip(direct, resp):
            assert r.status == K.KRY_OK
            for key in ("loglik", "logdet", "quad", "cg_iters", "lanczos_steps_used"):
                assert r.loglik.as_dict()[key] == d[key], key
    finally:
        for h in probs:
            K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)
