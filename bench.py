"""Benchmark of the Kryging hot path on one MI355X.

Workload (the metric shape): a 1024 x 1024 grid on the unit square with 30 %
of the cells missing uniformly at random (p = 734,003 observed cells), data
drawn by circulant embedding (Matern nu = 1.5, range 0.05) on a PSD torus plus
nugget noise (ratio 0.2), synthetic and seeded.

One step = one pass of the whole hot path over one batch of parameter points:
kry_loglik_batch over the 10 x 10 grid of range in [0.01, 0.2] x nugget ratio
in [0.01, 1] (log-spaced) with shift sharing -- lag grid and spectrum per
range, Rademacher probes, batched Lanczos (20 probes x 50 steps,
reorthogonalised; FP32 products, FP64 coefficients) on the nugget-free
covariance, Gauss quadrature per point, FP64 multi-shift CG to 1e-8 per range
and the likelihood assembly.  `value` is the masked products per second
applied inside the timed steps.  The JSON line also carries the likelihood
evaluations per second, the plain FP64 single-point form on a stratified
sample of the same grid and the batched form's accuracy against it, the
isolated batched product rates, the roofline of the dominant kernel (with the
counter-measured traffic from the committed profile), the served form, the
multi-problem form and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "masked BTTB matvecs/s + profile-loglik evals/s at 1024² grid; serve p50/p99"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--points", type=int, default=100, help="parameter points per step (a square grid)")
    ap.add_argument("--probes", type=int, default=20)
    ap.add_argument("--lanczos", type=int, default=50)
    ap.add_argument("--cg-rtol", type=float, default=1e-8)
    ap.add_argument("--cg-maxit", type=int, default=100000)
    ap.add_argument("--reorth", type=int, default=1, help="full reorthogonalisation in Lanczos (FP64 coefficients)")
    ap.add_argument("--mv-batch", type=int, default=32)
    ap.add_argument("--mv-reps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--matvec-only", action="store_true", help="only the isolated batched product (profiling)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=100)
    ap.add_argument("--serve-targets", type=int, default=4, help="kriging targets per request (with exact variances)")
    ap.add_argument("--serve-plain-sample", type=int, default=100,
                    help="requests of the stream also run in the plain FP64 form (accuracy and rate)")
    ap.add_argument("--serve-sides", type=str, default="128,2048",
                    help="grid sides log-uniform in [lo,hi] for the served stream (the full served workload uses 128,2048)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=int, default=64, help="the server's HBM budget")
    ap.add_argument("--serve-sweep", type=str, default="0.8", help="arrival rates, fractions of saturation")
    ap.add_argument("--multi", type=int, default=64, help="independent problems in the multi-problem form (0: skip)")
    ap.add_argument("--multi-sides", type=str, default="64,1024")
    ap.add_argument("--multi-only", action="store_true", help="only the multi-problem form")
    ap.add_argument("--serve-only", action="store_true", help="only the served form")
    ap.add_argument("--no-c4", action="store_true", help="skip the large anisotropic end-to-end problem")
    ap.add_argument("--c4-only", action="store_true", help="only the large anisotropic end-to-end problem")
    ap.add_argument("--c4-n", type=int, default=2048)
    ap.add_argument("--c4-probes", type=int, default=8)
    ap.add_argument("--c4-steps", type=int, default=1024)
    ap.add_argument("--c4-lanczos-rtol", type=float, default=0.0)
    ap.add_argument("--c4-lanczos-max", type=int, default=1024)
    ap.add_argument("--c4-cg-rtol", type=float, default=1e-7)
    ap.add_argument("--c4-maxiter", type=int, default=20)
    ap.add_argument("--c4-xtol", type=float, default=1e-2)
    ap.add_argument("--c4-boot", type=int, default=20)
    ap.add_argument("--c4-exact", type=int, default=32, help="missing cells with exact variances")
    ap.add_argument("--no-ext", action="store_true", help="skip the extension rows (irregular data, covariates, "
                                                          "the paper's objective, posterior variance)")
    ap.add_argument("--ext-only", action="store_true", help="only the extension rows")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic(stage):
    """HBM bytes per launch of an FP32 stage kernel ("a", "b" or "c"; batch
    32, 1024 x 1024 workload) from the committed rocprofv3 counter summary, or
    None when the kernel sources have changed since those counters were
    taken."""
    import hashlib
    import re

    try:
        with open(os.path.join(ROOT, "profiles", "masked_product_1024sq_b32.md")) as f:
            txt = f.read()
    except OSError:
        return None
    vals = dict(re.findall(r"^(traffic_stage_[abc]_fp32_bytes|kernel_sources_sha256): (\S+)$", txt, re.M))
    h = hashlib.sha256()
    for name in ("conv.hip", "fftk.hpp", "fftm.hpp", "fft.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2012_13133_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    key = "traffic_stage_%s_fp32_bytes" % stage
    if vals.get("kernel_sources_sha256") != h.hexdigest() or key not in vals:
        return None
    return int(vals[key])


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2012_13133_amd import kryging as K, synth

    if args.multi_only:
        print(json.dumps({"multi": multi_bench(args, K, synth, np)}))
        return
    if args.serve_only:
        print(json.dumps({"serve": serve_bench(args, K, synth, np)}))
        return
    if args.ext_only:
        print(json.dumps({"extensions": ext_bench(args, K, synth, np)}))
        return
    if args.c4_only:
        print(json.dumps({"config4": config4_bench(args, K, synth, np)}))
        return
    n = args.n
    nu, rho, eta = 1.5, 0.05, 0.2
    mask = synth.uniform_mask(n, n, 0.3, seed=101)
    th0 = K.theta(sigma2=1.0, tau2=eta, range=rho, nu=nu)
    P = K.Problem(n, n, mask)
    log("problem: %dx%d p=%d embedding %dx%d" % (n, n, P.p, P.N1, P.N2))
    # data: circulant-embedding field + nugget noise (setup, untimed)
    N = K.kry_psd_torus(P.h, th0)
    x, _ = K.kry_sample(P.h, th0, N[0], N[1], 202, 0, 1, n, n)
    rng = np.random.default_rng(303)
    y = x[0] + np.sqrt(eta) * rng.standard_normal((n, n))
    K.kry_problem_set_data(P.h, y)
    log("data sampled on a %dx%d torus" % N)

    # ---- launch configuration picked by the autotuner for this embedding ----
    tuning = {"fp32": K.kry_autotune(P.h, K.KRY_FP32, args.mv_batch),
              "fp64": K.kry_autotune(P.h, K.KRY_FP64, args.mv_batch),
              # products of at most 8 vectors (the multi-shift CG's, one vector per range group)
              "fp32_small": K.kry_autotune(P.h, K.KRY_FP32, 4),
              "fp64_small": K.kry_autotune(P.h, K.KRY_FP64, 4)}
    log("autotuned: %s" % tuning)

    # ---- isolated batched masked product (FP32 and FP64) with stage timing ----
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()  # default priority; the library launches on it
    torch.cuda.set_stream(stream)
    sp = stream.cuda_stream
    # products per second across batch sizes (the configuration tuned above)
    sweep = {}
    for prec, dt, key in ((K.KRY_FP32, torch.float32, "fp32"), (K.KRY_FP64, torch.float64, "fp64")):
        sweep[key] = {}
        for Bs in (1, 8, 32, 128):
            vin = torch.randn(Bs, P.p, device=dev, dtype=dt)
            vout = torch.empty_like(vin)
            K.kry_matvec_device(P.h, th0, prec, Bs, vin.data_ptr(), vout.data_ptr(), sp)
            reps = max(4, 640 // Bs) if Bs < 32 else 10
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                K.kry_matvec_device(P.h, th0, prec, Bs, vin.data_ptr(), vout.data_ptr(), sp)
            e1.record(stream)
            torch.cuda.synchronize()
            sweep[key][str(Bs)] = Bs * reps / (e0.elapsed_time(e1) / 1e3)
            del vin, vout
        torch.cuda.empty_cache()
    log("matvec products/s by batch: %s" % {k: {b: round(v) for b, v in d.items()} for k, d in sweep.items()})

    mv = {}
    for prec, dt in ((K.KRY_FP32, torch.float32), (K.KRY_FP64, torch.float64)):
        B = args.mv_batch
        vin = torch.randn(B, P.p, device=dev, dtype=dt)
        vout = torch.empty_like(vin)
        for _ in range(3):
            K.kry_matvec_device(P.h, th0, prec, B, vin.data_ptr(), vout.data_ptr(), sp)
        torch.cuda.synchronize()
        # an event between consecutive launches: the total and each launch's time
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.mv_reps + 1)]
        evs[0].record(stream)
        for i in range(args.mv_reps):
            K.kry_matvec_device(P.h, th0, prec, B, vin.data_ptr(), vout.data_ptr(), sp)
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        ms_total = evs[0].elapsed_time(evs[-1])
        per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.mv_reps)])
        # stage times in a second run of as many launches (the library's events
        # between stages cost a few per cent of the rate, so they are kept out
        # of the run above)
        K.kry_profile_begin(P.ctx)
        for i in range(args.mv_reps):
            K.kry_matvec_device(P.h, th0, prec, B, vin.data_ptr(), vout.data_ptr(), sp)
        torch.cuda.synchronize()
        st_ms, st_n, st_vec = K.kry_profile_end(P.ctx)
        rate = B * args.mv_reps / (ms_total / 1e3)
        mv[prec] = dict(batch=B, matvecs_per_s=rate, ms_per_launch=ms_total / args.mv_reps,
                        launch_ms_median=float(np.median(per)), launch_ms_p10=float(np.percentile(per, 10)),
                        launch_ms_p90=float(np.percentile(per, 90)),
                        stage_ms=[float(v / max(c, 1)) for v, c in zip(st_ms, st_n)])
        log("matvec %s B=%d: %.0f matvecs/s, stages A/B/C ms %s" %
            ("fp32" if prec == K.KRY_FP32 else "fp64", B, rate, mv[prec]["stage_ms"]))
        del vin, vout
    torch.cuda.empty_cache()
    if args.matvec_only:
        # a plain device copy of known size: the reference that scales the HBM
        # counters (FETCH_SIZE, WRITE_SIZE) read under a profiler
        src = torch.empty(1 << 28, device=dev, dtype=torch.float32).uniform_()
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(json.dumps({"matvec_batched": {"fp32": mv[K.KRY_FP32], "fp64": mv[K.KRY_FP64]},
                          "matvec_by_batch": sweep}))
        P.close()
        return

    # ---- algorithmic bytes of the dominant kernel (the slowest FP32 stage: B or C, about equal) ----
    p = P.p
    M = P.N2 // 2
    cs = 8  # complex FP32
    Bv = args.mv_batch
    inter = n * (M + 1) * cs                   # one vector's half-spectrum intermediate (n1 rows)
    lam_bytes = (M + 1) * P.N1 * 4             # FP32 spectrum, read once per launch
    stage_b_bytes = Bv * 2 * inter + lam_bytes
    stage_ms = mv[K.KRY_FP32]["stage_ms"]
    dom = int(np.argmax(stage_ms))
    words = n * ((n + 31) // 32) * 8           # mask words + word offsets
    stage_bytes = [Bv * (4 * p + inter) + words, stage_b_bytes, Bv * (inter + 4 * p + 4 * p) + words]
    achieved = stage_bytes[dom] / (stage_ms[dom] / 1e3) / 1e9
    # the same kernel against the vector ALU: 5 L log2 L flops per complex
    # transform of length L (row stages: M-point transforms plus the 10-flop
    # split or merge per output; column stage: forward and inverse N1-point
    # transforms plus the 2-flop spectrum scaling per point), FP32 without
    # packed instructions: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
    M_ = P.N2 // 2
    lgM, lgN1 = int(np.log2(M_)), int(np.log2(P.N1))
    row_fl = n * (5 * M_ * lgM + 10 * (M_ + 1))
    col_fl = (M_ + 1) * (2 * 5 * P.N1 * lgN1 + 2 * P.N1)
    stage_flops = [Bv * row_fl, Bv * col_fl, Bv * row_fl]
    ALU_PEAK_TFS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
    alu_achieved = stage_flops[dom] / (stage_ms[dom] / 1e3) / 1e12
    mv_bytes = sum(stage_bytes)
    mv_achieved = mv_bytes / (sum(stage_ms) / 1e3) / 1e9

    # ---- timed steps: batched likelihood over the (range, nugget) grid ----
    side = int(round(np.sqrt(args.points)))
    rhos = np.geomspace(0.01, 0.2, side)
    etas = np.geomspace(0.01, 1.0, side)
    thetas = [K.theta(sigma2=1.0, tau2=float(e), range=float(r), nu=nu) for r in rhos for e in etas]
    opts32 = K.kry_opts_default(lanczos_steps=args.lanczos, num_probes=args.probes, seed=303,
                                precision=K.KRY_FP32, cg_rtol=args.cg_rtol, cg_maxit=args.cg_maxit, shift_share=1,
                                reorth=args.reorth)
    for w in range(args.warmup):
        K.kry_loglik_batch(P.h, thetas, opts32)
        log("warmup %d done" % w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = None
    for s in range(args.steps):
        results = K.kry_loglik_batch(P.h, thetas, opts32)
        log("step %d done" % s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # products actually applied per step: per range group, probes x Lanczos
    # steps and the multi-shift CG's base iterations (its slowest nugget)
    groups = [results[i * side:(i + 1) * side] for i in range(side)]
    per_step = sum(args.probes * max(r["lanczos_steps_used"] for r in g_) + max(r["cg_iters"] for r in g_)
                   for g_ in groups)
    matvecs_per_s = per_step * args.steps / dt
    evals_per_s = len(thetas) * args.steps / dt
    log("batched: %.2f s per step, %.1f evals/s, cg iters per range %s" %
        (dt / args.steps, evals_per_s, [max(r["cg_iters"] for r in g_) for g_ in groups]))

    # ---- plain FP64 single-point form on a stratified sample of the grid ----
    plain = None
    if not args.no_plain:
        opts64 = K.kry_opts_default(lanczos_steps=args.lanczos, num_probes=args.probes, seed=303,
                                    precision=K.KRY_FP64, cg_rtol=args.cg_rtol, cg_maxit=args.cg_maxit,
                                    reorth=args.reorth)
        stride = max(1, side // 2)
        sample = [i * side + j for i in range(side) for j in range(side) if (i + j) % stride == 0]
        errs, errs_p, secs, its = [], [], [], []
        for k in sample:
            t1 = time.perf_counter()
            r64 = K.kry_loglik(P.h, thetas[k], opts64, allow_noconv=True)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t1)
            its.append(r64["cg_iters"])
            errs.append(abs(results[k]["loglik"] - r64["loglik"]) / abs(r64["loglik"]))
            errs_p.append(abs(results[k]["loglik_profiled"] - r64["loglik_profiled"]) / abs(r64["loglik_profiled"]))
            log("plain fp64 point %d: %.2f s, %d CG iterations, rel err %.2e" % (k, secs[-1], its[-1], errs[-1]))
        plain = dict(evals_per_s=len(sample) / sum(secs), sample_points=len(sample),
                     sample="grid points (i, j) with (i + j) mod %d == 0: every range and every nugget equally often"
                            % stride,
                     seconds=sum(secs), cg_iters=its,
                     batched_rel_err_vs_fp64_max=max(errs), batched_rel_err_vs_fp64_profiled_max=max(errs_p))
        log("plain fp64: %.2f evals/s over %d sampled points; batched max rel err %.2e (profiled %.2e)" %
            (plain["evals_per_s"], len(sample), max(errs), max(errs_p)))

    # ---- served form: Poisson stream of likelihood / kriging requests ----
    p_obs, emb = P.p, [P.N1, P.N2]
    serve = None
    if not args.no_serve:
        P.close()
        P = None
        torch.cuda.empty_cache()
        serve = serve_bench(args, K, synth, np)

    # ---- multi-problem form: independent grids of different sizes ----
    multi = multi_bench(args, K, synth, np) if args.multi > 0 else None

    # ---- extension rows ----
    ext = None if args.no_ext else ext_bench(args, K, synth, np)

    # ---- the large anisotropic problem end to end (2048 x 2048) ----
    c4 = None if args.no_c4 else config4_bench(args, K, synth, np)

    # ---- CPU oracle on a bounded sample ----
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(n, mask, dict(range=rho, nu=nu, sigma2=1.0, tau2=eta), p_obs)

    out = {
        "metric": METRIC,
        "value": matvecs_per_s,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {
            "workload": "1024x1024 grid, 30%% uniform missing (p=%d), Matern nu=1.5, data at range 0.05 nugget "
                        "ratio 0.2; one step = kry_loglik_batch over the %dx%d grid of range in [0.01, 0.2] x nugget "
                        "ratio in [0.01, 1] (log-spaced), %d probes x %d Lanczos steps, CG to %g; FP32 transforms "
                        "in Lanczos, FP64 multi-shift CG, FP64 scalars" % (p_obs, side, side, args.probes,
                                                                          args.lanczos, args.cg_rtol),
            "global_batch": len(thetas) * args.probes,
            "embedding": emb,
        },
        "loglik_evals_per_s": evals_per_s,
        "tuning": tuning,
        "matvec_by_batch": sweep,
        "matvec_batched": {"fp32": mv[K.KRY_FP32], "fp64": mv[K.KRY_FP64],
                           "bytes_per_launch_fp32": mv_bytes, "achieved_GBs_fp32": mv_achieved},
        "plain_fp64": plain,
        "batched_vs_plain_evals": (evals_per_s / plain["evals_per_s"]) if plain else None,
        "batched_cg_iters_per_range": [max(r["cg_iters"] for r in g_) for g_ in groups],
        "products_per_step": per_step,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("abc"[dom]) if (Bv == 32 and n == 1024) else None,
                     "kernel": ["stage A (row transform)", "stage B (column transform x spectrum)",
                                "stage C (inverse row transform, gather)"][dom],
                     "bytes_per_launch": stage_bytes[dom], "launch_ms": stage_ms[dom], "batch": Bv},
        "roofline_alu": {"bound": "alu", "achieved": alu_achieved, "peak": ALU_PEAK_TFS, "unit": "TFLOP/s",
                         "frac": alu_achieved / ALU_PEAK_TFS, "flops_per_launch": stage_flops[dom],
                         "note": "same kernel; FP32 vector rate without packed instructions"},
        "cpu_baseline": cpu,
        "results_first_point": results[0],
    }
    out["serve"] = serve
    out["multi"] = multi
    out["extensions"] = ext
    out["config4"] = c4
    print(json.dumps(out))
    if P is not None:
        P.close()


def serve_bench(args, K, synth, np):
    """Served form: a Poisson stream of requests (70 % likelihood, 30 % kriging
    at 16 held-out cells with exact variances) on grids with sides log-uniform
    in the given range, 10-50 % missing (uniform or blob masks), nu in
    {0.5, 1.5, 2.5}.  Problems are created once and stay device-resident; the
    server runs under a finite HBM budget.  Reports p50/p99 latency (submit to
    completion) and throughput with Poisson arrivals at 50, 80 and 100 % of
    the measured saturation rate (80 % is the headline).  Served requests run
    the precision form (FP32 transforms) at the same CG tolerance as the plain
    FP64 form; a stratified sample of the stream (every k-th request) is also
    run in the plain FP64 single-request form on the same GPU, for its rate
    and for each request's relative log-likelihood difference."""
    lo, hi = (int(x) for x in args.serve_sides.split(","))
    rng = np.random.default_rng(505)
    ctx = K.kry_ctx_create()
    nprob = 8
    sides = synth.log_uniform_sides(nprob, lo, hi, seed=506)
    probs, masks = [], []
    t_setup = time.perf_counter()
    for i, n in enumerate(sides):
        frac = float(rng.uniform(0.1, 0.5))
        if rng.uniform() < 0.5:
            mask = synth.uniform_mask(int(n), int(n), frac, seed=600 + i)
        else:
            mask = synth.blob_mask(int(n), int(n), frac, seed=600 + i, rmin=max(2.0, n / 100), rmax=max(4.0, n / 12))
        th = K.theta(sigma2=1.0, tau2=0.2, range=0.05, nu=1.5)
        h = K.kry_problem_create(ctx, int(n), int(n), mask)
        Nt = K.kry_psd_torus(h, th)
        x, _ = K.kry_sample(h, th, Nt[0], Nt[1], 700 + i, 0, 1, int(n), int(n))
        K.kry_problem_set_data(h, x[0] + np.sqrt(0.2) * rng.standard_normal((int(n), int(n))))
        probs.append(h)
        masks.append(mask)
    log("serve: %d problems, sides %s (%.1f s set-up)" % (nprob, [int(v) for v in sides],
                                                          time.perf_counter() - t_setup))
    reqs = []
    for _ in range(args.serve_requests):
        pi = int(rng.integers(nprob))
        th = K.theta(sigma2=1.0, tau2=float(np.exp(rng.uniform(np.log(0.05), np.log(0.5)))),
                     range=float(np.exp(rng.uniform(np.log(0.02), np.log(0.2)))), nu=float(rng.choice([0.5, 1.5, 2.5])))
        if rng.uniform() < 0.7:
            reqs.append(("loglik", pi, th, None))
        else:
            miss = np.flatnonzero(masks[pi].ravel() == 0)
            reqs.append(("krige", pi, th, rng.choice(miss, size=args.serve_targets, replace=False)))
    # served likelihoods: FP32 Lanczos products with reorthogonalisation (FP64
    # coefficients) and the FP64 multi-shift CG; served kriging: FP64 solves
    # (on these grids the condition numbers reach 1e6-1e7, where FP32 solves
    # inside FP64 refinement take more iterations than they save).  The plain
    # form: everything FP64, the same probes, steps, reorthogonalisation and
    # CG tolerance.
    common = dict(lanczos_steps=30, num_probes=10, reorth=1, cg_rtol=1e-8, cg_maxit=200000)
    o32 = K.kry_opts_default(precision=K.KRY_FP32, shift_share=1, **common)
    o64 = K.kry_opts_default(precision=K.KRY_FP64, **common)
    ok = K.kry_opts_default(precision=K.KRY_FP64, **common)
    budget = args.serve_budget_gib << 30

    def submit(srv, r, opts):
        kind, pi, th, tg = r
        if kind == "loglik":
            return K.kry_server_submit(srv, K.KRY_REQ_LOGLIK, probs[pi], th, opts)
        return K.kry_server_submit(srv, K.KRY_REQ_KRIGE, probs[pi], th, ok, tg, variances=True)

    base_mem, _ = K.kry_ctx_memory(ctx, reset_peak=True)
    srv = K.kry_server_create(ctx, slots=args.serve_slots, hbm_budget_bytes=budget, max_batch=16)
    try:
        # saturation: everything submitted at once
        t0 = time.perf_counter()
        pend0 = [submit(srv, r, o32) for r in reqs]
        resp0 = []
        for j, p_ in enumerate(pend0):
            resp0.append(K.kry_server_wait(srv, p_))
            if (j + 1) % 25 == 0:
                log("serve: saturation run, %d of %d done (%.1f s)" % (j + 1, len(reqs), time.perf_counter() - t0))
        sat = len(reqs) / (time.perf_counter() - t0)
        log("serve: saturation %.1f requests/s" % sat)
        # Poisson arrivals at fractions of saturation; the 80 % run is the headline
        sweep = {}
        for frac in [float(f) for f in args.serve_sweep.split(",")]:
            rate = frac * sat
            gaps = rng.exponential(1.0 / rate, size=len(reqs))
            t0 = time.perf_counter()
            pend = []
            tnext = t0
            for j, (r, gap) in enumerate(zip(reqs, gaps)):
                tnext += gap
                while time.perf_counter() < tnext:
                    time.sleep(min(0.0005, max(0.0, tnext - time.perf_counter())))
                pend.append(submit(srv, r, o32))
                if (j + 1) % 25 == 0:
                    log("serve: %d%% run, %d of %d submitted" % (100 * frac, j + 1, len(reqs)))
            resp_f = []
            for j, p_ in enumerate(pend):
                resp_f.append(K.kry_server_wait(srv, p_))
                if (j + 1) % 25 == 0:
                    log("serve: %d%% run, %d of %d done" % (100 * frac, j + 1, len(reqs)))
            wall_f = time.perf_counter() - t0
            lat_f = np.array([r.t_end - r.t_submit for r in resp_f]) * 1e3
            sweep[frac] = (rate, resp_f, wall_f, lat_f)
            log("serve at %d%% of saturation: p50 %.1f ms p99 %.1f ms, %.1f req/s" %
                (100 * frac, np.percentile(lat_f, 50), np.percentile(lat_f, 99), len(reqs) / wall_f))
        head = 0.8 if 0.8 in sweep else sorted(sweep)[-1]
        rate, resp, wall, lat = sweep[head]
    finally:
        K.kry_server_destroy(srv)
    _, peak_mem = K.kry_ctx_memory(ctx)
    statuses = {}
    for r in resp0 + [x for v in sweep.values() for x in v[1]]:
        statuses[int(r.status)] = statuses.get(int(r.status), 0) + 1
    n_ll = sum(1 for r in reqs if r[0] == "loglik")
    # service time (start to end) of the saturation run's requests, by grid side and kind
    service = {}
    for r, rs in zip(reqs, resp0):
        key = "%d %s" % (int(sides[r[1]]), r[0])
        service.setdefault(key, []).append(rs.t_end - rs.t_start)
    service = {k: {"requests": len(v), "mean_s": float(np.mean(v)), "max_s": float(np.max(v))}
               for k, v in sorted(service.items(), key=lambda kv: (int(kv[0].split()[0]), kv[0]))}
    # plain FP64 form, one request at a time, on every k-th request
    k = max(1, len(reqs) // max(1, args.serve_plain_sample))
    sample = list(range(0, len(reqs), k))
    errs, kerr = [], []
    t1 = time.perf_counter()
    for jj, i in enumerate(sample):
        if jj % 10 == 0:
            log("serve: plain FP64 sample, %d of %d" % (jj, len(sample)))
        kind, pi, th, tg = reqs[i]
        if kind == "loglik":
            ref = K.kry_loglik(probs[pi], th, o64, allow_noconv=True)["loglik"]
            errs.append(abs(resp0[i].loglik.loglik - ref) / abs(ref))
        else:
            m64, _, _ = K.kry_krige(probs[pi], th, o64, tg)  # (the served kriging is FP64 too)
            m32 = pend0[i].outputs["mean_x"]
            kerr.append(float(np.max(np.abs(m32 - m64)) / max(np.max(np.abs(m64)), 1e-300)))
    seq = time.perf_counter() - t1
    for h in probs:
        K.kry_problem_destroy(h)
    K.kry_ctx_destroy(ctx)
    plain_rate = len(sample) / seq
    out = {"requests": len(reqs), "loglik_fraction": n_ll / len(reqs), "sides": [lo, hi],
           "problem_sides": [int(v) for v in sides], "slots": args.serve_slots,
           "hbm_budget_bytes": budget, "slot_peak_bytes": int(peak_mem - base_mem), "statuses": statuses,
           "saturation_req_per_s": sat, "arrival_rate_per_s": rate, "headline_fraction": head,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "req_per_s": len(reqs) / wall, "loglik_evals_per_s": n_ll / wall,
           "max_batch_seen": int(max(r.batch for r in resp0 + resp)), "service_time_by_side": service,
           "served_precision": "likelihood: fp32 Lanczos products (reorthogonalised, fp64 coefficients), fp64 "
                                "multi-shift CG; kriging: fp64; cg_rtol 1e-8",
           "plain_fp64": {"sample": "every %d-th request (%d of %d), sequential, cg_rtol 1e-8" % (k, len(sample),
                                                                                                 len(reqs)),
                          "req_per_s": plain_rate, "loglik_requests": len(errs),
                          "loglik_rel_err_max": float(max(errs)) if errs else None,
                          "loglik_rel_err_median": float(np.median(errs)) if errs else None,
                          "krige_mean_rel_err_max": float(max(kerr)) if kerr else None},
           # capacity against capacity: the saturation run's rate (the runs at a
           # fraction of saturation are capped by their arrival rate)
           "served_vs_plain": sat / plain_rate,
           "arrival_sweep": [{"fraction_of_saturation": f, "arrival_rate_per_s": v[0],
                              "p50_ms": float(np.percentile(v[3], 50)), "p99_ms": float(np.percentile(v[3], 99)),
                              "req_per_s": len(reqs) / v[2]} for f, v in sweep.items()]}
    log("serve: p50 %.1f ms p99 %.1f ms at %.1f req/s; saturation %.1f req/s vs plain fp64 %.1f req/s; "
        "loglik rel err max %s" % (out["p50_ms"], out["p99_ms"], out["req_per_s"], sat, plain_rate,
                                   out["plain_fp64"]["loglik_rel_err_max"]))
    return out


def multi_bench(args, K, synth, np):
    """Multi-problem form: independent problems on square grids with sides
    log-uniform in the given range, 20-50 % missing uniformly at random, nu in
    {0.5, 1.5}, range log-uniform in [0.02, 0.2], nugget ratio 0.1, data drawn
    by circulant embedding plus nugget noise; 32 probes x 50 Lanczos steps
    (reorthogonalised) and CG to 1e-8 per problem, FP32 transforms.  Times one
    kry_loglik_multi call against the same problems one at a time (FP32) and
    in the plain FP64 form, and reports the largest relative difference of
    the batched log-likelihoods from the FP64 ones."""
    import torch

    lo, hi = (int(x) for x in args.multi_sides.split(","))
    rng = np.random.default_rng(808)
    ctx = K.kry_ctx_create()
    sides = synth.log_uniform_sides(args.multi, lo, hi, seed=809)
    hs, ths, cells = [], [], 0
    for i, n in enumerate(sides):
        n = int(n)
        mask = synth.uniform_mask(n, n, float(rng.uniform(0.2, 0.5)), seed=3000 + i)
        th = K.theta(sigma2=1.0, tau2=0.1, range=float(np.exp(rng.uniform(np.log(0.02), np.log(0.2)))),
                     nu=float(rng.choice([0.5, 1.5])))
        h = K.kry_problem_create(ctx, n, n, mask)
        Nt = K.kry_psd_torus(h, th)
        x, _ = K.kry_sample(h, th, Nt[0], Nt[1], 4000 + i, 0, 1, n, n)
        K.kry_problem_set_data(h, x[0] + np.sqrt(0.1) * rng.standard_normal((n, n)))
        hs.append(h)
        ths.append(th)
        cells += n * n
    o32 = K.kry_opts_default(lanczos_steps=50, num_probes=32, reorth=1, precision=K.KRY_FP32, cg_rtol=1e-8,
                             cg_maxit=100000)
    o64 = K.kry_opts_default(lanczos_steps=50, num_probes=32, reorth=1, precision=K.KRY_FP64, cg_rtol=1e-8,
                             cg_maxit=100000)
    try:
        K.kry_loglik_multi(hs[:2], ths[:2], o32)  # warm-up (kernels, buffers)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        multi = K.kry_loglik_multi(hs, ths, o32)
        t_multi = time.perf_counter() - t0
        log("multi: %d problems (%d cells) in %.2f s" % (len(hs), cells, t_multi))
        t0 = time.perf_counter()
        for h, th in zip(hs, ths):
            K.kry_loglik(h, th, o32)
        t_seq32 = time.perf_counter() - t0
        log("one at a time FP32: %.2f s" % t_seq32)
        t0 = time.perf_counter()
        plain = [K.kry_loglik(h, th, o64) for h, th in zip(hs, ths)]
        t_seq64 = time.perf_counter() - t0
        log("plain FP64 one at a time: %.2f s" % t_seq64)
    finally:
        for h in hs:
            K.kry_problem_destroy(h)
        K.kry_ctx_destroy(ctx)
    err = max(abs(m["loglik"] - p_["loglik"]) / abs(p_["loglik"]) for m, p_ in zip(multi, plain))
    return {"problems": len(hs), "sides": [lo, hi], "cells": cells, "seconds": t_multi,
            "evals_per_s": len(hs) / t_multi, "one_at_a_time_fp32_evals_per_s": len(hs) / t_seq32,
            "plain_fp64_evals_per_s": len(hs) / t_seq64, "multi_vs_plain_fp64": t_seq64 / t_multi,
            "multi_vs_one_at_a_time_fp32": t_seq32 / t_multi, "max_rel_err_vs_fp64": err}


def _timed(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, r


def ext_bench(args, K, synth, np):
    """Extension rows, each timed once on its own workload (not part of the
    headline step):
    * irregular observations (the paper's third study: 40,000 locations on a
      400 x 400 latent grid; and 734,003 locations on the 1024 x 1024 grid,
      listed at random and by grid cell): batched FP32 / FP64 product rates
      and one FP64 likelihood evaluation;
    * covariates: a 3 x 3 (range, nugget) shift-shared FP32 batch at 1024^2
      with an intercept (mean 44.49) against the same batch without;
    * the paper's objective at 1024^2: one pl~ evaluation with its gradient
      (k = 1: the quadrant log-determinant and its derivative dominate, FP64
      DFT contractions of about 24 n^3 flops per lag grid pair; k = 50);
    * the low-rank posterior variance at every cell of 1024^2 (k = 50)."""
    out = {}
    th = K.theta(sigma2=3.0, tau2=0.5, range=0.1, nu=0.5)
    B = args.mv_batch
    for name, n, p, order in (("irregular_400sq_40k", 400, 40000, "random"),
                              ("irregular_1024sq_734k", 1024, 734003, "random"),
                              ("irregular_1024sq_734k_cell_order", 1024, 734003, "cell")):
        g = (n, n, 1.0 / n, 1.0 / n)
        locs = synth.irregular_locations(g, p, seed=61)
        if order == "cell":  # the caller lists observations by nearest grid cell, the library's stored order
            near = np.minimum(np.floor(locs[:, 0] + 0.5), n - 1) * n + np.minimum(np.floor(locs[:, 1] + 0.5), n - 1)
            locs = locs[np.argsort(near, kind="stable")]
        rng = np.random.default_rng(62)
        P = K.IrregularProblem(n, n, locs, rng.standard_normal(p))
        row = {"grid": n, "observations": p, "order": order}
        for prec, key in ((K.KRY_FP32, "fp32"), (K.KRY_FP64, "fp64")):
            V = synth.random_vectors(p, B, seed=63, dtype=np.float32 if prec == K.KRY_FP32 else np.float64)
            import torch
            dv = torch.from_numpy(V).cuda()
            do = torch.empty_like(dv)
            st = torch.cuda.current_stream().cuda_stream
            K.kry_matvec_device(P.h, th, prec, B, dv.data_ptr(), do.data_ptr(), st)
            dt, _ = _timed(lambda: K.kry_matvec_device(P.h, th, prec, B, dv.data_ptr(), do.data_ptr(), st), 10)
            row["matvecs_per_s_" + key] = B / dt
        opts = K.kry_opts_default(lanczos_steps=30, num_probes=10, reorth=1, cg_rtol=1e-8, cg_maxit=100000)
        K.kry_loglik(P.h, th, opts)
        dt, r = _timed(lambda: K.kry_loglik(P.h, th, opts))
        row["loglik_fp64_s"] = dt
        row["loglik_cg_iters"] = r["cg_iters"]
        log("ext %s: fp32 %.0f fp64 %.0f matvecs/s, fp64 loglik %.2f s" % (name, row["matvecs_per_s_fp32"],
                                                                          row["matvecs_per_s_fp64"], dt))
        out[name] = row
        P.close()
    # covariates and the paper's objective on the metric workload
    n = args.n
    mask = synth.uniform_mask(n, n, 0.3, seed=101)
    P = K.Problem(n, n, mask)
    th0 = K.theta(sigma2=1.0, tau2=0.2, range=0.05, nu=1.5)
    N = K.kry_psd_torus(P.h, th0)
    x, _ = K.kry_sample(P.h, th0, N[0], N[1], 202, 0, 1, n, n)
    y = 44.49 + x[0] + np.sqrt(0.2) * np.random.default_rng(303).standard_normal((n, n))
    K.kry_problem_set_data(P.h, y)
    pts = [K.theta(sigma2=1.0, tau2=e, range=r, nu=1.5) for r in (0.02, 0.05, 0.1) for e in (0.05, 0.2, 0.8)]
    opts = K.kry_opts_default(lanczos_steps=50, num_probes=20, reorth=1, cg_rtol=1e-8, cg_maxit=100000,
                              precision=K.KRY_FP32, shift_share=1)
    K.kry_problem_set_covariates(P.h, synth.covariates(n, n, 1, seed=64))
    t_cov, rc = _timed(lambda: K.kry_loglik_batch(P.h, pts, opts))
    K.kry_problem_set_covariates(P.h, None)
    K.kry_problem_set_data(P.h, y - 44.49)
    t_plain, _ = _timed(lambda: K.kry_loglik_batch(P.h, pts, opts))
    out["covariates_1024sq_3x3"] = {"points": len(pts), "s_with_intercept": t_cov, "s_zero_mean": t_plain,
                                    "ratio": t_cov / t_plain, "beta_hat": float(rc[4]["beta"][0]),
                                    "beta_se": float(rc[4]["beta_se"][0])}
    log("ext covariates: %.2f s with an intercept vs %.2f s zero mean" % (t_cov, t_plain))
    K.kry_problem_set_data(P.h, y)
    K.kry_problem_set_covariates(P.h, synth.covariates(n, n, 1, seed=64))
    beta = [44.49]
    row = {}
    for k in (1, 50):
        o = K.kry_opts_default(gk_steps=k, reorth=1, precision=K.KRY_FP32)
        K.kry_plik(P.h, th0, o, beta=beta)
        dt, r = _timed(lambda: K.kry_plik(P.h, th0, o, beta=beta))
        row["k%d_s" % k] = dt
    M = 2 * n - 1
    flops = 2.0 * (2 * n) * (2 * M) * M + 4 * 2.0 * n * n * M
    row["quadrant_flops"] = flops
    row["quadrant_tflops_upper_bound_from_k1"] = flops / row["k1_s"] / 1e12
    out["plik_1024sq"] = row
    log("ext plik: k=1 %.3f s, k=50 %.3f s" % (row["k1_s"], row["k50_s"]))
    o = K.kry_opts_default(gk_steps=50, reorth=1, precision=K.KRY_FP32)
    K.kry_posterior_variance(P.h, th0, o, n * n, beta=beta)
    dt, _ = _timed(lambda: K.kry_posterior_variance(P.h, th0, o, n * n, beta=beta))
    out["posterior_variance_1024sq_k50_s"] = dt
    log("ext posterior variance: %.3f s" % dt)
    P.close()
    return out


def config4_bench(args, K, synth, np):
    """Large anisotropic problem end to end: a 2048 x 2048 grid with 40 % of
    the cells missing in blob-shaped (cloud-like) masks, Matern nu = 1, range
    0.05, geometric anisotropy ratio 2 at 30 degrees, nugget ratio 0.1, data
    by circulant embedding on a PSD torus; the profile-likelihood fit over
    (range, nugget ratio) by Nelder-Mead with FP32 transforms and FP64
    quadrature (common random numbers), then kriging means and bootstrap
    variances (B draws) at every missing cell, and exact variances at a
    seeded subset of them to bound the bootstrap's Monte-Carlo error."""
    n = args.c4_n
    ang = np.pi / 6
    truth = K.theta(sigma2=1.0, tau2=0.1, range=0.05, nu=1.0, aniso_ratio=2.0, aniso_angle=ang)
    mask = synth.blob_mask(n, n, 0.4, seed=401, rmin=10, rmax=80)
    ctx = K.kry_ctx_create()
    out = {"grid": n, "missing": float(1 - mask.mean())}
    try:
        t0 = time.perf_counter()
        h = K.kry_problem_create(ctx, n, n, mask)
        Nt = K.kry_psd_torus(h, truth)
        x, _ = K.kry_sample(h, truth, Nt[0], Nt[1], 402, 0, 1, n, n)
        rng = np.random.default_rng(403)
        K.kry_problem_set_data(h, x[0] + np.sqrt(truth.tau2) * rng.standard_normal((n, n)))
        del x
        p, N1, N2 = K.kry_problem_info(h)
        out.update({"p": int(p), "embedding": [N1, N2], "psd_torus": list(Nt),
                    "setup_s": time.perf_counter() - t0})
        log("config 4: %dx%d, p = %d, embedding %dx%d, sampling torus %s" % (n, n, p, N1, N2, Nt))
        # Lanczos runs 1024 steps: with 50 the quadrature is far from
        # converged at this size (the log-determinant is off by about 4 % and
        # the fit lands near range 0.03); the adaptive rule at rtol 1e-5
        # stops after 325-450 steps with the log-determinant still about 1000
        # off, an error that varies enough with the parameters to move the fit
        # to range 0.038, nugget ratio 0.17; at 1e-7 it stops after 615-910
        # steps within 10 of the 1024-step values, but its quadratures at the
        # checks cost more than the steps (one evaluation 4 s against 1.5 s)
        opts = K.kry_opts_default(lanczos_steps=args.c4_steps, num_probes=args.c4_probes, precision=K.KRY_FP32,
                                  reorth=0, cg_rtol=args.c4_cg_rtol, seed=303, lanczos_rtol=args.c4_lanczos_rtol,
                                  lanczos_max_steps=args.c4_lanczos_max)
        # a coarse (range, nugget ratio) grid in one shift-shared batch (the
        # nugget values of a range share Krylov spaces), then Nelder-Mead from
        # its best point, the same probes throughout (common random numbers)
        t1 = time.perf_counter()
        grid_r, grid_e = (0.02, 0.035, 0.06, 0.1), (0.03, 0.1, 0.3)
        pts = [K.theta(sigma2=1.0, tau2=e, range=r, nu=1.0, aniso_ratio=2.0, aniso_angle=ang)
               for r in grid_r for e in grid_e]
        gopts = dict((f, getattr(opts, f)) for f, _ in opts._fields_)
        gopts["shift_share"] = 1
        gres = K.kry_loglik_batch(h, pts, K.kry_opts_default(**gopts), allow_noconv=True)
        best = int(np.argmax([g["loglik_profiled"] for g in gres]))
        init = pts[best]
        grid_s = time.perf_counter() - t1
        log("config 4 coarse grid: best range %.3f nugget ratio %.3f (%.1f s)" % (init.range, init.tau2, grid_s))
        os.environ["KRY_VERBOSE"] = "1"  # a line per evaluation: the fit is one long library call
        try:
            est, at = K.kry_fit(h, init, 3, opts, xtol=args.c4_xtol, maxiter=args.c4_maxiter)
        finally:
            del os.environ["KRY_VERBOSE"]
        fit_s = time.perf_counter() - t1
        eta_hat = est.tau2 / est.sigma2
        out["fit"] = {"seconds": fit_s, "range": est.range, "nugget_ratio": eta_hat, "sigma2": est.sigma2,
                      "loglik_profiled": at["loglik_profiled"], "logdet_se": at["logdet_se"],
                      "lanczos_steps_at_estimate": at["lanczos_steps_used"], "cg_iters_at_estimate": at["cg_iters"],
                      "xtol": args.c4_xtol, "maxiter": args.c4_maxiter, "probes": args.c4_probes,
                      "lanczos": ("adaptive, rtol %g, at most %d steps" % (args.c4_lanczos_rtol, args.c4_lanczos_max)
                                  if args.c4_lanczos_rtol > 0 else "%d steps" % args.c4_steps),
                      "cg_rtol": args.c4_cg_rtol, "coarse_grid": {"ranges": list(grid_r), "nugget_ratios": list(grid_e),
                                                                  "seconds": grid_s, "start": [init.range, init.tau2]},
                      "truth": [0.05, 0.1]}
        log("config 4 fit: range %.4f nugget ratio %.4f sigma2 %.3f in %.1f s" % (est.range, eta_hat, est.sigma2,
                                                                                 fit_s))
        # kriging at every missing cell: means and bootstrap variances
        miss = np.flatnonzero(mask.ravel() == 0)
        kopts = K.kry_opts_default(precision=K.KRY_FP32, cg_rtol=1e-8, seed=404)
        t2 = time.perf_counter()
        mean, vx, vy = K.kry_krige(h, est, kopts, None, ntargets=miss.size, want_var=True,
                                   bootstrap_B=args.c4_boot)
        krige_s = time.perf_counter() - t2
        # exact variances at a seeded subset of the missing cells
        sub = np.sort(np.random.default_rng(405).choice(miss.size, size=args.c4_exact, replace=False))
        t3 = time.perf_counter()
        m2, ex, ey = K.kry_krige(h, est, kopts, miss[sub], want_var=True)
        exact_s = time.perf_counter() - t3
        ratio = vx[sub] / ex
        # each bootstrap variance is the exact one times chi2_B / B: mean
        # ratio 1 with standard error about sqrt(2 / B) / sqrt(cells), cells
        # treated as independent
        se = np.sqrt(2.0 / args.c4_boot) / np.sqrt(sub.size)
        out["krige"] = {"cells": int(miss.size), "bootstrap_B": args.c4_boot, "seconds": krige_s,
                        "cells_per_s": miss.size / krige_s, "exact_subset": int(sub.size),
                        "exact_subset_seconds": exact_s,
                        "mean_abs_diff_subset": float(np.max(np.abs(m2 - mean[sub]))),
                        "bootstrap_over_exact_mean": float(ratio.mean()), "bootstrap_over_exact_se": float(se),
                        "mean_var_x": float(vx.mean()), "mean_var_y": float(vy.mean())}
        log("config 4 kriging: %d cells, B = %d in %.1f s; bootstrap/exact %.3f +- %.3f" %
            (miss.size, args.c4_boot, krige_s, ratio.mean(), se))
        K.kry_problem_destroy(h)
    finally:
        K.kry_ctx_destroy(ctx)
    return out


def cpu_baseline(n, mask, th, p, budget_s=15.0):
    """The oracle's direct O(p^2) masked product on a bounded sample of output
    rows of the same workload, scaled to full products per second."""
    import numpy as np

    from oracle import direct
    from oracle.geometry import lag_table

    g = (n, n, 1.0 / n, 1.0 / n)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(p)
    host = {"cpu_count": os.cpu_count(), "model": None, "blas_threads": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    host["model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(limits=1)  # the oracle on one core, BLAS included
    except ImportError:
        limit = None
    try:
        if limit is not None:
            from threadpoolctl import threadpool_info
            host["blas_threads"] = [i.get("num_threads") for i in threadpool_info()]
        t0 = time.perf_counter()
        T = lag_table(n, n, 1.0 / n, 1.0 / n, th)
        t_table = time.perf_counter() - t0
        rows = 0
        t1 = time.perf_counter()
        while time.perf_counter() - t1 < budget_s:
            direct.masked_matvec(g, mask, th, v, rows=np.arange(rows, rows + 25), table=T)
            rows += 25
        dt = time.perf_counter() - t1
    finally:
        if limit is not None:
            limit.restore_original_limits()
    rate = rows / dt / p
    return {"value": rate, "unit": "matvecs/s", "cores": 1, "kind": "oracle", "host": host,
            "sample": "direct O(p^2) masked product, %d of %d output rows (%.1f s) plus the lag table (%.1f s, "
                      "not counted) at 1024x1024, 30%% missing; thread pools limited to one thread" %
                      (rows, p, dt, t_table)}


if __name__ == "__main__":
    main()
