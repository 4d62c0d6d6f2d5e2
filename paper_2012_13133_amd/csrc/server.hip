// Request server: continuous batching of likelihood and kriging requests on
// device-resident problems.
//
// `slots` worker threads each own a HIP stream (default priority) and a
// workspace; a request is admitted when a slot is free and the estimated
// device footprint of everything in flight stays within the HBM budget, so
// requests that arrive while others run start as soon as a slot and memory
// free up, and their kernels overlap on the device.  A worker that takes a
// likelihood request also takes every queued likelihood request with
// identical options on the same problem, or on another problem with the same
// embedding, (up to max_batch) and runs them as one batched evaluation
// (every (point, probe) vector in the same products; several problems through
// a per-vector problem table).  Reductions are fixed-order per vector, so a
// request batched with others on its own problem gets bit-identical results;
// batched with other problems, its Krylov vectors are padded to the largest
// observed count, which changes the reduction blocks and so the rounding.
#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "internal.hpp"

using namespace kry;

namespace {

struct Pending {
    uint64_t ticket;
    kry_request req;
    std::vector<int64_t> targets;
    uint64_t footprint;
    double t_submit;
};

// Workspace of one slot, moved into a problem view for the duration of a
// request.
struct SlotWork {
    DevBuf Y, lagtmp, spectmp, spec_multi64, spec_multi32, kws, scal, tmp1, tmp2, tmp3, tmp4, irr;
    Spectrum spec;
    const Problem* last = nullptr;
    std::array<DevBuf*, 14> bufs() {
        return {&Y, &lagtmp, &spectmp, &spec_multi64, &spec_multi32, &kws, &scal, &tmp1,
                &tmp2, &tmp3, &tmp4, &irr, &spec.s64, &spec.s32};
    }
    // device bytes the slot keeps between requests (its buffers only grow)
    uint64_t bytes() {
        uint64_t b = 0;
        for (DevBuf* d : bufs()) b += d->bytes;
        return b;
    }
    void release(Ctx& c) {
        for (DevBuf* d : bufs()) d->release(c);
        spec.valid = false;
    }
};

void swap_work(Problem& v, SlotWork& w) {
    std::swap(v.Y, w.Y);
    std::swap(v.lagtmp, w.lagtmp);
    std::swap(v.spectmp, w.spectmp);
    std::swap(v.spec_multi64, w.spec_multi64);
    std::swap(v.spec_multi32, w.spec_multi32);
    std::swap(v.kws, w.kws);
    std::swap(v.scal, w.scal);
    std::swap(v.tmp1, w.tmp1);
    std::swap(v.tmp2, w.tmp2);
    std::swap(v.tmp3, w.tmp3);
    std::swap(v.tmp4, w.tmp4);
    std::swap(v.irr, w.irr);
    std::swap(v.spec.s64, w.spec.s64);
    std::swap(v.spec.s32, w.spec.s32);
    std::swap(v.spec.theta, w.spec.theta);
    std::swap(v.spec.valid, w.spec.valid);
    std::swap(v.spec.lam_min, w.spec.lam_min);
    std::swap(v.spec.lam_max, w.spec.lam_max);
}

// Device bytes a request's workspace can reach (an upper bound that follows
// the drivers' allocations: spectrum and lag grid, Krylov basis, transform
// intermediates, solver vectors).  A batch of merged requests is bounded by
// the sum of its requests' bounds.
uint64_t footprint(const Problem& P, const kry_request& r) {
    const uint64_t p = P.p, n = (uint64_t)P.n1 * P.n2;
    const uint64_t M = P.N2 / 2, nspec = (M + 1) * P.N1;
    const bool fp32 = r.opts.precision == KRY_FP32;
    const uint64_t el = fp32 ? 4 : 8;
    // transform intermediate per vector: complex values on (M + 1) x (rows
    // rounded up to a row tile of at most 64 rows)
    const uint64_t inter = (M + 1) * ((uint64_t)P.n1 + 64) * 2;  // times bytes per real
    const uint64_t lagspec = (uint64_t)P.N1 * P.N2 * 8 + (M + 1) * (uint64_t)P.N1 * 16 + 16384;
    const uint64_t nd = 1 + (uint64_t)P.q;  // right-hand sides per point
    const uint64_t grid = P.irregular ? 2 * n * 8 : 0;  // grid vectors of the irregular product (per vector)
    // a solve of k right-hand sides: CG vectors (FP64 or FP32 with FP64
    // refinement), partials, products in both precisions
    auto solve = [&](uint64_t k) {
        return k * p * (fp32 ? 36 : 24) + k * 4096 + 4096;
    };
    auto prod = [&](uint64_t k, uint64_t e) { return k * (inter * e + grid); };
    if (r.kind == KRY_REQ_LOGLIK) {
        const uint64_t np = nprobes_of(&r.opts);
        const uint64_t m = lanczos_cap(&r.opts);
        const uint64_t slots = r.opts.reorth ? m + 1 : 3;
        const uint64_t nblk = 256;
        const uint64_t kws = np * p * el * (slots + 2) + np * (m + 1) * nblk * 8 + np * (3 * m + 8) * 8 + 65536;
        const uint64_t spec = nd * nspec * 12;
        // the multi-shift CG's p . w partials: one block's worth, or the
        // column stage's spectral partials on a power-of-two embedding
        const uint64_t pwp = nd * (uint64_t)std::max(256, spectral_qf_count(P.N1, P.N2)) * 8;
        const uint64_t rhs = nd * p * 16 + 4096 + nd * 257 * 8 + pwp;
        const uint64_t gk = r.opts.solver == KRY_SOLVER_GENGK
                                ? (uint64_t)(r.opts.gk_steps + 2) * 2 * n * el + 4 * n * 8 + p * 8 * 4
                                : 0;
        const uint64_t Y = std::max({prod(np, el), prod(nd, 8), prod(nd, el), prod(1, 8)});
        return lagspec + spec + rhs + kws + solve(nd) + Y + gk + nspec * 12;
    }
    const uint64_t nt = std::max<int64_t>(r.ntargets, 1);
    const uint64_t c = r.variances ? std::min<uint64_t>(nt, 256) : 1;
    const uint64_t io = 8192 + nt * 32 + p * 16 + n * 8;
    const uint64_t var = r.variances ? c * p * 16 + c * 257 * 8 + 1024 : 0;
    const uint64_t Y = std::max(prod(c * nd, 8), prod(1, 8));
    return lagspec + nspec * 12 + io + var + solve(c * nd) + Y + nd * p * 8 * 4;
}
}  // namespace

struct kry_server {
    Ctx* ctx = nullptr;
    int slots = 1, max_batch = 1, max_queue = 1;
    uint64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, kry_response> done;
    std::unordered_map<uint64_t, bool> known;
    uint64_t next_ticket = 1;
    // Device memory of the slots: a running slot may use up to its retained
    // workspace plus its batch's estimated footprint; an idle one holds its
    // retained workspace, which can be released to admit a request.
    std::vector<uint64_t> retained, running;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::vector<SlotWork> work;
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    static bool same_opts(const kry_opts& a, const kry_opts& b) {
        return a.lanczos_steps == b.lanczos_steps && a.num_probes == b.num_probes && a.probe_kind == b.probe_kind &&
               a.colour_period == b.colour_period && a.seed == b.seed && a.reorth == b.reorth &&
               a.precision == b.precision && a.cg_rtol == b.cg_rtol && a.cg_maxit == b.cg_maxit &&
               a.solver == b.solver && a.gk_steps == b.gk_steps && a.shift_share == b.shift_share &&
               a.lanczos_max_steps == b.lanczos_max_steps && a.lanczos_rtol == b.lanczos_rtol && a.reml == b.reml;
    }

    // Likelihood requests that can run in one batch with the head h: the same
    // problem, or (CG, no shift sharing, no covariates) a problem with the
    // same embedding, whose products then share launches through a problem
    // table.
    static bool mergeable(const kry_request& h, const kry_request& r) {
        if (r.kind != KRY_REQ_LOGLIK || !same_opts(r.opts, h.opts)) return false;
        if (r.prob == h.prob) return true;
        return h.opts.solver == KRY_SOLVER_CG && h.opts.shift_share == 0 && r.prob->P.N1 == h.prob->P.N1 &&
               r.prob->P.N2 == h.prob->P.N2 && r.prob->P.q == 0 && h.prob->P.q == 0 && !r.prob->P.irregular &&
               !h.prob->P.irregular;
    }

    // Memory held by the running slots (requires mu).  A running slot may
    // hold its retained workspace plus its batch's footprint: its buffers
    // grow one by one to what the batch needs, so a buffer the batch leaves
    // small keeps its retained size while others grow (the larger of the two
    // totals is not a bound when the retained workspace and the batch differ
    // in which buffers are large).
    uint64_t busy_bytes() const {
        uint64_t b = 0;
        for (size_t s = 0; s < running.size(); ++s)
            if (running[s]) b += retained[s] + running[s];
        return b;
    }
    bool any_running() const {
        for (uint64_t r : running)
            if (r) return true;
        return false;
    }
    // Memory held by every slot other than `slot` (requires mu).
    uint64_t other_bytes(int slot) const {
        uint64_t b = 0;
        for (size_t s = 0; s < running.size(); ++s)
            if ((int)s != slot) b += retained[s] + running[s];
        return b;
    }
    // Make room for a batch of footprint fp on `slot` by releasing idle
    // slots' workspaces, its own first (requires mu; the idle slots' threads
    // are waiting for work, so their buffers are not in use).
    void make_room(int slot, uint64_t fp) {
        auto need = [&] { return other_bytes(slot) + retained[slot] + fp; };
        if (need() <= budget) return;
        if (retained[slot]) {
            work[slot].release(*ctx);
            retained[slot] = 0;
        }
        for (size_t s = 0; s < running.size() && need() > budget; ++s) {
            if ((int)s == slot || running[s] || !retained[s]) continue;
            work[s].release(*ctx);
            retained[s] = 0;
        }
    }

    void run_slot(int slot) {
        (void)hipSetDevice(ctx->device);
        hipStream_t st = streams[slot];
        SlotWork& w = work[slot];
        while (true) {
            std::vector<Pending> batch;
            uint64_t fp = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                // a request is admitted when it fits beside the running
                // slots (idle slots' workspaces can be released), or when
                // nothing runs (it alone is within the budget, checked at submit)
                cv_work.wait(lk, [&] {
                    return stop || (!queue.empty() && (busy_bytes() + queue.front().footprint <= budget || !any_running()));
                });
                if (queue.empty()) {
                    if (stop) return;
                    continue;
                }
                batch.push_back(std::move(queue.front()));
                queue.pop_front();
                fp = batch[0].footprint;
                const kry_request& h = batch[0].req;
                if (h.kind == KRY_REQ_LOGLIK) {
                    for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < max_batch;) {
                        const kry_request& r = it->req;
                        if (mergeable(h, r) && busy_bytes() + fp + it->footprint <= budget) {
                            fp += it->footprint;
                            batch.push_back(std::move(*it));
                            it = queue.erase(it);
                        } else {
                            ++it;
                        }
                    }
                }
                make_room(slot, fp);
                running[slot] = fp;
            }
            const double t_start = now();
            std::vector<kry_response> resp(batch.size());
            execute(batch, resp, w, st);
            const double t_end = now();
            {
                std::lock_guard<std::mutex> lk(mu);
                running[slot] = 0;
                retained[slot] = w.bytes();
                for (size_t i = 0; i < batch.size(); ++i) {
                    resp[i].footprint_bytes = fp;
                    resp[i].workspace_bytes = retained[slot];
                    resp[i].t_submit = batch[i].t_submit;
                    resp[i].t_start = t_start;
                    resp[i].t_end = t_end;
                    resp[i].batch = (int32_t)batch.size();
                    done[batch[i].ticket] = resp[i];
                }
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }

    void execute(std::vector<Pending>& batch, std::vector<kry_response>& resp, SlotWork& w, hipStream_t st) {
        const Problem& base = batch[0].req.prob->P;
        Problem v = base.view();
        // slots run concurrently in several threads: no stream capture there
        // (a capture crashed inside the runtime under a kernel tracer)
        v.no_graphs = true;
        w.spec.valid = false;  // the cached spectrum may belong to another problem
        w.last = &base;
        swap_work(v, w);
        const kry_request& h = batch[0].req;
        kry_status status = KRY_OK;
        std::string msg;
        try {
            if (h.kind == KRY_REQ_LOGLIK) {
                std::vector<kry_matern> th(batch.size());
                std::vector<kry_loglik_result> res(batch.size());
                std::vector<Problem*> ps(batch.size());
                bool one_problem = true;
                for (size_t i = 0; i < batch.size(); ++i) {
                    th[i] = batch[i].req.theta;
                    ps[i] = &batch[i].req.prob->P;
                    one_problem = one_problem && batch[i].req.prob == h.prob;
                }
                if (one_problem) loglik_points(v, th.data(), (int)th.size(), &h.opts, res.data(), st);
                else loglik_multi(v, ps, th.data(), &h.opts, res.data(), st);
                int nprob = 0;
                for (size_t i = 0; i < batch.size(); ++i) {
                    bool seen = false;
                    for (size_t j = 0; j < i; ++j) seen = seen || batch[j].req.prob == batch[i].req.prob;
                    nprob += seen ? 0 : 1;
                }
                for (auto& r : resp) r.problems = nprob;
                for (size_t i = 0; i < batch.size(); ++i) {
                    resp[i].loglik = res[i];
                    resp[i].status = (h.opts.solver == KRY_SOLVER_CG && res[i].cg_relres > h.opts.cg_rtol)
                                         ? KRY_ENOCONV
                                         : KRY_OK;
                }
            } else {
                bool noconv = false;
                krige_impl(v, &h.theta, &h.opts, batch[0].targets, h.mean_x, h.variances ? h.var_x : nullptr,
                           h.variances ? h.var_y : nullptr, 0, &noconv, st);
                resp[0].status = noconv ? KRY_ENOCONV : KRY_OK;
                resp[0].problems = 1;
            }
        } catch (const Error& e) {
            status = e.status;
            msg = e.what();
        } catch (const std::exception& e) {
            status = KRY_EDEVICE;
            msg = e.what();
        }
        (void)hipStreamSynchronize(st);
        swap_work(v, w);
        if (status != KRY_OK)
            for (auto& r : resp) r.status = status;
    }
};

kry_status kry_server_create(kry_ctx* kctx, int32_t slots, uint64_t hbm_budget_bytes, int32_t max_batch,
                             int32_t max_queue, kry_server** out) {
    try {
        if (!kctx || !out || slots < 1 || slots > 16 || max_batch < 1 || max_queue < 1) return KRY_EINVAL;
        Ctx& c = kctx->c;
        auto* s = new kry_server();
        s->ctx = &c;
        s->slots = slots;
        s->max_batch = max_batch;
        s->max_queue = max_queue;
        s->budget = hbm_budget_bytes ? hbm_budget_bytes : ~0ull;
        s->t0 = std::chrono::steady_clock::now();
        if (hipSetDevice(c.device) != hipSuccess) {
            delete s;
            return KRY_EDEVICE;
        }
        s->streams.resize(slots, nullptr);
        s->work.resize(slots);
        s->retained.assign(slots, 0);
        s->running.assign(slots, 0);
        for (int i = 0; i < slots; ++i) {
            if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipStreamDestroy(s->streams[j]);
                delete s;
                return KRY_EDEVICE;
            }
        }
        for (int i = 0; i < slots; ++i) s->workers.emplace_back([s, i] { s->run_slot(i); });
        *out = s;
        return KRY_OK;
    } catch (...) {
        return KRY_EDEVICE;
    }
}

kry_status kry_server_submit(kry_server* s, const kry_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket || !req->prob) return KRY_EINVAL;
    try {
        check_theta(&req->theta);
        check_opts(&req->opts);
        if (req->kind != KRY_REQ_LOGLIK && req->kind != KRY_REQ_KRIGE) return KRY_EINVAL;
        Pending pd;
        pd.req = *req;
        const Problem& P = req->prob->P;
        if (req->kind == KRY_REQ_KRIGE) {
            if (!req->targets || req->ntargets < 1 || !req->mean_x) return KRY_EINVAL;
            const int64_t n = (int64_t)P.n1 * P.n2;
            pd.targets.assign(req->targets, req->targets + req->ntargets);
            for (int64_t t : pd.targets)
                if (t < 0 || t >= n) return KRY_EINVAL;
        }
        pd.footprint = footprint(P, *req);
        if (pd.footprint > s->budget) return KRY_ENOMEM;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if ((int)s->queue.size() >= s->max_queue) return KRY_EBUSY;
            pd.ticket = s->next_ticket++;
            pd.t_submit = s->now();
            s->known[pd.ticket] = true;
            *ticket = pd.ticket;
            s->queue.push_back(std::move(pd));
        }
        s->cv_work.notify_one();
        return KRY_OK;
    } catch (const Error& e) {
        return e.status;
    } catch (...) {
        return KRY_EDEVICE;
    }
}

kry_status kry_server_poll(kry_server* s, uint64_t ticket, kry_response* out, int32_t* is_done) {
    if (!s || !out || !is_done) return KRY_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return KRY_EINVAL;
    auto it = s->done.find(ticket);
    if (it == s->done.end()) {
        *is_done = 0;
        return KRY_OK;
    }
    *out = it->second;
    *is_done = 1;
    s->done.erase(it);
    s->known.erase(ticket);
    return KRY_OK;
}

kry_status kry_server_wait(kry_server* s, uint64_t ticket, kry_response* out) {
    if (!s || !out) return KRY_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return KRY_EINVAL;
    s->cv_done.wait(lk, [&] { return s->done.count(ticket) > 0; });
    *out = s->done[ticket];
    s->done.erase(ticket);
    s->known.erase(ticket);
    return KRY_OK;
}

void kry_server_destroy(kry_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    (void)hipSetDevice(s->ctx->device);
    for (auto& w : s->work) w.release(*s->ctx);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
}
