// C ABI of the library (include/kryging.h) and the host-side drivers that
// sequence the device kernels: likelihood (Sec. 3.1, 3.3 alternative, 3.4),
// generalized Golub-Kahan (Sec. 3.2, Algorithm 1), kriging and the parametric
// bootstrap (Sec. 3.5), circulant-embedding sampling (Sec. 3.6 caveat) and the
// profile-likelihood fit (Sec. 3.4).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "krylov.hpp"

using namespace kry;

static thread_local std::string g_last_error;

template <typename F>
static kry_status guard(F&& f) {
    try {
        f();
        return KRY_OK;
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return KRY_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return KRY_EDEVICE;
    }
}

namespace kry {

kry_status run_guarded(const std::function<void()>& f) { return guard(f); }

void* dev_alloc(Ctx& c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    {
        std::lock_guard<std::mutex> g(c.alloc_mu);
        if (c.budget && c.allocated + bytes > c.budget)
            throw Error(KRY_ENOMEM, "request of " + std::to_string(bytes) + " bytes exceeds the HBM budget (" +
                                        std::to_string(c.allocated) + " of " + std::to_string(c.budget) +
                                        " in use)");
        c.allocated += bytes;
        c.peak = std::max(c.peak, c.allocated);
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> g(c.alloc_mu);
        c.allocated -= bytes;
        throw Error(KRY_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

void dev_free(Ctx& c, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    std::lock_guard<std::mutex> g(c.alloc_mu);
    c.allocated -= std::min<uint64_t>(c.allocated, bytes);
}

}  // namespace kry

namespace {

// Carves sub-buffers out of one growable device allocation.  Used in two
// passes: measure (base == nullptr) and then assign.
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

template <typename F>
void with_arena(Problem& P, F&& layout) {
    Arena m;
    layout(m);
    P.kws.ensure(*P.ctx, m.off + 256);
    Arena a;
    a.base = P.kws.as<char>();
    layout(a);
}

}  // namespace

namespace kry {
void check_theta(const kry_matern* t) {
    KRY_REQUIRE(t != nullptr, "theta is NULL");
    const double v[6] = {t->sigma2, t->tau2, t->range, t->nu, t->aniso_ratio, t->aniso_angle};
    for (double x : v) KRY_REQUIRE(std::isfinite(x), "theta has a non-finite entry");
    KRY_REQUIRE(t->sigma2 > 0, "sigma2 must be > 0");
    KRY_REQUIRE(t->tau2 >= 0, "tau2 must be >= 0");
    KRY_REQUIRE(t->range > 0, "range must be > 0");
    KRY_REQUIRE(t->nu > 0 && t->nu <= 20, "nu must be in (0, 20]");
    KRY_REQUIRE(t->aniso_ratio >= 1, "aniso_ratio must be >= 1");
}

void check_opts(const kry_opts* o) {
    KRY_REQUIRE(o != nullptr, "opts is NULL");
    KRY_REQUIRE(o->lanczos_steps >= 1 && o->lanczos_steps <= KRY_MAX_LANCZOS, "lanczos_steps must be in [1, 1024]");
    KRY_REQUIRE(o->probe_kind == KRY_PROBE_RADEMACHER || o->probe_kind == KRY_PROBE_COLOURED, "bad probe_kind");
    if (o->probe_kind == KRY_PROBE_RADEMACHER) KRY_REQUIRE(o->num_probes >= 1 && o->num_probes <= 4096, "num_probes must be in [1, 4096]");
    else KRY_REQUIRE(o->colour_period >= 1 && o->colour_period <= 64, "colour_period must be in [1, 64]");
    KRY_REQUIRE(o->precision == KRY_FP64 || o->precision == KRY_FP32, "bad precision");
    KRY_REQUIRE(o->cg_rtol > 0 && o->cg_rtol < 1, "cg_rtol must be in (0, 1)");
    KRY_REQUIRE(o->cg_maxit >= 1, "cg_maxit must be >= 1");
    KRY_REQUIRE(o->solver == KRY_SOLVER_CG || o->solver == KRY_SOLVER_GENGK, "bad solver");
    KRY_REQUIRE(o->gk_steps >= 1 && o->gk_steps <= 2000, "gk_steps must be in [1, 2000]");
    KRY_REQUIRE(o->shift_share == 0 || o->shift_share == 1, "shift_share must be 0 or 1");
    KRY_REQUIRE(std::isfinite(o->lanczos_rtol) && o->lanczos_rtol >= 0, "lanczos_rtol must be >= 0");
    if (o->lanczos_rtol > 0)
        KRY_REQUIRE(o->lanczos_max_steps >= 10 && o->lanczos_max_steps <= KRY_MAX_LANCZOS,
                    "lanczos_max_steps must be in [10, 1024] in the adaptive mode");
    KRY_REQUIRE(o->reml == 0 || o->reml == 1, "reml must be 0 or 1");
}

int nprobes_of(const kry_opts* o) {
    return o->probe_kind == KRY_PROBE_COLOURED ? o->colour_period * o->colour_period : o->num_probes;
}

int lanczos_cap(const kry_opts* o) { return o->lanczos_rtol > 0 ? o->lanczos_max_steps : o->lanczos_steps; }
}  // namespace kry

namespace {

Matern to_matern(const kry_matern* t) {
    return Matern{t->sigma2, t->tau2, t->range, t->nu, t->aniso_ratio, t->aniso_angle};
}

int pow2_at_least(int m) {
    int N = 16;
    while (N < m) N *= 2;
    return N;
}

void bind(Ctx& c) { KRY_HIP(hipSetDevice(c.device)); }

// ---- product operators ----------------------------------------------------------------
template <typename R>
MatvecFn<R> masked_op(Problem& P, const void* lam, int64_t lam_tstride, int vpt, const double* d_eta,
                      bool lam_even = false) {
    if (P.irregular) return irregular_op<R>(P, lam, lam_tstride, vpt, d_eta);
    Problem* pp = &P;
    return [pp, lam, lam_tstride, vpt, d_eta, lam_even](const R* x, R* y, int nvec, hipStream_t st,
                                                        const int* active) {
        Problem& Q = *pp;
        ConvSpec s;
        s.N1 = Q.N1;
        s.N2 = Q.N2;
        s.nvec = nvec;
        s.in_mode = IN_COMPACT;
        s.in = x;
        s.in_vstride = Q.p;
        s.rows_in = Q.n1;
        s.row_len = Q.n2;
        s.out_mode = OUT_COMPACT;
        s.out = y;
        s.out_vstride = Q.p;
        s.rows_out = Q.n1;
        s.cols_out = Q.n2;
        s.vin = x;
        s.vin_vstride = Q.p;
        s.eta = d_eta;
        s.lam = lam;
        s.lam_tstride = lam_tstride;
        s.vecs_per_theta = vpt;
        s.lam_even = lam_even && !Q.tab;
        s.tab = Q.tab;
        s.tab_vpp = vpt;
        s.active = active;
        conv_apply<R>(Q, s, st);
    };
}

// The FP64 masked product of the multi-shift CG with its direction update
// p = r + beta p folded into the first stage (masked grid problems).  The
// multi-shift CG's base operators have no nugget (d_eta points at zeros):
// the p . w partials the column stage forms from the spectrum (pw non-null)
// hold the quadratic form of Sigma_oo alone.
MsFusedFn masked_op_update(Problem& P, const void* lam, int64_t lam_tstride, const double* d_eta,
                           bool lam_even = false) {
    Problem* pp = &P;
    return [pp, lam, lam_tstride, d_eta, lam_even](const double* r, double* p, const double* beta, double* w,
                                                   int nvec, double* pw, hipStream_t st) {
        Problem& Q = *pp;
        ConvSpec s;
        s.N1 = Q.N1;
        s.N2 = Q.N2;
        s.nvec = nvec;
        s.in_mode = IN_COMPACT;
        s.in = p;
        s.in_vstride = Q.p;
        s.rows_in = Q.n1;
        s.row_len = Q.n2;
        s.out_mode = OUT_COMPACT;
        s.out = w;
        s.out_vstride = Q.p;
        s.rows_out = Q.n1;
        s.cols_out = Q.n2;
        s.vin = p;
        s.vin_vstride = Q.p;
        s.eta = d_eta;
        s.lam = lam;
        s.lam_tstride = lam_tstride;
        s.vecs_per_theta = 1;
        s.lam_even = lam_even;
        s.pw_out = pw;
        s.upd_r = r;
        s.upd_beta = beta;
        conv_apply<double>(Q, s, st);
    };
}

// Sigma A^T w: compact in, full grid out, no nugget.
template <typename R>
void cov_full(Problem& P, const void* lam, const R* w, R* out, int nvec, hipStream_t st) {
    ConvSpec s;
    s.N1 = P.N1;
    s.N2 = P.N2;
    s.nvec = nvec;
    s.in_mode = IN_COMPACT;
    s.in = w;
    s.in_vstride = P.p;
    if (P.irregular) {  // A^T w on the grid first (FP64 sums), then the dense product
        const int64_t n = (int64_t)P.n1 * P.n2;
        P.irr.ensure(*P.ctx, (size_t)nvec * n * sizeof(R) + 256);
        irr_scatter<R, R>(P, w, P.p, nvec, P.irr.as<R>(), 1.0, nullptr, st);
        s.in_mode = IN_DENSE;
        s.in = P.irr.ptr;
        s.in_vstride = n;
        s.in_rstride = P.n2;
    }
    s.rows_in = P.n1;
    s.row_len = P.n2;
    s.out_mode = OUT_GRID;
    s.out = out;
    s.out_vstride = (int64_t)P.n1 * P.n2;
    s.rows_out = P.n1;
    s.cols_out = P.n2;
    s.scale = 1.0;
    s.lam = lam;
    s.lam_tstride = 0;
    s.vecs_per_theta = nvec;
    conv_apply<R>(P, s, st);
}

template <typename R>
const void* spec_ptr(Spectrum& S);
template <>
const void* spec_ptr<double>(Spectrum& S) { return S.s64.ptr; }
template <>
const void* spec_ptr<float>(Spectrum& S) { return S.s32.ptr; }

// ---- element kernels used by the drivers --------------------------------------------
template <typename R>
__global__ void k_gather(const R* __restrict__ full, const int32_t* __restrict__ cell, int64_t p, int64_t n,
                         R* __restrict__ out) {
    const int vec = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x)
        out[vec * p + i] = full[vec * n + cell[i]];
}

// full = 0 off the mask, scale * u on it
template <typename R>
__global__ void k_scatter(const R* __restrict__ u, const int32_t* __restrict__ cell, int64_t p, R* __restrict__ full,
                          double scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x)
        full[cell[i]] = (R)(scale * (double)u[i]);
}

// out[v * p + i] = c( cell_i - target_v ) from the embedding lag grid (row-major N1 x N2)
__global__ void k_cross_corr(const double* __restrict__ lag, int N1, int N2, const int32_t* __restrict__ cell,
                             int64_t p, int n2, const int64_t* __restrict__ targets, double* __restrict__ out) {
    const int v = blockIdx.y;
    const int64_t t = targets[v];
    const int tr = (int)(t / n2), tc = (int)(t % n2);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = cell[i];
        const int r = c / n2, cc = c - (c / n2) * n2;
        int l1 = (r - tr) % N1;
        if (l1 < 0) l1 += N1;
        int l2 = (cc - tc) % N2;
        if (l2 < 0) l2 += N2;
        out[v * p + i] = lag[(int64_t)l1 * N2 + l2];
    }
}

// y_b at observed cells: field value plus nugget noise (stream b, domain NOISE)
__global__ void k_boot_obs(const double* __restrict__ fields, int64_t n, const int32_t* __restrict__ cell, int64_t p,
                           double tau, uint64_t seed, double* __restrict__ yb) {
    const int b = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = cell[i];
        yb[b * p + i] = fields[b * n + c] + tau * philox_normal((uint32_t)c, (uint32_t)b, DOMAIN_NOISE, seed);
    }
}

// accumulate (x_b - xhat_b)^2 and (y_b - xhat_b)^2 at the targets over b in
// a fixed order (one thread per target)
__global__ void k_boot_acc(const double* __restrict__ fields, const double* __restrict__ xhat, int64_t n, int B,
                           const int64_t* __restrict__ targets, int64_t nt, double tau, uint64_t seed,
                           double* __restrict__ vx, double* __restrict__ vy) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = targets[t];
        double sx = 0.0, sy = 0.0;
        for (int b = 0; b < B; ++b) {
            const double x = fields[b * n + c];
            const double xh = xhat[b * n + c];
            const double y = x + tau * philox_normal((uint32_t)c, (uint32_t)b, DOMAIN_TARGET, seed);
            sx += (x - xh) * (x - xh);
            sy += (y - xh) * (y - xh);
        }
        vx[t] = sx / B;
        vy[t] = sy / B;
    }
}

__global__ void k_pick(const double* __restrict__ full, const int64_t* __restrict__ targets, int64_t nt,
                       double* __restrict__ out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x)
        out[t] = full[targets[t]];
}

__global__ void k_fill_eta(double* __restrict__ eta, const double* __restrict__ src, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) eta[i] = src[i];
}

dim3 grid1(int64_t n, int y = 1) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return dim3((unsigned)b, y);
}

// ---- solves ------------------------------------------------------------------------------
struct SolveStats {
    std::vector<int> iters;
    std::vector<double> relres;
};

// K X = B for nrhs compact right-hand sides in FP64 (device), with the
// operator's parameter points given by (spectrum pointers, eta).  FP32 form:
// restarted FP32 CG inside an FP64 residual refinement loop.
void solve_device(Problem& P, int precision, const void* lam64, const void* lam32, int64_t lam_tstride, int vpt,
                  const double* d_eta, int nrhs, const double* B, double* X, double rtol, int maxit, SolveStats& out,
                  hipStream_t st) {
    const int64_t p = P.p;
    const int64_t vn = (int64_t)nrhs * p;
    out.iters.assign(nrhs, 0);
    out.relres.assign(nrhs, 0.0);
    if (precision == KRY_FP64) {
        CgBuffers<double> cb{};
        auto lay = [&](Arena& a) {
            cb.r = a.take<double>(vn);
            cb.p = a.take<double>(vn);
            cb.w = a.take<double>(vn);
            cb.rr = a.take<double>(nrhs);
            cb.bnorm2 = a.take<double>(nrhs);
            cb.beta = a.take<double>(nrhs);
            cb.pw = a.take<double>(nrhs);
            cb.tmp = a.take<double>(nrhs);
            cb.partial = a.take<double>((size_t)nrhs * 256);
            cb.active = a.take<int>(nrhs);
            cb.iters = a.take<int>(nrhs);
            cb.limit = a.take<int>(nrhs);
        };
        Arena m;
        lay(m);
        P.scal.ensure(*P.ctx, m.off + 256);
        Arena a;
        a.base = P.scal.as<char>();
        lay(a);
        auto A = masked_op<double>(P, lam64, lam_tstride, vpt, d_eta);
        cg_run<double>(A, p, nrhs, B, X, rtol, maxit, cb, out.iters, out.relres, st, nullptr,
                       P.ctx->graphs && !P.ctx->prof.on && !P.no_graphs);
        return;
    }
    // mixed form
    CgBuffers<float> cb{};
    float *b32 = nullptr, *x32 = nullptr;
    double *r64 = nullptr, *t64 = nullptr, *nrm = nullptr, *part = nullptr;
    auto lay = [&](Arena& a) {
        cb.r = a.take<float>(vn);
        cb.p = a.take<float>(vn);
        cb.w = a.take<float>(vn);
        cb.rr = a.take<double>(nrhs);
        cb.bnorm2 = a.take<double>(nrhs);
        cb.beta = a.take<double>(nrhs);
        cb.pw = a.take<double>(nrhs);
        cb.tmp = a.take<double>(nrhs);
        cb.partial = a.take<double>((size_t)nrhs * 256);
        cb.active = a.take<int>(nrhs);
        cb.iters = a.take<int>(nrhs);
        cb.limit = a.take<int>(nrhs);
        b32 = a.take<float>(vn);
        x32 = a.take<float>(vn);
        r64 = a.take<double>(vn);
        t64 = a.take<double>(vn);
        nrm = a.take<double>(2 * (size_t)nrhs);
        part = a.take<double>((size_t)nrhs * 256);
    };
    Arena m;
    lay(m);
    P.scal.ensure(*P.ctx, m.off + 256);
    Arena a;
    a.base = P.scal.as<char>();
    lay(a);
    auto A32 = masked_op<float>(P, lam32, lam_tstride, vpt, d_eta);
    auto A64 = masked_op<double>(P, lam64, lam_tstride, vpt, d_eta);
    KRY_HIP(hipMemsetAsync(X, 0, vn * sizeof(double), st));
    KRY_HIP(hipMemcpyAsync(r64, B, vn * sizeof(double), hipMemcpyDeviceToDevice, st));
    dot_batched<double>(B, p, B, p, p, nrhs, part, nrm, st);
    std::vector<double> bn(nrhs), rn(nrhs);
    KRY_HIP(hipMemcpyAsync(bn.data(), nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
    const double inner = std::max(1e-5, rtol);
    // at most 12 corrections; the residual is measured after each of them,
    // so relres always describes the X that is returned
    for (int outer = 0;; ++outer) {
        // residual norms of the FP64 residual
        dot_batched<double>(r64, p, r64, p, p, nrhs, part, nrm, st);
        KRY_HIP(hipMemcpyAsync(rn.data(), nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        bool done = true;
        for (int v = 0; v < nrhs; ++v) {
            out.relres[v] = bn[v] > 0 ? std::sqrt(rn[v] / bn[v]) : 0.0;
            if (out.relres[v] > rtol) done = false;
        }
        if (done || outer == 12) break;
        // right-hand sides already at tolerance get a zero inner system, so
        // each solution is the same whatever else shares the launch
        convert<double, float>(r64, b32, vn, st);
        std::vector<int> lim(nrhs);
        bool any = false;
        for (int v = 0; v < nrhs; ++v) {
            const bool conv = out.relres[v] <= rtol;
            lim[v] = conv ? 0 : maxit - out.iters[v];
            if (conv) KRY_HIP(hipMemsetAsync(b32 + (size_t)v * p, 0, p * sizeof(float), st));
            any = any || lim[v] > 0;
        }
        if (!any) break;
        std::vector<int> it;
        std::vector<double> rr;
        cg_run<float>(A32, p, nrhs, b32, x32, inner, maxit, cb, it, rr, st, &lim,
                      P.ctx->graphs && !P.ctx->prof.on && !P.no_graphs);
        for (int v = 0; v < nrhs; ++v) out.iters[v] += it[v];
        add_f32(x32, X, vn, st);
        A64(X, t64, nrhs, st, nullptr);
        KRY_HIP(hipMemcpyAsync(r64, B, vn * sizeof(double), hipMemcpyDeviceToDevice, st));
        axpby<double>(t64, r64, -1.0, 1.0, p, nrhs, st);
    }
}

// ---- likelihood ----------------------------------------------------------------------------
struct LoglikWork {
    std::vector<double> gamma;  // per vector
    std::vector<int> steps;
    std::vector<int> point_stop;  // adaptive mode: step where each point settled (0: ran to the cap)
};

// Lanczos steps reported for point t: the most any of its probes ran, or the
// step where the point settled in the adaptive mode.
int steps_used(const LoglikWork& W, int t, int np, int first_recurrence) {
    int smax = 0;
    for (int k = 0; k < np; ++k) smax = std::max(smax, W.steps[(size_t)first_recurrence + k]);
    if (t < (int)W.point_stop.size() && W.point_stop[t]) smax = std::min(smax, W.point_stop[t]);
    return smax;
}

// Quadrature outputs that read shifted copies of the recurrences' tridiagonals:
// output v uses recurrence src[v] with T + shift[v] I (device arrays).
struct ShiftQuad {
    int nout = 0;
    const int* src = nullptr;
    const double* shift = nullptr;
};

// SLQ for `count` parameter points sharing the probes (common random numbers).
// Vectors are ordered theta-major: v = t * nprobe + k.  With sq, W.gamma holds
// sq->nout shifted quadratures instead of one per recurrence.
template <typename R>
void slq_device(Problem& P, const kry_opts* o, const void* lam, int64_t lam_tstride, const double* d_eta, int count,
                LoglikWork& W, std::vector<double>* alpha_out, std::vector<double>* beta_out, hipStream_t st,
                const ShiftQuad* sq = nullptr, const std::function<void(R*)>* fill_probes = nullptr) {
    const int np = nprobes_of(o);
    const int nvec = count * np;
    // the adaptive mode applies to log-determinants, not to a caller that
    // asks for the coefficients of exactly lanczos_steps steps
    const bool adaptive = o->lanczos_rtol > 0 && !alpha_out;
    const int m = adaptive ? o->lanczos_max_steps : o->lanczos_steps;
    const bool reorth = o->reorth != 0;
    const int64_t p = P.p;
    const int nblk = dot_blocks(p);
    const int nout = sq ? sq->nout : nvec;
    LanczosBuffers<R> B{};
    LanczosAdaptive ad{};
    R* Z = nullptr;
    double* gamma = nullptr;
    auto lay = [&](Arena& a) {
        if (adaptive) {
            ad.g_prev = a.take<double>(nout);
            ad.g_cur = a.take<double>(nout);
            ad.g_final = a.take<double>(nout);
            ad.stop = a.take<int>(nout / np);
            ad.done = a.take<int>(1);
        }
        Z = a.take<R>((size_t)nvec * p);
        B.Q = a.take<R>((size_t)(reorth ? m + 1 : 3) * nvec * p);
        B.W = a.take<R>((size_t)nvec * p);
        B.alpha = a.take<double>((size_t)m * nvec);
        B.beta = a.take<double>((size_t)m * nvec);
        B.znorm2 = a.take<double>(nvec);
        B.scale = a.take<double>(nvec);
        B.active = a.take<int>(nvec);
        B.steps = a.take<int>(nvec);
        B.partial = a.take<double>((size_t)nvec * (m + 1) * nblk);
        B.h = a.take<double>((size_t)nvec * (m + 1));
        gamma = a.take<double>(sq ? std::max(nvec, sq->nout) : nvec);
    };
    with_arena(P, lay);
    if (fill_probes) {
        (*fill_probes)(Z);
    } else {
        make_probes<R>(P, np, o->seed, o->probe_kind == KRY_PROBE_COLOURED ? o->colour_period : 0, Z, st);
        for (int t = 1; t < count; ++t)
            KRY_HIP(hipMemcpyAsync(Z + (size_t)t * np * p, Z, (size_t)np * p * sizeof(R), hipMemcpyDeviceToDevice,
                                   st));
    }
    auto A = masked_op<R>(P, lam, lam_tstride, np, d_eta);
    if (adaptive) {
        ad.rtol = o->lanczos_rtol;
        ad.nout = nout;
        ad.per_point = np;
        ad.src = sq ? sq->src : nullptr;
        ad.shift = sq ? sq->shift : nullptr;
    }
    lanczos_run<R>(A, p, nvec, m, reorth, Z, B, st, adaptive ? &ad : nullptr);
    if (sq) quadrature(B.alpha, B.beta, B.steps, B.znorm2, nout, nvec, gamma, st, sq->src, sq->shift);
    else quadrature(B.alpha, B.beta, B.steps, B.znorm2, nvec, nvec, gamma, st);
    W.gamma.resize(nout);
    W.steps.resize(nvec);
    W.point_stop.assign(nout / np, 0);
    KRY_HIP(hipMemcpyAsync(W.gamma.data(), gamma, nout * sizeof(double), hipMemcpyDeviceToHost, st));
    if (adaptive) {
        // settled points keep the values of the step where they settled
        std::vector<double> gf(nout);
        KRY_HIP(hipMemcpyAsync(gf.data(), ad.g_final, nout * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipMemcpyAsync(W.point_stop.data(), ad.stop, (nout / np) * sizeof(int), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        for (int v = 0; v < nout; ++v)
            if (W.point_stop[v / np]) W.gamma[v] = gf[v];
    }
    KRY_HIP(hipMemcpyAsync(W.steps.data(), B.steps, nvec * sizeof(int), hipMemcpyDeviceToHost, st));
    if (alpha_out) {
        alpha_out->resize((size_t)m * nvec);
        beta_out->resize((size_t)m * nvec);
        KRY_HIP(hipMemcpyAsync(alpha_out->data(), B.alpha, (size_t)m * nvec * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipMemcpyAsync(beta_out->data(), B.beta, (size_t)m * nvec * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    KRY_HIP(hipStreamSynchronize(st));
}

void combine(const double* vals, int N, bool coloured, double* est, double* se) {
    double mean = 0;
    for (int i = 0; i < N; ++i) mean += vals[i];
    mean /= N;
    double ss = 0;
    for (int i = 0; i < N; ++i) ss += (vals[i] - mean) * (vals[i] - mean);
    const double sd = N > 1 ? std::sqrt(ss / (N - 1)) : 0.0;
    if (coloured) {
        *est = mean * N;
        *se = std::sqrt((double)N) * sd;
    } else {
        *est = mean;
        *se = sd / std::sqrt((double)N);
    }
}

void assemble(kry_loglik_result* r, int64_t p, double logdet, double se, double Q, double sigma2) {
    const double two_pi = 6.283185307179586476925286766559;
    r->p = p;
    r->logdet = logdet;
    r->logdet_se = se;
    r->quad = Q;
    r->loglik = -0.5 * ((double)p * std::log(two_pi * sigma2) + logdet + Q / sigma2);
    r->sigma2_hat = Q / (double)p;
    r->loglik_profiled = -0.5 * ((double)p * (std::log(two_pi) + std::log(r->sigma2_hat) + 1.0) + logdet);
}

// ---- covariates: generalised least squares ---------------------------------------------
// Small dense symmetric positive definite matrices (q <= KRY_MAX_COVARIATES),
// row-major, on the host.  In-place lower Cholesky factor; false when a
// pivot falls to rel_tol times its column's diagonal or below (the column is
// numerically a combination of the earlier ones).
bool chol_small(std::vector<double>& A, int q, double rel_tol) {
    for (int j = 0; j < q; ++j) {
        double d = A[j * q + j];
        const double ajj = d;
        for (int k = 0; k < j; ++k) d -= A[j * q + k] * A[j * q + k];
        if (!(d > rel_tol * ajj) || !(ajj > 0)) return false;
        const double l = std::sqrt(d);
        A[j * q + j] = l;
        for (int i = j + 1; i < q; ++i) {
            double v = A[i * q + j];
            for (int k = 0; k < j; ++k) v -= A[i * q + k] * A[j * q + k];
            A[i * q + j] = v / l;
        }
    }
    return true;
}

// x = (L L^T)^{-1} b with the factor from chol_small.
std::vector<double> chol_solve(const std::vector<double>& L, int q, std::vector<double> b) {
    for (int i = 0; i < q; ++i) {
        for (int k = 0; k < i; ++k) b[i] -= L[i * q + k] * b[k];
        b[i] /= L[i * q + i];
    }
    for (int i = q - 1; i >= 0; --i) {
        for (int k = i + 1; k < q; ++k) b[i] -= L[k * q + i] * b[k];
        b[i] /= L[i * q + i];
    }
    return b;
}

double chol_logdet(const std::vector<double>& L, int q) {
    double s = 0;
    for (int i = 0; i < q; ++i) s += 2.0 * std::log(L[i * q + i]);
    return s;
}

// GLS pieces at one parameter point from M[a * nd + b] = D_b^T K^{-1} D_a,
// nd = q + 1, D_0 = yc = y - X beta_ols, D_j = X_j:
//   G = X^T K^{-1} X,  g = X^T K^{-1} yc,  delta = G^{-1} g,
//   beta_hat = beta_ols + delta,  Q = yc^T K^{-1} yc - g^T delta
// (the GLS residual y - X beta_hat = yc - X delta, and Q is its K^{-1} norm;
// off-diagonal pairs are averaged, K being symmetric).
struct Gls {
    double Q = 0, logdet_G = 0;
    std::vector<double> delta, beta, Ginv_diag;
};

Gls gls_combine(const Problem& P, const double* M) {
    const int q = P.q, nd = q + 1;
    Gls r;
    std::vector<double> G((size_t)q * q), g(q);
    for (int i = 0; i < q; ++i) {
        g[i] = 0.5 * (M[0 * nd + (i + 1)] + M[(i + 1) * nd + 0]);
        for (int j = 0; j < q; ++j) G[i * q + j] = 0.5 * (M[(i + 1) * nd + (j + 1)] + M[(j + 1) * nd + (i + 1)]);
    }
    KRY_REQUIRE(chol_small(G, q, 1e-13), "X^T K^{-1} X is not numerically positive definite");
    r.logdet_G = chol_logdet(G, q);
    r.delta = chol_solve(G, q, g);
    double gd = 0;
    for (int i = 0; i < q; ++i) gd += g[i] * r.delta[i];
    r.Q = M[0] - gd;
    r.beta.resize(q);
    for (int i = 0; i < q; ++i) r.beta[i] = P.beta_ols[i] + r.delta[i];
    r.Ginv_diag.resize(q);
    for (int i = 0; i < q; ++i) {
        std::vector<double> e(q, 0.0);
        e[i] = 1.0;
        r.Ginv_diag[i] = chol_solve(G, q, e)[i];
    }
    return r;
}

// Likelihood assembly with covariates: maximum likelihood at beta_hat
// (assemble with the GLS Q), or the restricted likelihood (reml) of the
// error contrasts with m = p - q:
//   l = -1/2 [m log(2 pi sigma2) + logdet + log det G - log det X^T X + Q / sigma2],
//   sigma2_hat = Q / m,  l_p = -1/2 [m (log 2 pi + log sigma2_hat + 1) + logdet + log det G - log det X^T X];
// beta_se from sigma2_hat G^{-1}.
void assemble_gls(kry_loglik_result* r, const Problem& P, double logdet, double se, const Gls& g, double sigma2,
                  bool reml) {
    assemble(r, P.p, logdet, se, g.Q, sigma2);
    if (reml) {
        const double two_pi = 6.283185307179586476925286766559;
        const double m = (double)(P.p - P.q);
        const double extra = logdet + g.logdet_G - P.logdet_xx;
        r->loglik = -0.5 * (m * std::log(two_pi * sigma2) + extra + g.Q / sigma2);
        r->sigma2_hat = g.Q / m;
        r->loglik_profiled = -0.5 * (m * (std::log(two_pi) + std::log(r->sigma2_hat) + 1.0) + extra);
    }
    r->ncov = P.q;
    for (int i = 0; i < P.q; ++i) {
        r->beta[i] = g.beta[i];
        r->beta_se[i] = std::sqrt(r->sigma2_hat * g.Ginv_diag[i]);
    }
    r->logdet_xkx = g.logdet_G;
}

// The nd = q + 1 vectors D_0 = yc, D_j = X_j (D_0 = y without covariates),
// copied contiguously to dst (nd x p, FP64).
void copy_rhs_set(const Problem& P, double* dst, hipStream_t st) {
    const size_t vb = (size_t)P.p * sizeof(double);
    if (P.q == 0) {
        KRY_HIP(hipMemcpyAsync(dst, P.y64.ptr, vb, hipMemcpyDeviceToDevice, st));
        return;
    }
    KRY_HIP(hipMemcpyAsync(dst, P.yc64.ptr, vb, hipMemcpyDeviceToDevice, st));
    KRY_HIP(hipMemcpyAsync(dst + P.p, P.X64.ptr, (size_t)P.q * vb, hipMemcpyDeviceToDevice, st));
}

// genGK quadratic form and x_k* (Algorithm 1 with the one-product reading:
// s_i = Sigma v_i is carried along, so each step needs one product Sigma A^T u).
struct GkOut {
    std::vector<double> alpha, beta, z;
    double J = 0;
    double beta1 = 0;
    const void* V = nullptr;   // V_k, k full-grid vectors (workspace)
    const void* Sv = nullptr;  // Sigma V_k
};

// data64 (device, compact FP64, nullable) replaces the problem's data as b.
template <typename R>
void gengk_device(Problem& P, const Matern& th, const kry_opts* o, GkOut& G, double* x_full_host, hipStream_t st,
                  const double* data64 = nullptr) {
    const int k = o->gk_steps;
    const bool reorth = o->reorth != 0;
    const int64_t p = P.p, n = (int64_t)P.n1 * P.n2;
    const double tau2 = th.tau2 / th.sigma2;  // unit-variance form: sigma^2 = 1, tau^2 = eta
    const double sig2 = 1.0;
    KRY_REQUIRE(tau2 > 0, "genGK needs a positive nugget");
    const double tau = std::sqrt(tau2);
    Spectrum& S = problem_spectrum(P, th, st);
    const void* lam = spec_ptr<R>(S);
    R *U = nullptr, *V = nullptr, *Sv = nullptr, *u = nullptr, *g = nullptr, *t = nullptr, *xi = nullptr, *sx = nullptr;
    R* b = nullptr;
    double *dots = nullptr, *part = nullptr, *coef = nullptr;
    const int nb = dot_blocks(n);
    auto lay = [&](Arena& a) {
        U = a.take<R>((size_t)(k + 1) * p);
        V = a.take<R>((size_t)(k + 1) * n);
        Sv = a.take<R>((size_t)(k + 1) * n);
        g = a.take<R>(p);
        t = a.take<R>(n);
        xi = a.take<R>(n);
        sx = a.take<R>(n);
        b = a.take<R>(p);
        dots = a.take<double>(4 * (size_t)(k + 2));
        part = a.take<double>((size_t)nb * (k + 2));
        coef = a.take<double>((size_t)(k + 2));
    };
    with_arena(P, lay);
    (void)u;
    const int32_t* cell = P.cell.as<int32_t>();
    // b = y (compact data in the working precision)
    if (data64) convert<double, R>(data64, b, p, st);
    else if (sizeof(R) == 8) KRY_HIP(hipMemcpyAsync(b, P.y64.ptr, p * sizeof(double), hipMemcpyDeviceToDevice, st));
    else KRY_HIP(hipMemcpyAsync(b, P.y32.ptr, p * sizeof(float), hipMemcpyDeviceToDevice, st));
    auto dot = [&](const R* x, const R* y, int64_t len) {
        double h;
        dot_batched<R>(x, len, y, len, len, 1, part, dots, st);
        KRY_HIP(hipMemcpyAsync(&h, dots, sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        return h;
    };
    auto scatter = [&](const R* src, R* full, double sc) {  // sc A^T src
        if (P.irregular) {
            irr_scatter<R, R>(P, src, p, 1, full, sc, nullptr, st);
            return;
        }
        KRY_HIP(hipMemsetAsync(full, 0, n * sizeof(R), st));
        hipLaunchKernelGGL(k_scatter<R>, grid1(p), dim3(256), 0, st, src, cell, p, full, sc);
        KRY_HIP(hipGetLastError());
    };
    auto gather = [&](const R* full, R* out) {  // A full
        if (P.irregular) {
            irr_gather<R, R>(P, full, 1, out, nullptr, nullptr, 1, nullptr, st);
            return;
        }
        hipLaunchKernelGGL(k_gather<R>, grid1(p), dim3(256), 0, st, full, cell, p, n, out);
        KRY_HIP(hipGetLastError());
    };
    // orthogonalise x against the first nq columns of M (Euclidean, scaled by w) : x -= M (M^T x) * w
    auto reorth_against = [&](const R* Mbase, int64_t len, int nq, R* x, const R* Tbase, R* x2, double w) {
        // coefficients c_i = T_i . x (T = M for Euclidean, T = Sigma V for the Sigma-inner product)
        std::vector<double> c(nq);
        for (int i = 0; i < nq; ++i) c[i] = dot(Tbase + (size_t)i * len, x, len) * w;
        for (int i = 0; i < nq; ++i) {
            axpby<R>(Mbase + (size_t)i * len, x, -c[i], 1.0, len, 1, st);
            if (x2) axpby<R>(Tbase + (size_t)i * len, x2, -c[i], 1.0, len, 1, st);
        }
    };

    G.alpha.clear();
    G.beta.clear();
    const double beta1 = std::sqrt(dot(b, b, p)) / tau;
    KRY_REQUIRE(beta1 > 0, "genGK needs nonzero data");
    G.beta1 = beta1;
    G.beta.push_back(beta1);
    // u1 = b / beta1
    KRY_HIP(hipMemcpyAsync(U, b, p * sizeof(R), hipMemcpyDeviceToDevice, st));
    axpby<R>(b, U, 0.0, 1.0 / beta1, p, 1, st);
    // xi = A^T u1 / tau2, Sigma xi = Sigma A^T u1 / tau2
    scatter(U, xi, 1.0 / tau2);
    cov_full<R>(P, lam, U, t, 1, st);
    KRY_HIP(hipMemcpyAsync(sx, t, n * sizeof(R), hipMemcpyDeviceToDevice, st));
    axpby<R>(t, sx, 0.0, 1.0 / tau2, n, 1, st);
    double alpha = std::sqrt(dot(xi, sx, n));
    G.alpha.push_back(alpha);
    KRY_HIP(hipMemcpyAsync(V, xi, n * sizeof(R), hipMemcpyDeviceToDevice, st));
    axpby<R>(xi, V, 0.0, 1.0 / alpha, n, 1, st);
    KRY_HIP(hipMemcpyAsync(Sv, sx, n * sizeof(R), hipMemcpyDeviceToDevice, st));
    axpby<R>(sx, Sv, 0.0, 1.0 / alpha, n, 1, st);
    for (int i = 0; i < k; ++i) {
        R* vi = V + (size_t)i * n;
        R* si = Sv + (size_t)i * n;
        R* ui = U + (size_t)i * p;
        R* un = U + (size_t)(i + 1) * p;
        // g = A Sigma v_i - alpha_i u_i
        gather(si, g);
        axpby<R>(ui, g, -alpha, 1.0, p, 1, st);
        if (reorth) {
            for (int pass = 0; pass < 2; ++pass) reorth_against(U, p, i + 1, g, U, nullptr, 1.0 / tau2);
        }
        const double beta = std::sqrt(dot(g, g, p)) / tau;
        G.beta.push_back(beta);
        KRY_HIP(hipMemcpyAsync(un, g, p * sizeof(R), hipMemcpyDeviceToDevice, st));
        axpby<R>(g, un, 0.0, 1.0 / beta, p, 1, st);
        if (i == k - 1) break;  // B_k needs alpha_1..alpha_k, beta_2..beta_{k+1}
        // xi = A^T u_{i+1} / tau2 - beta v_i ; Sigma xi = Sigma A^T u_{i+1} / tau2 - beta s_i
        scatter(un, xi, 1.0 / tau2);
        axpby<R>(vi, xi, -beta, 1.0, n, 1, st);
        cov_full<R>(P, lam, un, t, 1, st);
        KRY_HIP(hipMemcpyAsync(sx, si, n * sizeof(R), hipMemcpyDeviceToDevice, st));
        axpby<R>(t, sx, 1.0 / tau2, -beta, n, 1, st);
        if (reorth) {
            for (int pass = 0; pass < 2; ++pass) reorth_against(V, n, i + 1, xi, Sv, sx, 1.0);
        }
        alpha = std::sqrt(dot(xi, sx, n));
        G.alpha.push_back(alpha);
        R* vn = V + (size_t)(i + 1) * n;
        R* sn = Sv + (size_t)(i + 1) * n;
        KRY_HIP(hipMemcpyAsync(vn, xi, n * sizeof(R), hipMemcpyDeviceToDevice, st));
        axpby<R>(xi, vn, 0.0, 1.0 / alpha, n, 1, st);
        KRY_HIP(hipMemcpyAsync(sn, sx, n * sizeof(R), hipMemcpyDeviceToDevice, st));
        axpby<R>(sx, sn, 0.0, 1.0 / alpha, n, 1, st);
    }
    // projected Tikhonov problem (eq. xhat_est): (B^T B + I / sigma^2) z = B^T beta1 e1
    // B^T B is tridiagonal: diag alpha_i^2 + beta_{i+1}^2, off-diag alpha_{i+1} beta_{i+1}
    std::vector<double> dg(k), od(k > 1 ? k - 1 : 1), rhs(k, 0.0);
    for (int i = 0; i < k; ++i) dg[i] = G.alpha[i] * G.alpha[i] + G.beta[i + 1] * G.beta[i + 1] + 1.0 / sig2;
    for (int i = 0; i + 1 < k; ++i) od[i] = G.alpha[i + 1] * G.beta[i + 1];
    rhs[0] = G.alpha[0] * beta1;
    // symmetric tridiagonal solve (Thomas algorithm; the matrix is positive definite)
    std::vector<double> cp(k), dp(k);
    cp[0] = k > 1 ? od[0] / dg[0] : 0.0;
    dp[0] = rhs[0] / dg[0];
    for (int i = 1; i < k; ++i) {
        const double den = dg[i] - od[i - 1] * cp[i - 1];
        cp[i] = (i + 1 < k) ? od[i] / den : 0.0;
        dp[i] = (rhs[i] - od[i - 1] * dp[i - 1]) / den;
    }
    G.V = V;
    G.Sv = Sv;
    G.z.assign(k, 0.0);
    G.z[k - 1] = dp[k - 1];
    for (int i = k - 2; i >= 0; --i) G.z[i] = dp[i] - cp[i] * G.z[i + 1];
    // J = ||B z - beta1 e1||^2 + ||z||^2 / sigma^2
    double J = 0, zz = 0;
    for (int i = 0; i <= k; ++i) {
        double bz = 0;
        if (i < k) bz += G.alpha[i] * G.z[i];
        if (i >= 1) bz += G.beta[i] * G.z[i - 1];
        if (i == 0) bz -= beta1;
        J += bz * bz;
    }
    for (int i = 0; i < k; ++i) zz += G.z[i] * G.z[i];
    G.J = J + zz / sig2;
    if (x_full_host) {
        // x_k* = Sigma V_k z = sum_i z_i s_i
        KRY_HIP(hipMemsetAsync(t, 0, n * sizeof(R), st));
        for (int i = 0; i < k; ++i) axpby<R>(Sv + (size_t)i * n, t, G.z[i], 1.0, n, 1, st);
        std::vector<R> h(n);
        KRY_HIP(hipMemcpyAsync(h.data(), t, n * sizeof(R), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        for (int64_t i = 0; i < n; ++i) x_full_host[i] = (double)h[i];
    }
}

// Points with equal range, smoothness and anisotropy: their covariances
// differ only in the nugget ratio.  Returns the group of every point and the
// first point of every group.
std::vector<int> shift_groups(const kry_matern* th, int count, std::vector<int>& rep) {
    std::vector<int> grp(count);
    rep.clear();
    for (int t = 0; t < count; ++t) {
        int g = 0;
        for (; g < (int)rep.size(); ++g) {
            const kry_matern& a = th[rep[g]];
            if (a.range == th[t].range && a.nu == th[t].nu && a.aniso_ratio == th[t].aniso_ratio &&
                a.aniso_angle == th[t].aniso_angle)
                break;
        }
        if (g == (int)rep.size()) rep.push_back(t);
        grp[t] = g;
    }
    return grp;
}

// Likelihood of `count` points where every group of nugget-only variants
// shares its Krylov spaces: Lanczos on the nugget-free Sigma_oo per probe and
// group, quadrature of T + eta I per point; multi-shift CG on Sigma_oo with
// shifts eta for the quadratic forms.
void loglik_points_shared(Problem& P, const kry_matern* thetas, int count, const kry_opts* o,
                          kry_loglik_result* out, hipStream_t st) {
    Ctx& C = *P.ctx;
    const int np = nprobes_of(o);
    const int64_t nspec = (int64_t)(P.N2 / 2 + 1) * P.N1;
    const bool fp32 = o->precision == KRY_FP32;
    const int64_t p = P.p;
    std::vector<int> rep;
    const std::vector<int> grp = shift_groups(thetas, count, rep);
    const int G = (int)rep.size();
    // Multi-shift CG runs one Krylov space per (group, right-hand side): the
    // data and, with covariates, every covariate column (nd in all), each
    // position holding its own copy of the group's spectrum (positions are
    // permuted as groups finish).  The SLQ uses copy 0 of every group.
    const int nd = 1 + P.q;
    const bool need_ms = o->solver == KRY_SOLVER_CG || P.q > 0;
    const int Gm = need_ms ? G * nd : G;
    const int64_t gstride = (int64_t)(need_ms ? nd : 1) * nspec;
    P.spec_multi64.ensure(C, (size_t)Gm * nspec * sizeof(double));
    if (fp32) P.spec_multi32.ensure(C, (size_t)G * nspec * sizeof(float));
    for (int g = 0; g < G; ++g) {
        const Matern th = to_matern(&thetas[rep[g]]);
        double lo, hi;
        double* dst = P.spec_multi64.as<double>() + (size_t)g * gstride;
        spectrum_device(P, P.N1, P.N2, th, dst, &lo, &hi, st);
        spectrum_scale(dst, nspec, 1.0 / ((double)P.N1 * P.N2), false, dst,
                       fp32 ? P.spec_multi32.as<float>() + (size_t)g * nspec : nullptr, st);
        if (need_ms)
            for (int a = 1; a < nd; ++a)
                KRY_HIP(hipMemcpyAsync(dst + (size_t)a * nspec, dst, nspec * sizeof(double), hipMemcpyDeviceToDevice,
                                       st));
    }
    // zero nugget per position, and per (point, probe) output its recurrence and shift
    const int nout = count * np;
    std::vector<double> eta(count), shift(nout), zeros(Gm, 0.0);
    std::vector<int> src(nout);
    for (int t = 0; t < count; ++t) {
        eta[t] = thetas[t].tau2 / thetas[t].sigma2;
        for (int k = 0; k < np; ++k) {
            src[(size_t)t * np + k] = grp[t] * np + k;
            shift[(size_t)t * np + k] = eta[t];
        }
    }
    DevBuf& sb = P.tmp3;
    const size_t zoff = 0, soff = ((size_t)Gm * 8 + 255) & ~size_t(255);
    const size_t ioff = soff + (((size_t)nout * 8 + 255) & ~size_t(255));
    sb.ensure(C, ioff + (size_t)nout * 4 + 256);
    double* d_zero = reinterpret_cast<double*>(sb.as<char>() + zoff);
    double* d_shift = reinterpret_cast<double*>(sb.as<char>() + soff);
    int* d_src = reinterpret_cast<int*>(sb.as<char>() + ioff);
    KRY_HIP(hipMemcpyAsync(d_zero, zeros.data(), Gm * sizeof(double), hipMemcpyHostToDevice, st));
    KRY_HIP(hipMemcpyAsync(d_shift, shift.data(), nout * sizeof(double), hipMemcpyHostToDevice, st));
    KRY_HIP(hipMemcpyAsync(d_src, src.data(), nout * sizeof(int), hipMemcpyHostToDevice, st));
    ShiftQuad sq{nout, d_src, d_shift};
    LoglikWork W;
    auto run_slq = [&](Problem& Qp, hipStream_t s) {
        if (fp32) slq_device<float>(Qp, o, P.spec_multi32.ptr, nspec, d_zero, G, W, nullptr, nullptr, s, &sq);
        else slq_device<double>(Qp, o, P.spec_multi64.ptr, gstride, d_zero, G, W, nullptr, nullptr, s, &sq);
    };
    // log-determinants first, then the multi-shift solves (running the two
    // on separate streams was measured to gain nothing: each fills the device)
    run_slq(P, st);
    std::vector<double> Q(count, 0.0), relres(count, 0.0), M;
    std::vector<int> iters(count, 0);
    std::vector<Gls> gls(P.q > 0 ? count : 0);
    double* D = nullptr;  // the nd right-hand-side vectors
    if (need_ms) {
        if (P.q == 0) {
            D = P.y64.as<double>();
        } else {
            P.tmp2.ensure(C, (size_t)nd * p * sizeof(double) + 256);
            D = P.tmp2.as<double>();
            copy_rhs_set(P, D, st);
        }
        const int S = count * nd;
        const int nblk = dot_blocks(p);
        // power-of-two columns form p . w in the product, from the spectrum of p
        const int fused_pw = P.irregular ? 0 : spectral_qf_count(P.N1, P.N2);
        MsCgBuffers B{};
        auto lay = [&](Arena& a) {
            B.r = a.take<double>((size_t)Gm * p);
            B.p = a.take<double>((size_t)Gm * p);
            B.w = a.take<double>((size_t)Gm * p);
            for (double** d : {&B.rr, &B.pw, &B.alpha, &B.alpha_old, &B.beta, &B.beta_old, &B.bnorm2})
                *d = a.take<double>(Gm);
            B.rc = a.take<double>((size_t)(1 + nd) * Gm);
            for (double** d : {&B.zeta, &B.zeta_old, &B.zeta_new, &B.alpha_s, &B.sigma, &B.relres})
                *d = a.take<double>(S);
            B.d = a.take<double>((size_t)S * nd);
            B.Q = a.take<double>((size_t)S * nd);
            for (int** d : {&B.active, &B.iters, &B.limit, &B.pos, &B.list}) *d = a.take<int>(S);
            B.gram = a.take<double>((size_t)nd * nd);
            B.rhs = a.take<int>(Gm);
            B.partial = a.take<double>((size_t)(1 + nd) * Gm * nblk);
            B.partial_pw = a.take<double>((size_t)Gm * std::max(nblk, fused_pw));
        };
        with_arena(P, lay);
        // one spectrum per vector here, so the column stage's spectrum reads
        // are a third of its bytes; even spectra halve them
        bool even = true;
        for (int g = 0; g < G; ++g) even = even && matern_even(to_matern(&thetas[rep[g]]));
        auto A = masked_op<double>(P, P.spec_multi64.ptr, nspec, 1, d_zero, even);
        const MsFusedFn fused =
            P.irregular ? MsFusedFn() : masked_op_update(P, P.spec_multi64.ptr, nspec, d_zero, even);
        double* lam64 = P.spec_multi64.as<double>();
        auto swp = [&](int a, int b) { swap_vectors<double>(lam64, nspec, a, b, nspec, st); };
        // shift entry t nd + a: point t's system with right-hand side D_a
        std::vector<int> gos(S), rhs(Gm);
        std::vector<double> sig(S);
        for (int t = 0; t < count; ++t)
            for (int a = 0; a < nd; ++a) {
                gos[(size_t)t * nd + a] = grp[t] * nd + a;
                sig[(size_t)t * nd + a] = eta[t];
            }
        for (int g = 0; g < Gm; ++g) rhs[g] = g % nd;
        std::vector<int> it;
        std::vector<double> rr;
        mscg_run(A, P.irregular ? nullptr : &fused, fused_pw, swp, p, Gm, gos, sig, D, nd, rhs, o->cg_rtol, o->cg_maxit, B, it,
                 rr, M, st);
        for (int t = 0; t < count; ++t) {
            for (int a = 0; a < nd; ++a) {
                iters[t] = std::max(iters[t], it[(size_t)t * nd + a]);
                relres[t] = std::max(relres[t], rr[(size_t)t * nd + a]);
            }
            const double* Mt = M.data() + (size_t)t * nd * nd;
            if (P.q > 0) gls[t] = gls_combine(P, Mt);
            Q[t] = P.q > 0 ? gls[t].Q : Mt[0];
        }
    }
    if (o->solver != KRY_SOLVER_CG) {
        double* resid = nullptr;
        if (P.q > 0) {
            P.tmp4.ensure(C, (size_t)p * sizeof(double) + 256);
            resid = P.tmp4.as<double>();
        }
        for (int t = 0; t < count; ++t) {
            GkOut Gk;
            const Matern th = to_matern(&thetas[t]);
            if (P.q > 0) {  // genGK on the GLS residual yc - X delta
                KRY_HIP(hipMemcpyAsync(resid, P.yc64.ptr, p * sizeof(double), hipMemcpyDeviceToDevice, st));
                for (int j = 0; j < P.q; ++j)
                    axpby<double>(P.X64.as<double>() + (size_t)j * p, resid, -gls[t].delta[j], 1.0, p, 1, st);
            }
            if (fp32) gengk_device<float>(P, th, o, Gk, nullptr, st, resid);
            else gengk_device<double>(P, th, o, Gk, nullptr, st, resid);
            Q[t] = Gk.J;
            if (P.q > 0) gls[t].Q = Gk.J;
            iters[t] = o->gk_steps;
            relres[t] = 0.0;
        }
    }
    for (int t = 0; t < count; ++t) {
        double est, se;
        combine(W.gamma.data() + (size_t)t * np, np, o->probe_kind == KRY_PROBE_COLOURED, &est, &se);
        kry_loglik_result& r = out[t];
        std::memset(&r, 0, sizeof(r));
        if (P.q > 0) assemble_gls(&r, P, est, se, gls[t], thetas[t].sigma2, o->reml != 0);
        else assemble(&r, p, est, se, Q[t], thetas[t].sigma2);
        r.lanczos_steps_used = steps_used(W, t, np, grp[t] * np);
        r.cg_iters = iters[t];
        r.cg_relres = relres[t];
    }
}

// Likelihood of one parameter point per problem for problems that share an
// embedding.  Every masked product covers all of them at once: the stage
// kernels read a per-vector problem table (mask, block, spectrum), and the
// Krylov vectors are stored with the largest observed count as stride, zero
// past each problem's own count.  Probes and data are each problem's own.
// Q carries the workspace (a view of any problem on the same context); its
// block sizes and table are set for the call and restored after it.
template <typename R>
void loglik_multi_group(Problem& Q, const std::vector<Problem*>& probs, const kry_matern* th, const kry_opts* o,
                        kry_loglik_result* out, hipStream_t st) {
    Ctx& C = *Q.ctx;
    const int G = (int)probs.size();
    const int np = nprobes_of(o);
    struct Restore {
        Problem& q;
        int n1, n2;
        int64_t p;
        double dx1, dx2;
        ~Restore() {
            q.tab = nullptr;
            q.n1 = n1;
            q.n2 = n2;
            q.p = p;
            q.dx1 = dx1;
            q.dx2 = dx2;
        }
    } restore{Q, Q.n1, Q.n2, Q.p, Q.dx1, Q.dx2};
    int n1m = 0, n2m = 0;
    int64_t pm = 0;
    for (Problem* q : probs) {
        n1m = std::max(n1m, q->n1);
        n2m = std::max(n2m, q->n2);
        pm = std::max(pm, q->p);
    }
    Q.n1 = n1m;
    Q.n2 = n2m;
    Q.p = pm;
    const int64_t nspec = (int64_t)(Q.N2 / 2 + 1) * Q.N1;
    Q.spec_multi64.ensure(C, (size_t)G * nspec * sizeof(double));
    if (sizeof(R) == 4) Q.spec_multi32.ensure(C, (size_t)G * nspec * sizeof(float));
    std::vector<ProbDesc> tab(G);
    std::vector<double> eta(G);
    for (int g = 0; g < G; ++g) {
        Problem& Pg = *probs[g];
        double lo, hi;
        double* d64 = Q.spec_multi64.as<double>() + (size_t)g * nspec;
        float* d32 = sizeof(R) == 4 ? Q.spec_multi32.as<float>() + (size_t)g * nspec : nullptr;
        // the spectrum uses Q's workspace with Pg's spacing (the problems'
        // own workspaces may be in use elsewhere)
        Q.dx1 = Pg.dx1;
        Q.dx2 = Pg.dx2;
        spectrum_device(Q, Q.N1, Q.N2, to_matern(&th[g]), d64, &lo, &hi, st);
        spectrum_scale(d64, nspec, 1.0 / ((double)Q.N1 * Q.N2), false, d64, d32, st);
        tab[g] = ProbDesc{Pg.bits.as<uint32_t>(), Pg.base.as<uint32_t>(), Pg.words_per_row, Pg.n1, Pg.n2, Pg.p,
                          d64, d32};
        eta[g] = th[g].tau2 / th[g].sigma2;
    }
    // table, nugget ratios, padded data and solutions
    const size_t tab_b = ((size_t)G * sizeof(ProbDesc) + 255) & ~size_t(255);
    const size_t eta_b = ((size_t)G * 8 + 255) & ~size_t(255);
    DevBuf& tb = Q.tmp3;
    tb.ensure(C, tab_b + eta_b + 2 * (size_t)G * pm * sizeof(double) + ((size_t)G * 257 + 8) * sizeof(double));
    ProbDesc* d_tab = tb.as<ProbDesc>();
    double* d_eta = reinterpret_cast<double*>(tb.as<char>() + tab_b);
    double* Yd = reinterpret_cast<double*>(tb.as<char>() + tab_b + eta_b);
    double* Xd = Yd + (size_t)G * pm;
    double* part = Xd + (size_t)G * pm;
    KRY_HIP(hipMemcpyAsync(d_tab, tab.data(), G * sizeof(ProbDesc), hipMemcpyHostToDevice, st));
    KRY_HIP(hipMemcpyAsync(d_eta, eta.data(), G * sizeof(double), hipMemcpyHostToDevice, st));
    Q.tab = d_tab;
    // log-determinants: each problem's probes, zero past its count
    const int period = o->probe_kind == KRY_PROBE_COLOURED ? o->colour_period : 0;
    std::function<void(R*)> fill = [&](R* Z) {
        KRY_HIP(hipMemsetAsync(Z, 0, (size_t)G * np * pm * sizeof(R), st));
        for (int g = 0; g < G; ++g) make_probes<R>(*probs[g], np, o->seed, period, Z + (size_t)g * np * pm, st, pm);
    };
    LoglikWork W;
    slq_device<R>(Q, o, nullptr, 0, d_eta, G, W, nullptr, nullptr, st, nullptr, &fill);
    // quadratic forms
    KRY_HIP(hipMemsetAsync(Yd, 0, (size_t)G * pm * sizeof(double), st));
    for (int g = 0; g < G; ++g)
        KRY_HIP(hipMemcpyAsync(Yd + (size_t)g * pm, probs[g]->y64.ptr, probs[g]->p * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
    SolveStats ss;
    solve_device(Q, o->precision, nullptr, nullptr, 0, 1, d_eta, G, Yd, Xd, o->cg_rtol, o->cg_maxit, ss, st);
    std::vector<double> Qf(G);
    dot_batched<double>(Yd, pm, Xd, pm, pm, G, part, part + (size_t)G * 256, st);
    KRY_HIP(hipMemcpyAsync(Qf.data(), part + (size_t)G * 256, G * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
    for (int g = 0; g < G; ++g) {
        double est, se;
        combine(W.gamma.data() + (size_t)g * np, np, o->probe_kind == KRY_PROBE_COLOURED, &est, &se);
        kry_loglik_result& r = out[g];
        std::memset(&r, 0, sizeof(r));
        assemble(&r, probs[g]->p, est, se, Qf[g], th[g].sigma2);
        r.lanczos_steps_used = steps_used(W, g, np, g * np);
        r.cg_iters = ss.iters[g];
        r.cg_relres = ss.relres[g];
    }
}

bool any_not_converged(const kry_loglik_result* r, int count, const kry_opts* o) {
    if (o->solver != KRY_SOLVER_CG) return false;
    for (int t = 0; t < count; ++t)
        if (r[t].cg_relres > o->cg_rtol) return true;
    return false;
}

}  // namespace

namespace kry {
Matern to_matern_abi(const kry_matern* t) { return to_matern(t); }

void gengk_run(Problem& P, const Matern& th, const kry_opts* o, GkRun& G, const double* data64, hipStream_t st) {
    GkOut g;
    if (o->precision == KRY_FP32) gengk_device<float>(P, th, o, g, nullptr, st, data64);
    else gengk_device<double>(P, th, o, g, nullptr, st, data64);
    G.alpha = g.alpha;
    G.beta = g.beta;
    G.z = g.z;
    G.J = g.J;
    G.beta1 = g.beta1;
    G.V = g.V;
    G.Sv = g.Sv;
    G.real_bytes = o->precision == KRY_FP32 ? 4 : 8;
}

std::vector<double> gls_beta(Problem& P, const kry_matern* theta, const kry_opts* o, double* d_w, bool* noconv,
                             hipStream_t st) {
    KRY_REQUIRE(P.q > 0, "the problem has no covariates");
    const Matern th = to_matern(theta);
    const double eta = th.tau2 / th.sigma2;
    Spectrum& S = problem_spectrum(P, th, st);
    const int64_t p = P.p;
    const int nd = 1 + P.q;
    P.tmp2.ensure(*P.ctx, ((size_t)2 * nd * p + (size_t)nd * 256 + (size_t)nd * nd + 64) * sizeof(double));
    double* Dset = P.tmp2.as<double>();
    double* Wset = Dset + (size_t)nd * p;
    double* part = Wset + (size_t)nd * p;
    double* dots = part + (size_t)nd * 256;
    double* d_eta = dots + (size_t)nd * nd;
    KRY_HIP(hipMemcpyAsync(d_eta, &eta, sizeof(double), hipMemcpyHostToDevice, st));
    copy_rhs_set(P, Dset, st);
    SolveStats ss;
    solve_device(P, o->precision, S.s64.ptr, S.s32.ptr, 0, nd, d_eta, nd, Dset, Wset, o->cg_rtol, o->cg_maxit, ss,
                 st);
    for (int v = 0; v < nd; ++v)
        if (ss.relres[v] > o->cg_rtol && noconv) *noconv = true;
    for (int b = 0; b < nd; ++b) dot_batched<double>(Dset + (size_t)b * p, 0, Wset, p, p, nd, part, dots + b * nd, st);
    std::vector<double> h((size_t)nd * nd), M((size_t)nd * nd);
    KRY_HIP(hipMemcpyAsync(h.data(), dots, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
    for (int a2 = 0; a2 < nd; ++a2)
        for (int b = 0; b < nd; ++b) M[(size_t)a2 * nd + b] = h[(size_t)b * nd + a2];
    const Gls g = gls_combine(P, M.data());
    if (d_w) {
        KRY_HIP(hipMemcpyAsync(d_w, Wset, p * sizeof(double), hipMemcpyDeviceToDevice, st));
        for (int j = 0; j < P.q; ++j) axpby<double>(Wset + (size_t)(j + 1) * p, d_w, -g.delta[j], 1.0, p, 1, st);
    }
    return g.beta;
}

void loglik_multi(Problem& work, const std::vector<Problem*>& probs, const kry_matern* th, const kry_opts* o,
                  kry_loglik_result* out, hipStream_t st) {
    if (o->precision == KRY_FP32) loglik_multi_group<float>(work, probs, th, o, out, st);
    else loglik_multi_group<double>(work, probs, th, o, out, st);
}

// log-likelihood for `count` parameter points that share nu and anisotropy
// handling (each with its own spectrum) on one problem.
void loglik_points(Problem& P, const kry_matern* thetas, int count, const kry_opts* o, kry_loglik_result* out,
                   hipStream_t st) {
    if (o->shift_share) {
        loglik_points_shared(P, thetas, count, o, out, st);
        return;
    }
    Ctx& C = *P.ctx;
    const int np = nprobes_of(o);
    const int64_t nspec = (int64_t)(P.N2 / 2 + 1) * P.N1;
    const bool fp32 = o->precision == KRY_FP32;
    // spectra for every point
    P.spec_multi64.ensure(C, (size_t)count * nspec * sizeof(double));
    if (fp32) P.spec_multi32.ensure(C, (size_t)count * nspec * sizeof(float));
    std::vector<double> eta(count);
    for (int t = 0; t < count; ++t) {
        const Matern th = to_matern(&thetas[t]);
        eta[t] = th.tau2 / th.sigma2;
        double lo, hi;
        double* dst = P.spec_multi64.as<double>() + (size_t)t * nspec;
        spectrum_device(P, P.N1, P.N2, th, dst, &lo, &hi, st);
        spectrum_scale(dst, nspec, 1.0 / ((double)P.N1 * P.N2), false, dst,
                       fp32 ? P.spec_multi32.as<float>() + (size_t)t * nspec : nullptr, st);
    }
    // eta and the right-hand sides of every point: the data and, with
    // covariates, every covariate column (nd per point, point-major)
    const int nd = 1 + P.q;
    const bool need_cg = o->solver == KRY_SOLVER_CG || P.q > 0;
    const int64_t nv = (int64_t)count * nd;
    DevBuf& etab = P.tmp1;
    etab.ensure(C, count * sizeof(double) + (size_t)nv * P.p * 2 * sizeof(double) + 512);
    double* d_eta = etab.as<double>();
    double* Y = reinterpret_cast<double*>(etab.as<char>() + 256);
    double* X = Y + (size_t)nv * P.p;
    KRY_HIP(hipMemcpyAsync(d_eta, eta.data(), count * sizeof(double), hipMemcpyHostToDevice, st));
    // log-determinants
    LoglikWork W;
    if (fp32) slq_device<float>(P, o, P.spec_multi32.ptr, nspec, d_eta, count, W, nullptr, nullptr, st);
    else slq_device<double>(P, o, P.spec_multi64.ptr, nspec, d_eta, count, W, nullptr, nullptr, st);
    // quadratic forms
    std::vector<double> Q(count, 0.0);
    std::vector<int> iters(count, 0);
    std::vector<double> relres(count, 0.0);
    std::vector<Gls> gls(P.q > 0 ? count : 0);
    if (need_cg) {
        for (int t = 0; t < count; ++t) copy_rhs_set(P, Y + (size_t)t * nd * P.p, st);
        SolveStats ss;
        solve_device(P, o->precision, P.spec_multi64.ptr, fp32 ? P.spec_multi32.ptr : nullptr, nspec, nd, d_eta,
                     (int)nv, Y, X, o->cg_rtol, o->cg_maxit, ss, st);
        // M_t[a][b] = D_b . x_{t,a}, x_{t,a} = K_t^{-1} D_a
        P.lagtmp.ensure(C, (size_t)(nv * 256 + nv * nd + 8) * sizeof(double));
        double* part = P.lagtmp.as<double>();
        double* dots = part + nv * 256;
        for (int b = 0; b < nd; ++b) dot_batched<double>(Y + (size_t)b * P.p, 0, X, P.p, P.p, (int)nv, part,
                                                         dots + (size_t)b * nv, st);
        std::vector<double> h((size_t)nv * nd);
        KRY_HIP(hipMemcpyAsync(h.data(), dots, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        std::vector<double> Mt((size_t)nd * nd);
        for (int t = 0; t < count; ++t) {
            for (int a = 0; a < nd; ++a) {
                const int64_t v = (int64_t)t * nd + a;
                iters[t] = std::max(iters[t], ss.iters[v]);
                relres[t] = std::max(relres[t], ss.relres[v]);
                for (int b = 0; b < nd; ++b) Mt[(size_t)a * nd + b] = h[(size_t)b * nv + v];
            }
            if (P.q > 0) gls[t] = gls_combine(P, Mt.data());
            Q[t] = P.q > 0 ? gls[t].Q : Mt[0];
        }
    }
    if (o->solver != KRY_SOLVER_CG) {
        double* resid = nullptr;
        if (P.q > 0) {
            P.tmp4.ensure(C, (size_t)P.p * sizeof(double) + 256);
            resid = P.tmp4.as<double>();
        }
        for (int t = 0; t < count; ++t) {
            GkOut G;
            const Matern th = to_matern(&thetas[t]);
            if (P.q > 0) {  // genGK on the GLS residual yc - X delta
                KRY_HIP(hipMemcpyAsync(resid, P.yc64.ptr, P.p * sizeof(double), hipMemcpyDeviceToDevice, st));
                for (int j = 0; j < P.q; ++j)
                    axpby<double>(P.X64.as<double>() + (size_t)j * P.p, resid, -gls[t].delta[j], 1.0, P.p, 1, st);
            }
            if (fp32) gengk_device<float>(P, th, o, G, nullptr, st, resid);
            else gengk_device<double>(P, th, o, G, nullptr, st, resid);
            Q[t] = G.J;  // unit-variance form: sigma^2 = 1 so Q = J
            if (P.q > 0) gls[t].Q = G.J;
            iters[t] = o->gk_steps;
            relres[t] = 0.0;
        }
    }
    for (int t = 0; t < count; ++t) {
        double est, se;
        combine(W.gamma.data() + (size_t)t * np, np, o->probe_kind == KRY_PROBE_COLOURED, &est, &se);
        kry_loglik_result& r = out[t];
        std::memset(&r, 0, sizeof(r));
        if (P.q > 0) assemble_gls(&r, P, est, se, gls[t], thetas[t].sigma2, o->reml != 0);
        else assemble(&r, P.p, est, se, Q[t], thetas[t].sigma2);
        r.lanczos_steps_used = steps_used(W, t, np, t * np);
        r.cg_iters = iters[t];
        r.cg_relres = relres[t];
    }
}
}  // namespace kry

// ===========================================================================
// ABI (C linkage comes from the declarations in kryging.h)
// ===========================================================================

const char* kry_status_string(kry_status s) {
    switch (s) {
        case KRY_OK: return "ok";
        case KRY_EINVAL: return "invalid argument";
        case KRY_ENOMEM: return "out of device memory or above the HBM budget";
        case KRY_EDEVICE: return "HIP runtime error";
        case KRY_ENOTPSD: return "circulant embedding not positive semi-definite";
        case KRY_ENOCONV: return "iteration limit reached";
        case KRY_EBUSY: return "server queue full";
        case KRY_ENOTIMPL: return "not implemented";
    }
    return "unknown status";
}

const char* kry_last_error(void) { return g_last_error.c_str(); }

kry_status kry_opts_default(kry_opts* out) {
    return guard([&] {
        KRY_REQUIRE(out != nullptr, "out is NULL");
        kry_opts o;
        std::memset(&o, 0, sizeof(o));
        o.lanczos_steps = 30;
        o.num_probes = 10;
        o.probe_kind = KRY_PROBE_RADEMACHER;
        o.colour_period = 4;
        o.seed = 303;
        o.reorth = 0;
        o.precision = KRY_FP64;
        o.cg_rtol = 1e-8;
        o.cg_maxit = 20000;
        o.solver = KRY_SOLVER_CG;
        o.gk_steps = 100;
        o.shift_share = 0;
        o.lanczos_max_steps = 500;
        o.lanczos_rtol = 0.0;
        o.reml = 0;
        *out = o;
    });
}

kry_status kry_ctx_create(int32_t device, uint64_t hbm_budget_bytes, kry_ctx** out) {
    return guard([&] {
        KRY_REQUIRE(out != nullptr, "out is NULL");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
            (void)hipGetLastError();
            throw Error(KRY_EDEVICE, "no HIP device available");
        }
        KRY_REQUIRE(device >= 0 && device < ndev, "device index out of range");
        auto* k = new kry_ctx();
        try {
            k->c.device = device;
            k->c.budget = hbm_budget_bytes;
            KRY_HIP(hipSetDevice(device));
            KRY_HIP(hipStreamCreateWithFlags(&k->c.stream, hipStreamNonBlocking));
            // twiddles exp(-2 pi i e / TW_N), computed in long double
            std::vector<cpx<double>> t64(TW_N);
            std::vector<cpx<float>> t32(TW_N);
            const long double pi = 3.141592653589793238462643383279502884L;
            for (int e = 0; e < TW_N; ++e) {
                const long double a = -2.0L * pi * (long double)e / (long double)TW_N;
                t64[e] = {(double)cosl(a), (double)sinl(a)};
                t32[e] = {(float)cosl(a), (float)sinl(a)};
            }
            k->c.tw64 = static_cast<cpx<double>*>(dev_alloc(k->c, TW_N * sizeof(cpx<double>)));
            k->c.tw32 = static_cast<cpx<float>*>(dev_alloc(k->c, TW_N * sizeof(cpx<float>)));
            KRY_HIP(hipMemcpy(k->c.tw64, t64.data(), TW_N * sizeof(cpx<double>), hipMemcpyHostToDevice));
            KRY_HIP(hipMemcpy(k->c.tw32, t32.data(), TW_N * sizeof(cpx<float>), hipMemcpyHostToDevice));
            // every transform length's pass twiddles now, so that products
            // allocate nothing later; and the no-allocation product's scratch
            build_plan_tables(k->c);
            k->c.scratch = noalloc_scratch_init(device);
        } catch (...) {
            kry_ctx_destroy(k);
            throw;
        }
        *out = k;
    });
}

kry_status kry_ctx_set_embedding(kry_ctx* ctx, int32_t rule) {
    return run_guarded([&] {
        KRY_REQUIRE(ctx, "NULL context");
        KRY_REQUIRE(rule == KRY_EMBED_FAST || rule == KRY_EMBED_SMALLEST, "unknown embedding rule");
        ctx->c.embed_rule = rule;
    });
}

kry_status kry_ctx_memory(kry_ctx* ctx, uint64_t* allocated, uint64_t* peak, int32_t reset_peak) {
    return guard([&] {
        KRY_REQUIRE(ctx && allocated && peak, "NULL argument");
        std::lock_guard<std::mutex> g(ctx->c.alloc_mu);
        *allocated = ctx->c.allocated;
        *peak = ctx->c.peak;
        if (reset_peak) ctx->c.peak = ctx->c.allocated;
    });
}

kry_status kry_profile_begin(kry_ctx* ctx) {
    return guard([&] {
        KRY_REQUIRE(ctx != nullptr, "ctx is NULL");
        bind(ctx->c);
        ctx->c.prof.on = true;
        ctx->c.prof.recs.clear();
        ctx->c.prof.next = 0;
    });
}

kry_status kry_profile_end(kry_ctx* ctx, double* ms, int64_t* launches, int64_t* vectors) {
    return guard([&] {
        KRY_REQUIRE(ctx && ms && launches && vectors, "NULL argument");
        bind(ctx->c);
        StageProfile& pr = ctx->c.prof;
        KRY_HIP(hipDeviceSynchronize());
        for (int i = 0; i < 3; ++i) {
            ms[i] = 0.0;
            launches[i] = 0;
        }
        *vectors = 0;
        for (const auto& r : pr.recs) {
            for (int i = 0; i < 3; ++i) {
                float t = 0.f;
                KRY_HIP(hipEventElapsedTime(&t, pr.pool[r[i]], pr.pool[r[i + 1]]));
                ms[i] += t;
                launches[i] += 1;
            }
            *vectors += r[4];
        }
        pr.on = false;
        pr.recs.clear();
        pr.next = 0;
    });
}

void kry_ctx_destroy(kry_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->c.device);
    if (ctx->c.stream) (void)hipStreamSynchronize(ctx->c.stream);
    for (hipEvent_t e : ctx->c.prof.pool) (void)hipEventDestroy(e);
    for (int i = 0; i < 14; ++i) {
        if (ctx->c.plan64[i]) (void)hipFree(ctx->c.plan64[i]);
        if (ctx->c.plan32[i]) (void)hipFree(ctx->c.plan32[i]);
    }
    for (auto& kv : ctx->c.mplan64) (void)hipFree(kv.second);
    for (auto& kv : ctx->c.mplan32) (void)hipFree(kv.second);
    dev_free(ctx->c, ctx->c.tw64, TW_N * sizeof(cpx<double>));
    dev_free(ctx->c, ctx->c.tw32, TW_N * sizeof(cpx<float>));
    if (ctx->c.stream) (void)hipStreamDestroy(ctx->c.stream);
    delete ctx;
}

// OLS centring for the GLS forms (host, FP64): from the covariates at the
// observed cells, X^T X and its Cholesky factor, beta_ols = (X^T X)^{-1} X^T y
// and yc = y - X beta_ols.  Removing any X b from the data leaves the GLS
// residual unchanged; removing the OLS fit keeps Q = c - g^T G^{-1} g free of
// the mean's magnitude.  Computes into the outputs only; throws on
// dependent columns.
static void ols_centre(const Problem& P, int q, const std::vector<double>& Xfull, const std::vector<double>& y,
                       std::vector<double>& Xc, std::vector<double>& yc, std::vector<double>& beta,
                       double& logdet_xx) {
    const int64_t p = P.p, n = (int64_t)P.n1 * P.n2;
    Xc.assign((size_t)q * p, 0.0);
    for (int j = 0; j < q; ++j)
        for (int64_t i = 0; i < p; ++i)  // irregular problems take the covariates per observation
            Xc[(size_t)j * p + i] = P.irregular ? Xfull[(size_t)j * p + (*P.h_obs_user)[i]]
                                                : Xfull[(size_t)j * n + (*P.h_cell)[i]];
    std::vector<double> A((size_t)q * q, 0.0), b(q, 0.0);
    for (int i = 0; i < q; ++i) {
        const double* xi = Xc.data() + (size_t)i * p;
        for (int j = 0; j <= i; ++j) {
            const double* xj = Xc.data() + (size_t)j * p;
            double acc = 0;
            for (int64_t k = 0; k < p; ++k) acc += xi[k] * xj[k];
            A[i * q + j] = A[j * q + i] = acc;
        }
        double acc = 0;
        for (int64_t k = 0; k < p; ++k) acc += xi[k] * y[k];
        b[i] = acc;
    }
    KRY_REQUIRE(chol_small(A, q, 1e-10), "covariate columns are linearly dependent on the observed cells");
    logdet_xx = chol_logdet(A, q);
    beta = chol_solve(A, q, b);
    yc = y;
    for (int j = 0; j < q; ++j)
        for (int64_t k = 0; k < p; ++k) yc[k] -= Xc[(size_t)j * p + k] * beta[j];
}

static void upload_centred(Problem& P, const std::vector<double>& Xc, const std::vector<double>& yc) {
    P.X64.ensure(*P.ctx, Xc.size() * sizeof(double));
    P.yc64.ensure(*P.ctx, yc.size() * sizeof(double));
    KRY_HIP(hipMemcpy(P.X64.ptr, Xc.data(), Xc.size() * sizeof(double), hipMemcpyHostToDevice));
    KRY_HIP(hipMemcpy(P.yc64.ptr, yc.data(), yc.size() * sizeof(double), hipMemcpyHostToDevice));
}

static void upload_compact(Problem& P, const std::vector<double>& yc);

static void upload_data(Problem& P, const double* y) {
    std::vector<double> yc(P.p, 0.0);
    if (y) {
        for (int64_t i = 0; i < P.p; ++i) {
            const double v = P.irregular ? y[(*P.h_obs_user)[i]] : y[(*P.h_cell)[i]];
            KRY_REQUIRE(std::isfinite(v), "y has a non-finite value at an observed cell");
            yc[i] = v;
        }
    }
    upload_compact(P, yc);
}

// Compact data (p values) to the device, with the OLS centring when the
// problem has covariates.
static void upload_compact(Problem& P, const std::vector<double>& yc) {
    std::vector<double> Xc, ycent, beta;
    double ldxx = 0;
    if (P.q > 0) ols_centre(P, P.q, *P.h_X, yc, Xc, ycent, beta, ldxx);
    std::vector<float> yf(yc.begin(), yc.end());
    KRY_HIP(hipMemcpy(P.y64.ptr, yc.data(), P.p * sizeof(double), hipMemcpyHostToDevice));
    KRY_HIP(hipMemcpy(P.y32.ptr, yf.data(), P.p * sizeof(float), hipMemcpyHostToDevice));
    if (P.q > 0) {
        upload_centred(P, Xc, ycent);
        P.beta_ols = beta;
        P.logdet_xx = ldxx;
    }
}

kry_status kry_problem_create(kry_ctx* ctx, const kry_grid* grid, const uint8_t* mask, const double* y,
                              kry_problem** out) {
    return guard([&] {
        KRY_REQUIRE(ctx && grid && mask && out, "NULL argument");
        KRY_REQUIRE(grid->n1 >= 2 && grid->n2 >= 2 && grid->n1 <= 4096 && grid->n2 <= 4096,
                    "grid sides must be in [2, 4096]");
        KRY_REQUIRE(std::isfinite(grid->dx1) && std::isfinite(grid->dx2) && grid->dx1 > 0 && grid->dx2 > 0,
                    "grid spacings must be finite and > 0");
        const int n1 = grid->n1, n2 = grid->n2;
        const int64_t n = (int64_t)n1 * n2;
        int64_t p = 0;
        for (int64_t i = 0; i < n; ++i) p += mask[i] ? 1 : 0;
        KRY_REQUIRE(p > 0, "mask has no observed cell");
        if (y)
            for (int64_t i = 0; i < n; ++i)
                if (mask[i]) KRY_REQUIRE(std::isfinite(y[i]), "y has a non-finite value at an observed cell");
        bind(ctx->c);
        auto* kp = new kry_problem();
        Problem& P = kp->P;
        try {
            P.ctx = &ctx->c;
            P.n1 = n1;
            P.n2 = n2;
            P.dx1 = grid->dx1;
            P.dx2 = grid->dx2;
            P.N1 = embedding_side(2 * n1 - 1, P.ctx->embed_rule);
            P.N2 = embedding_side(2 * n2 - 1, P.ctx->embed_rule);
            build_embedding_tables(*P.ctx, P.N1, P.N2);
            P.p = p;
            P.words_per_row = (n2 + 31) / 32;
            const int64_t nw = (int64_t)n1 * P.words_per_row;
            std::vector<uint32_t> bits(nw, 0u), base(nw, 0u);
            auto hc = std::make_shared<std::vector<int64_t>>(p);
            auto hm = std::make_shared<std::vector<uint8_t>>(n);
            std::vector<int32_t> cell(p);
            int64_t c = 0;
            for (int i = 0; i < n1; ++i)
                for (int j = 0; j < n2; ++j) {
                    const int64_t id = (int64_t)i * n2 + j;
                    (*hm)[id] = mask[id] ? 1 : 0;
                    if (mask[id]) {
                        bits[(int64_t)i * P.words_per_row + (j >> 5)] |= 1u << (j & 31);
                        (*hc)[c] = id;
                        cell[c] = (int32_t)id;
                        ++c;
                    }
                }
            P.h_cell = hc;
            P.h_mask = hm;
            uint32_t acc = 0;
            for (int64_t w = 0; w < nw; ++w) {
                base[w] = acc;
                acc += (uint32_t)__builtin_popcount(bits[w]);
            }
            P.bits.ensure(ctx->c, nw * sizeof(uint32_t));
            P.base.ensure(ctx->c, nw * sizeof(uint32_t));
            P.cell.ensure(ctx->c, p * sizeof(int32_t));
            P.y64.ensure(ctx->c, p * sizeof(double));
            P.y32.ensure(ctx->c, p * sizeof(float));
            KRY_HIP(hipMemcpy(P.bits.ptr, bits.data(), nw * sizeof(uint32_t), hipMemcpyHostToDevice));
            KRY_HIP(hipMemcpy(P.base.ptr, base.data(), nw * sizeof(uint32_t), hipMemcpyHostToDevice));
            KRY_HIP(hipMemcpy(P.cell.ptr, cell.data(), p * sizeof(int32_t), hipMemcpyHostToDevice));
            upload_data(P, y);
        } catch (...) {
            kry_problem_destroy(kp);
            throw;
        }
        *out = kp;
    });
}

kry_status kry_problem_set_data(kry_problem* prob, const double* y) {
    return guard([&] {
        KRY_REQUIRE(prob && y, "NULL argument");
        Problem& P = prob->P;
        for (int64_t i = 0; i < P.p; ++i)
            KRY_REQUIRE(std::isfinite(P.irregular ? y[i] : y[(*P.h_cell)[i]]),
                        "y has a non-finite value at an observed cell");
        bind(*P.ctx);
        upload_data(P, y);
    });
}

kry_status kry_problem_create_irregular(kry_ctx* ctx, const kry_grid* grid, int64_t p, const double* locs,
                                        const double* y, kry_problem** out) {
    return guard([&] {
        KRY_REQUIRE(ctx && grid && locs && out, "NULL argument");
        KRY_REQUIRE(grid->n1 >= 2 && grid->n2 >= 2 && grid->n1 <= 4096 && grid->n2 <= 4096,
                    "grid sides must be in [2, 4096]");
        KRY_REQUIRE(std::isfinite(grid->dx1) && std::isfinite(grid->dx2) && grid->dx1 > 0 && grid->dx2 > 0,
                    "grid spacings must be finite and > 0");
        KRY_REQUIRE(p >= 1 && p <= ((int64_t)1 << 30), "p must be in [1, 2^30]");
        const int n1 = grid->n1, n2 = grid->n2;
        const int64_t n = (int64_t)n1 * n2;
        for (int64_t i = 0; i < p; ++i) {
            const double u1 = locs[2 * i], u2 = locs[2 * i + 1];
            KRY_REQUIRE(std::isfinite(u1) && std::isfinite(u2) && u1 >= 0 && u2 >= 0 && u1 <= n1 - 1 && u2 <= n2 - 1,
                        "observation locations must lie in [0, n1 - 1] x [0, n2 - 1] (grid units)");
            if (y) KRY_REQUIRE(std::isfinite(y[i]), "y has a non-finite value");
        }
        // stored order: by nearest grid cell, ties in the caller's order
        auto nearest = [&](int64_t i) {
            const int ra = std::min((int)std::lround(locs[2 * i]), n1 - 1);
            const int rb = std::min((int)std::lround(locs[2 * i + 1]), n2 - 1);
            return (int64_t)ra * n2 + rb;
        };
        auto order = std::make_shared<std::vector<int32_t>>(p);
        {
            std::vector<int64_t> key(p);
            for (int64_t i = 0; i < p; ++i) key[i] = nearest(i);
            std::iota(order->begin(), order->end(), 0);
            std::stable_sort(order->begin(), order->end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
        }
        // A: the Wendland weights of the corners of each observation's cell
        // (Sec. 2), normalised; A^T by rows over the cells
        std::vector<int32_t> cell4((size_t)4 * p, -1), near(p);
        std::vector<double> w4((size_t)4 * p, 0.0);
        std::vector<int32_t> cnt(n + 1, 0);
        auto hc = std::make_shared<std::vector<int64_t>>(p);
        for (int64_t i = 0; i < p; ++i) {
            const int64_t u = (*order)[i];
            const double u1 = locs[2 * u], u2 = locs[2 * u + 1];
            const int a0 = std::min((int)std::floor(u1), n1 - 1), b0 = std::min((int)std::floor(u2), n2 - 1);
            double sum = 0;
            int s = 0;
            for (int da = 0; da < 2; ++da)
                for (int db = 0; db < 2; ++db) {
                    const int a = a0 + da, b = b0 + db;
                    if (a >= n1 || b >= n2) continue;
                    const double d = std::max(std::fabs(u1 - a), std::fabs(u2 - b));
                    if (!(d < 1.0)) continue;
                    const double t = 1.0 - d;
                    const double wv = t * t * t * t * (1.0 + 4.0 * d);
                    cell4[4 * i + s] = a * n2 + b;
                    w4[4 * i + s] = wv;
                    sum += wv;
                    ++s;
                }
            KRY_REQUIRE(s > 0 && sum > 0, "an observation has no grid neighbour");
            for (int k = 0; k < s; ++k) {
                w4[4 * i + k] /= sum;
                ++cnt[cell4[4 * i + k] + 1];
            }
            near[i] = (int32_t)nearest(u);
            (*hc)[i] = near[i];
        }
        for (int64_t c = 0; c < n; ++c) cnt[c + 1] += cnt[c];
        const int64_t nnz = cnt[n];
        std::vector<int32_t> at_obs(std::max<int64_t>(nnz, 1)), fill(cnt.begin(), cnt.end() - 1);
        std::vector<double> at_w(std::max<int64_t>(nnz, 1));
        for (int64_t i = 0; i < p; ++i)  // increasing observation id within every cell
            for (int k = 0; k < 4; ++k) {
                const int c = cell4[4 * i + k];
                if (c < 0) continue;
                at_obs[fill[c]] = (int32_t)i;
                at_w[fill[c]] = w4[4 * i + k];
                ++fill[c];
            }
        bind(ctx->c);
        auto* kp = new kry_problem();
        Problem& P = kp->P;
        try {
            P.ctx = &ctx->c;
            P.n1 = n1;
            P.n2 = n2;
            P.dx1 = grid->dx1;
            P.dx2 = grid->dx2;
            P.N1 = embedding_side(2 * n1 - 1, P.ctx->embed_rule);
            P.N2 = embedding_side(2 * n2 - 1, P.ctx->embed_rule);
            build_embedding_tables(*P.ctx, P.N1, P.N2);
            P.p = p;
            P.irregular = true;
            P.h_cell = hc;
            P.h_obs_user = order;
            for (int64_t i = 0; i < p && !P.obs_permuted; ++i) P.obs_permuted = (*order)[i] != i;
            P.h_mask = std::make_shared<std::vector<uint8_t>>(n, 0);
            auto up = [&](DevBuf& b, const void* src, size_t bytes) {
                b.ensure(ctx->c, bytes);
                KRY_HIP(hipMemcpy(b.ptr, src, bytes, hipMemcpyHostToDevice));
            };
            up(P.cell, near.data(), p * sizeof(int32_t));
            up(P.obs_user, order->data(), p * sizeof(int32_t));
            up(P.a_cell, cell4.data(), cell4.size() * sizeof(int32_t));
            up(P.a_w, w4.data(), w4.size() * sizeof(double));
            up(P.at_off, cnt.data(), cnt.size() * sizeof(int32_t));
            up(P.at_obs, at_obs.data(), at_obs.size() * sizeof(int32_t));
            up(P.at_w, at_w.data(), at_w.size() * sizeof(double));
            P.y64.ensure(ctx->c, p * sizeof(double));
            P.y32.ensure(ctx->c, p * sizeof(float));
            upload_data(P, y);
        } catch (...) {
            kry_problem_destroy(kp);
            throw;
        }
        *out = kp;
    });
}

kry_status kry_problem_set_covariates(kry_problem* prob, int32_t q, const double* X) {
    return guard([&] {
        KRY_REQUIRE(prob != nullptr, "prob is NULL");
        Problem& P = prob->P;
        KRY_REQUIRE(q >= 0 && q <= KRY_MAX_COVARIATES, "q must be in [0, KRY_MAX_COVARIATES]");
        KRY_REQUIRE(q < P.p, "q must be below the observed count");
        KRY_REQUIRE(q == 0 || X != nullptr, "X is NULL");
        const int64_t n = P.irregular ? P.p : (int64_t)P.n1 * P.n2;  // values per column
        for (int64_t i = 0; i < (int64_t)q * n; ++i) KRY_REQUIRE(std::isfinite(X[i]), "X has a non-finite value");
        bind(*P.ctx);
        if (q == 0) {
            KRY_HIP(hipStreamSynchronize(P.ctx->stream));
            P.X64.release(*P.ctx);
            P.yc64.release(*P.ctx);
            P.h_X.reset();
            P.beta_ols.clear();
            P.logdet_xx = 0;
            P.q = 0;
            return;
        }
        auto hx = std::make_shared<std::vector<double>>(X, X + (size_t)q * n);
        std::vector<double> y(P.p);
        KRY_HIP(hipStreamSynchronize(P.ctx->stream));
        KRY_HIP(hipMemcpy(y.data(), P.y64.ptr, P.p * sizeof(double), hipMemcpyDeviceToHost));
        std::vector<double> Xc, yc, beta;
        double ldxx = 0;
        ols_centre(P, q, *hx, y, Xc, yc, beta, ldxx);  // validates before any change
        upload_centred(P, Xc, yc);
        P.q = q;
        P.h_X = hx;
        P.beta_ols = beta;
        P.logdet_xx = ldxx;
    });
}

kry_status kry_problem_info(const kry_problem* prob, int64_t* p, int32_t* N1, int32_t* N2) {
    return guard([&] {
        KRY_REQUIRE(prob != nullptr, "prob is NULL");
        if (p) *p = prob->P.p;
        if (N1) *N1 = prob->P.N1;
        if (N2) *N2 = prob->P.N2;
    });
}

void kry_problem_destroy(kry_problem* prob) {
    if (!prob) return;
    Problem& P = prob->P;
    if (P.ctx) {
        Ctx& c = *P.ctx;
        (void)hipSetDevice(c.device);
        (void)hipStreamSynchronize(c.stream);
        for (DevBuf* b : {&P.bits, &P.base, &P.cell, &P.y64, &P.y32, &P.X64, &P.yc64, &P.a_cell, &P.a_w, &P.at_off,
                          &P.at_obs, &P.at_w, &P.obs_user})
            b->release(c);
        P.release_work();
    }
    delete prob;
}

static void torus_args(Problem& P, int32_t& N1, int32_t& N2) {
    if (N1 == 0 && N2 == 0) {
        N1 = P.N1;
        N2 = P.N2;
    }
    KRY_REQUIRE(torus_side_ok(N1) && torus_side_ok(N2),
                "torus sides must be in [16, 8192]: powers of two or multiples of 16 of the form 2^a 3^b 5^c 7^d");
}

kry_status kry_lag_grid(kry_problem* prob, const kry_matern* theta, int32_t N1, int32_t N2, double* c_out) {
    return guard([&] {
        KRY_REQUIRE(prob && c_out, "NULL argument");
        check_theta(theta);
        Problem& P = prob->P;
        torus_args(P, N1, N2);
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        P.lagtmp.ensure(*P.ctx, (size_t)N1 * N2 * sizeof(double));
        lag_grid_device(*P.ctx, N1, N2, P.dx1, P.dx2, to_matern(theta), P.lagtmp.as<double>(), st);
        KRY_HIP(hipMemcpyAsync(c_out, P.lagtmp.ptr, (size_t)N1 * N2 * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
    });
}

kry_status kry_spectrum(kry_problem* prob, const kry_matern* theta, int32_t N1, int32_t N2, double* lam_out,
                        double* minmax) {
    return guard([&] {
        KRY_REQUIRE(prob && lam_out, "NULL argument");
        check_theta(theta);
        Problem& P = prob->P;
        torus_args(P, N1, N2);
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        const size_t n = (size_t)(N2 / 2 + 1) * N1;
        DevBuf tmp;
        tmp.ensure(*P.ctx, n * sizeof(double));
        try {
            double lo, hi;
            spectrum_device(P, N1, N2, to_matern(theta), tmp.as<double>(), &lo, &hi, st);
            KRY_HIP(hipMemcpyAsync(lam_out, tmp.ptr, n * sizeof(double), hipMemcpyDeviceToHost, st));
            KRY_HIP(hipStreamSynchronize(st));
            if (minmax) {
                minmax[0] = lo;
                minmax[1] = hi;
            }
        } catch (...) {
            tmp.release(*P.ctx);
            throw;
        }
        tmp.release(*P.ctx);
    });
}

template <typename R>
static void matvec_dev_impl(Problem& P, const Matern& th, int nvec, const void* in, void* out, hipStream_t st) {
    Spectrum& S = problem_spectrum(P, th, st);
    const double eta = th.tau2 / th.sigma2;
    P.scal.ensure(*P.ctx, 256);
    KRY_HIP(hipMemcpyAsync(P.scal.ptr, &eta, sizeof(double), hipMemcpyHostToDevice, st));
    auto A = masked_op<R>(P, spec_ptr<R>(S), 0, nvec, P.scal.as<double>());
    if (P.obs_permuted) {  // the caller's order to the stored order and back
        const size_t vb = ((size_t)nvec * P.p * sizeof(R) + 255) & ~size_t(255);
        P.tmp2.ensure(*P.ctx, 2 * vb);
        R* a = P.tmp2.as<R>();
        R* b = reinterpret_cast<R*>(P.tmp2.as<char>() + vb);
        irr_permute<R>(P, static_cast<const R*>(in), a, nvec, true, st);
        A(a, b, nvec, st, nullptr);
        irr_permute<R>(P, b, static_cast<R*>(out), nvec, false, st);
        return;
    }
    A(static_cast<const R*>(in), static_cast<R*>(out), nvec, st, nullptr);
}

kry_status kry_matvec_device(kry_problem* prob, const kry_matern* theta, int32_t precision, int32_t nvec,
                             const void* d_v, void* d_out, void* hip_stream) {
    return guard([&] {
        KRY_REQUIRE(prob && d_v && d_out, "NULL argument");
        check_theta(theta);
        KRY_REQUIRE(nvec >= 1, "nvec must be >= 1");
        KRY_REQUIRE(precision == KRY_FP64 || precision == KRY_FP32, "bad precision");
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : P.ctx->stream;
        if (precision == KRY_FP64) matvec_dev_impl<double>(P, to_matern(theta), nvec, d_v, d_out, st);
        else matvec_dev_impl<float>(P, to_matern(theta), nvec, d_v, d_out, st);
    });
}

kry_status kry_matvec(kry_problem* prob, const kry_matern* theta, int32_t precision, int32_t nvec, const double* v,
                      double* out) {
    return guard([&] {
        KRY_REQUIRE(prob && v && out, "NULL argument");
        check_theta(theta);
        KRY_REQUIRE(nvec >= 1, "nvec must be >= 1");
        KRY_REQUIRE(precision == KRY_FP64 || precision == KRY_FP32, "bad precision");
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        const size_t n = (size_t)nvec * P.p;
        DevBuf io;
        io.ensure(*P.ctx, 2 * n * sizeof(double));
        struct Free {
            Ctx& c;
            DevBuf& b;
            ~Free() { b.release(c); }
        } fr{*P.ctx, io};
        double* d_in = io.as<double>();
        double* d_out = d_in + n;
        KRY_HIP(hipMemcpyAsync(d_in, v, n * sizeof(double), hipMemcpyHostToDevice, st));
        if (precision == KRY_FP64) {
            matvec_dev_impl<double>(P, to_matern(theta), nvec, d_in, d_out, st);
        } else {
            float* f_in = reinterpret_cast<float*>(d_out);  // staging: out region holds the float input first
            float* f_out = reinterpret_cast<float*>(d_in);
            convert<double, float>(d_in, f_in, n, st);
            // f_out overlaps d_in, which is no longer needed once converted
            matvec_dev_impl<float>(P, to_matern(theta), nvec, f_in, f_out, st);
            convert<float, double>(f_out, d_out, n, st);
        }
        KRY_HIP(hipMemcpyAsync(out, d_out, n * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
    });
}

kry_status kry_cov_apply_full(kry_problem* prob, const kry_matern* theta, int32_t precision, int32_t nvec,
                              const double* w, double* out) {
    return guard([&] {
        KRY_REQUIRE(prob && w && out, "NULL argument");
        check_theta(theta);
        KRY_REQUIRE(nvec >= 1, "nvec must be >= 1");
        KRY_REQUIRE(precision == KRY_FP64 || precision == KRY_FP32, "bad precision");
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        const int64_t n = (int64_t)P.n1 * P.n2;
        const size_t nin = (size_t)nvec * P.p, nout = (size_t)nvec * n;
        DevBuf io;
        io.ensure(*P.ctx, (nin + 2 * nout) * sizeof(double) + 512);
        struct Free {
            Ctx& c;
            DevBuf& b;
            ~Free() { b.release(c); }
        } fr{*P.ctx, io};
        double* d_in = io.as<double>();
        double* d_out = d_in + nin;
        Spectrum& S = problem_spectrum(P, to_matern(theta), st);
        if (P.obs_permuted) {  // the caller's order to the stored order
            std::vector<double> ws(nin);
            for (int v = 0; v < nvec; ++v)
                for (int64_t i = 0; i < P.p; ++i)
                    ws[(size_t)v * P.p + i] = w[(size_t)v * P.p + (*P.h_obs_user)[i]];
            KRY_HIP(hipMemcpyAsync(d_in, ws.data(), nin * sizeof(double), hipMemcpyHostToDevice, st));
            KRY_HIP(hipStreamSynchronize(st));
        } else {
            KRY_HIP(hipMemcpyAsync(d_in, w, nin * sizeof(double), hipMemcpyHostToDevice, st));
        }
        if (precision == KRY_FP64) {
            cov_full<double>(P, S.s64.ptr, d_in, d_out, nvec, st);
        } else {
            float* f_in = reinterpret_cast<float*>(d_out + nout);
            float* f_out = reinterpret_cast<float*>(d_out);
            convert<double, float>(d_in, f_in, nin, st);
            float* tmp = reinterpret_cast<float*>(d_out + nout) + nin;
            cov_full<float>(P, S.s32.ptr, f_in, tmp, nvec, st);
            convert<float, double>(tmp, d_out, nout, st);
            (void)f_out;
        }
        KRY_HIP(hipMemcpyAsync(out, d_out, nout * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
    });
}

kry_status kry_probes(kry_problem* prob, const kry_opts* opts, int32_t* nprobe, double* out) {
    return guard([&] {
        KRY_REQUIRE(prob && nprobe, "NULL argument");
        check_opts(opts);
        Problem& P = prob->P;
        const int np = nprobes_of(opts);
        *nprobe = np;
        if (!out) return;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        DevBuf tmp;
        tmp.ensure(*P.ctx, (size_t)np * P.p * sizeof(double));
        struct Free {
            Ctx& c;
            DevBuf& b;
            ~Free() { b.release(c); }
        } fr{*P.ctx, tmp};
        make_probes<double>(P, np, opts->seed, opts->probe_kind == KRY_PROBE_COLOURED ? opts->colour_period : 0,
                            tmp.as<double>(), st);
        KRY_HIP(hipMemcpyAsync(out, tmp.ptr, (size_t)np * P.p * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        if (P.obs_permuted) {  // the stored order to the caller's order
            std::vector<double> h(out, out + (size_t)np * P.p);
            for (int k = 0; k < np; ++k)
                for (int64_t i = 0; i < P.p; ++i)
                    out[(size_t)k * P.p + (*P.h_obs_user)[i]] = h[(size_t)k * P.p + i];
        }
    });
}

static void single_point_spectrum(Problem& P, const Matern& th, const kry_opts* o, const void** lam, double** d_eta,
                                  hipStream_t st) {
    Spectrum& S = problem_spectrum(P, th, st);
    *lam = o->precision == KRY_FP32 ? S.s32.ptr : S.s64.ptr;
    const double eta = th.tau2 / th.sigma2;
    P.lagtmp.ensure(*P.ctx, 256);
    *d_eta = P.lagtmp.as<double>();
    KRY_HIP(hipMemcpyAsync(*d_eta, &eta, sizeof(double), hipMemcpyHostToDevice, st));
}

kry_status kry_lanczos(kry_problem* prob, const kry_matern* theta, const kry_opts* opts, double* alpha, double* beta,
                       int32_t* steps) {
    return guard([&] {
        KRY_REQUIRE(prob && alpha && beta && steps, "NULL argument");
        check_theta(theta);
        check_opts(opts);
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        const void* lam;
        double* d_eta;
        // keep eta outside lagtmp (the spectrum path reuses lagtmp): copy to scal
        single_point_spectrum(P, to_matern(theta), opts, &lam, &d_eta, st);
        P.scal.ensure(*P.ctx, 256);
        KRY_HIP(hipMemcpyAsync(P.scal.ptr, d_eta, sizeof(double), hipMemcpyDeviceToDevice, st));
        LoglikWork W;
        std::vector<double> a, b;
        const int np = nprobes_of(opts), m = opts->lanczos_steps;
        if (opts->precision == KRY_FP32)
            slq_device<float>(P, opts, lam, 0, P.scal.as<double>(), 1, W, &a, &b, st);
        else
            slq_device<double>(P, opts, lam, 0, P.scal.as<double>(), 1, W, &a, &b, st);
        for (int k = 0; k < np; ++k) {
            steps[k] = W.steps[k];
            for (int j = 0; j < m; ++j) {
                alpha[(size_t)k * m + j] = a[(size_t)j * np + k];
                beta[(size_t)k * m + j] = b[(size_t)j * np + k];
            }
        }
    });
}

kry_status kry_logdet(kry_problem* prob, const kry_matern* theta, const kry_opts* opts, double* logdet, double* se,
                      double* per_probe) {
    return guard([&] {
        KRY_REQUIRE(prob && logdet, "NULL argument");
        check_theta(theta);
        check_opts(opts);
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        const void* lam;
        double* d_eta;
        single_point_spectrum(P, to_matern(theta), opts, &lam, &d_eta, st);
        P.scal.ensure(*P.ctx, 256);
        KRY_HIP(hipMemcpyAsync(P.scal.ptr, d_eta, sizeof(double), hipMemcpyDeviceToDevice, st));
        LoglikWork W;
        if (opts->precision == KRY_FP32)
            slq_device<float>(P, opts, lam, 0, P.scal.as<double>(), 1, W, nullptr, nullptr, st);
        else
            slq_device<double>(P, opts, lam, 0, P.scal.as<double>(), 1, W, nullptr, nullptr, st);
        const int np = nprobes_of(opts);
        double est, s;
        combine(W.gamma.data(), np, opts->probe_kind == KRY_PROBE_COLOURED, &est, &s);
        *logdet = est;
        if (se) *se = s;
        if (per_probe) std::copy(W.gamma.begin(), W.gamma.end(), per_probe);
    });
}

kry_status kry_gauss_quadrature(int32_t nprobe, int32_t m, const double* alpha, const double* beta,
                                const int32_t* steps, const double* znorm2, double* gamma) {
    return guard([&] {
        KRY_REQUIRE(alpha && beta && steps && znorm2 && gamma, "NULL argument");
        KRY_REQUIRE(nprobe >= 1 && m >= 1 && m <= KRY_MAX_LANCZOS, "bad sizes");
        for (int k = 0; k < nprobe; ++k) KRY_REQUIRE(steps[k] >= 0 && steps[k] <= m, "steps out of range");
        int dev = 0;
        KRY_HIP(hipGetDevice(&dev));
        // device copies in step-major layout
        std::vector<double> a((size_t)m * nprobe), b((size_t)m * nprobe);
        for (int k = 0; k < nprobe; ++k)
            for (int j = 0; j < m; ++j) {
                a[(size_t)j * nprobe + k] = alpha[(size_t)k * m + j];
                b[(size_t)j * nprobe + k] = beta[(size_t)k * m + j];
            }
        void* d = nullptr;
        const size_t bytes = (2 * (size_t)m * nprobe + 2 * nprobe) * sizeof(double) + nprobe * sizeof(int);
        KRY_HIP(hipMalloc(&d, bytes));
        struct F {
            void* p;
            ~F() { (void)hipFree(p); }
        } f{d};
        double* da = static_cast<double*>(d);
        double* db = da + (size_t)m * nprobe;
        double* dz = db + (size_t)m * nprobe;
        double* dg = dz + nprobe;
        int* ds = reinterpret_cast<int*>(dg + nprobe);
        KRY_HIP(hipMemcpy(da, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice));
        KRY_HIP(hipMemcpy(db, b.data(), b.size() * sizeof(double), hipMemcpyHostToDevice));
        KRY_HIP(hipMemcpy(dz, znorm2, nprobe * sizeof(double), hipMemcpyHostToDevice));
        KRY_HIP(hipMemcpy(ds, steps, nprobe * sizeof(int), hipMemcpyHostToDevice));
        quadrature(da, db, ds, dz, nprobe, nprobe, dg, nullptr);
        KRY_HIP(hipMemcpy(gamma, dg, nprobe * sizeof(double), hipMemcpyDeviceToHost));
    });
}

kry_status kry_solve(kry_problem* prob, const kry_matern* theta, const kry_opts* opts, int32_t nrhs, const double* b,
                     double* x, int32_t* iters, double* relres) {
    bool noconv = false;
    kry_status s = guard([&] {
        KRY_REQUIRE(prob && b && x, "NULL argument");
        check_theta(theta);
        check_opts(opts);
        KRY_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        const Matern th = to_matern(theta);
        Spectrum& S = problem_spectrum(P, th, st);
        const double eta = th.tau2 / th.sigma2;
        const size_t n = (size_t)nrhs * P.p;
        DevBuf io;
        io.ensure(*P.ctx, 2 * n * sizeof(double) + 512);
        struct Free {
            Ctx& c;
            DevBuf& b;
            ~Free() { b.release(c); }
        } fr{*P.ctx, io};
        double* d_eta = io.as<double>();
        double* d_b = reinterpret_cast<double*>(io.as<char>() + 256);
        double* d_x = d_b + n;
        KRY_HIP(hipMemcpyAsync(d_eta, &eta, sizeof(double), hipMemcpyHostToDevice, st));
        std::vector<double> hb;
        const double* bsrc = b;
        if (P.obs_permuted) {  // the caller's order to the stored order
            hb.resize(n);
            for (int v = 0; v < nrhs; ++v)
                for (int64_t i = 0; i < P.p; ++i) hb[(size_t)v * P.p + i] = b[(size_t)v * P.p + (*P.h_obs_user)[i]];
            bsrc = hb.data();
        }
        KRY_HIP(hipMemcpyAsync(d_b, bsrc, n * sizeof(double), hipMemcpyHostToDevice, st));
        SolveStats ss;
        solve_device(P, opts->precision, S.s64.ptr, S.s32.ptr, 0, nrhs, d_eta, nrhs, d_b, d_x, opts->cg_rtol,
                     opts->cg_maxit, ss, st);
        KRY_HIP(hipMemcpyAsync(x, d_x, n * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        if (P.obs_permuted) {  // back to the caller's order
            std::vector<double> hx(x, x + n);
            for (int v = 0; v < nrhs; ++v)
                for (int64_t i = 0; i < P.p; ++i) x[(size_t)v * P.p + (*P.h_obs_user)[i]] = hx[(size_t)v * P.p + i];
        }
        for (int v = 0; v < nrhs; ++v) {
            if (iters) iters[v] = ss.iters[v];
            if (relres) relres[v] = ss.relres[v];
            if (ss.relres[v] > opts->cg_rtol) noconv = true;
        }
    });
    if (s == KRY_OK && noconv) {
        g_last_error = "CG reached cg_maxit before cg_rtol";
        return KRY_ENOCONV;
    }
    return s;
}

kry_status kry_gengk(kry_problem* prob, const kry_matern* theta, const kry_opts* opts, double* alpha, double* beta,
                     double* z, double* x_full, double* J) {
    return guard([&] {
        KRY_REQUIRE(prob && alpha && beta && z && J, "NULL argument");
        check_theta(theta);
        check_opts(opts);
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        GkOut G;
        if (opts->precision == KRY_FP32) gengk_device<float>(P, to_matern(theta), opts, G, x_full, st);
        else gengk_device<double>(P, to_matern(theta), opts, G, x_full, st);
        const int k = opts->gk_steps;
        for (int i = 0; i < k; ++i) {
            alpha[i] = G.alpha[i];
            z[i] = G.z[i];
        }
        alpha[k] = 0.0;
        for (int i = 0; i <= k; ++i) beta[i] = G.beta[i];
        *J = G.J;
    });
}

kry_status kry_loglik_batch(kry_problem* prob, const kry_matern* thetas, int32_t count, const kry_opts* opts,
                            kry_loglik_result* out) {
    bool noconv = false;
    kry_status s = guard([&] {
        KRY_REQUIRE(prob && thetas && out, "NULL argument");
        KRY_REQUIRE(count >= 1, "count must be >= 1");
        for (int t = 0; t < count; ++t) check_theta(&thetas[t]);
        check_opts(opts);
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        // points go through in chunks that bound the Krylov workspace
        const int np = nprobes_of(opts);
        const int nd = 1 + P.q;  // right-hand sides per point (data, covariate columns)
        const size_t per_point = (size_t)np * P.p * (opts->precision == KRY_FP32 ? 4 : 8) *
                                     (opts->reorth ? lanczos_cap(opts) + 3 : 5) +
                                 (size_t)nd * P.p * 8 * 8;
        // workspace per chunk: 48 GB, or half the context's budget when one is set
        size_t cap = (size_t)48e9;
        if (P.ctx->budget > 0) cap = std::min<size_t>(cap, P.ctx->budget / 2);
        std::vector<kry_loglik_result> res(count);
        if (opts->shift_share) {
            // whole groups per chunk: one Lanczos block and 3 CG base vectors
            // per group, 2 FP64 vectors per point; results do not depend on
            // the chunking
            std::vector<int> rep;
            const std::vector<int> grp = shift_groups(thetas, count, rep);
            const size_t per_group = per_point + 3 * (size_t)nd * P.p * 8, per_shift = 2 * (size_t)P.p * 8;
            std::vector<std::vector<int>> members(rep.size());
            for (int t = 0; t < count; ++t) members[grp[t]].push_back(t);
            std::vector<int> idx;
            size_t mem = 0;
            auto flush = [&]() {
                if (idx.empty()) return;
                std::vector<kry_matern> th(idx.size());
                std::vector<kry_loglik_result> r(idx.size());
                for (size_t i = 0; i < idx.size(); ++i) th[i] = thetas[idx[i]];
                loglik_points(P, th.data(), (int)idx.size(), opts, r.data(), st);
                for (size_t i = 0; i < idx.size(); ++i) res[idx[i]] = r[i];
                idx.clear();
                mem = 0;
            };
            for (const auto& mb : members) {
                if (mem > 0 && mem + per_group + mb.size() * per_shift > cap) flush();
                mem += per_group;
                for (int t : mb) {
                    if (mem + per_shift > cap && mem > per_group) {
                        flush();
                        mem = per_group;
                    }
                    idx.push_back(t);
                    mem += per_shift;
                }
            }
            flush();
        } else {
            int chunk = (int)std::max<size_t>(1, cap / std::max<size_t>(per_point, 1));
            chunk = std::min(chunk, (int)count);
            for (int t0 = 0; t0 < count; t0 += chunk) {
                const int c = std::min(chunk, (int)count - t0);
                loglik_points(P, thetas + t0, c, opts, res.data() + t0, st);
            }
        }
        std::copy(res.begin(), res.end(), out);
        noconv = any_not_converged(out, count, opts);
    });
    if (s == KRY_OK && noconv) {
        g_last_error = "CG reached cg_maxit before cg_rtol";
        return KRY_ENOCONV;
    }
    return s;
}

// ---- launch configuration ---------------------------------------------------------------
namespace {
void check_tuning(const kry_tuning* t) {
    KRY_REQUIRE(t->col_vectors == 1 || t->col_vectors == 2, "col_vectors must be 1 or 2");
    KRY_REQUIRE(t->row_tile_scale == 1 || t->row_tile_scale == 2, "row_tile_scale must be 1 or 2");
    KRY_REQUIRE(t->row_vthreads == 1 || t->row_vthreads == 2, "row_vthreads must be 1 or 2");
    KRY_REQUIRE(t->col_split == 0 || t->col_split == 1, "col_split must be 0 or 1");
    KRY_REQUIRE(t->row_split >= 0 && t->row_split <= 3, "row_split must be in 0..3");
}

kry_tuning to_abi(const Tuning& t, int real_bytes) {
    kry_tuning o;
    o.col_vectors = t.col_v ? t.col_v : (real_bytes == 4 ? 2 : 1);
    o.row_tile_scale = t.rt_scale;
    o.row_vthreads = t.row_vt;
    o.col_split = t.col_split;
    o.row_split = t.row_split;
    o.ms = t.ms;
    return o;
}

template <typename R>
Tuning autotune_impl(Problem& P, int nvec, hipStream_t st) {
    Ctx& C = *P.ctx;
    const int rb = (int)sizeof(R);
    const auto key = std::make_tuple(P.N1, P.N2, rb, Ctx::batch_class(nvec));
    // The row stages' parameters (rows per tile, values per thread, split
    // exchanges) and the column stage's (vectors per workgroup, split
    // exchange) act on different kernels: the rows are tuned first with the
    // column stage at its default, then the columns with the best rows.
    const bool big_rows = P.N2 / 2 >= 1024;
    std::vector<Tuning> rows_cand;
    for (int rs : {1, 2})
        for (int vt : {1, 2})
            for (int rsp = 0; rsp < 4; ++rsp) {
                if ((vt == 2 || rsp != 0) && !big_rows) continue;
                Tuning t;
                t.col_v = rb == 4 ? 2 : 1;
                t.rt_scale = rs;
                t.row_vt = vt;
                t.row_split = rsp;
                rows_cand.push_back(t);
            }
    // inputs: Rademacher vectors on the problem and the spectrum of a fixed point
    const kry_matern th{1.0, 0.1, 0.1, 0.5, 1.0, 0.0};
    Spectrum& S = problem_spectrum(P, to_matern(&th), st);
    const size_t vb = (size_t)nvec * P.p * sizeof(R);
    DevBuf& buf = P.tmp4;
    buf.ensure(C, 2 * vb + 256);
    R* in = buf.as<R>();
    R* outv = reinterpret_cast<R*>(buf.as<char>() + vb);
    double* d_eta = reinterpret_cast<double*>(buf.as<char>() + 2 * vb);
    const double eta = 0.1;
    KRY_HIP(hipMemcpyAsync(d_eta, &eta, sizeof(double), hipMemcpyHostToDevice, st));
    make_probes<R>(P, nvec, 1, 0, in, st);
    auto A = masked_op<R>(P, spec_ptr<R>(S), 0, nvec, d_eta);
    hipEvent_t e0, e1;
    KRY_HIP(hipEventCreate(&e0));
    KRY_HIP(hipEventCreate(&e1));
    Tuning best;
    best.ms = 1e300;
    auto try_config = [&](Tuning t) {
        {
            std::lock_guard<std::mutex> g(C.tune_mu);
            C.tuning[key] = t;
        }
        for (int w = 0; w < 2; ++w) A(in, outv, nvec, st, nullptr);
        std::vector<float> ms(5);
        for (float& m : ms) {
            KRY_HIP(hipEventRecord(e0, st));
            A(in, outv, nvec, st, nullptr);
            KRY_HIP(hipEventRecord(e1, st));
            KRY_HIP(hipEventSynchronize(e1));
            KRY_HIP(hipEventElapsedTime(&m, e0, e1));
        }
        std::sort(ms.begin(), ms.end());
        t.ms = ms[2];
        if (t.ms < best.ms) best = t;
    };
    try {
        for (const Tuning& t : rows_cand) try_config(t);
        const Tuning rows = best;
        for (int cv : {1, 2})
            for (int cs : {0, 1}) {
                if (cs == 1 && P.N1 < 256) continue;
                if (cv == rows.col_v && cs == rows.col_split) continue;  // timed in the first round
                Tuning t = rows;
                t.col_v = cv;
                t.col_split = cs;
                try_config(t);
            }
    } catch (...) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        std::lock_guard<std::mutex> g(C.tune_mu);
        C.tuning.erase(key);
        throw;
    }
    KRY_HIP(hipEventDestroy(e0));
    KRY_HIP(hipEventDestroy(e1));
    std::lock_guard<std::mutex> g(C.tune_mu);
    C.tuning[key] = best;
    return best;
}
}  // namespace

kry_status kry_autotune(kry_problem* prob, int32_t precision, int32_t nvec, kry_tuning* out) {
    return guard([&] {
        KRY_REQUIRE(prob && out, "NULL argument");
        KRY_REQUIRE(precision == KRY_FP64 || precision == KRY_FP32, "bad precision");
        KRY_REQUIRE(nvec >= 1 && nvec <= 4096, "nvec must be in [1, 4096]");
        Problem& P = prob->P;
        bind(*P.ctx);
        const Tuning t = precision == KRY_FP32 ? autotune_impl<float>(P, nvec, P.ctx->stream)
                                               : autotune_impl<double>(P, nvec, P.ctx->stream);
        *out = to_abi(t, precision == KRY_FP32 ? 4 : 8);
    });
}

kry_status kry_set_graphs(kry_ctx* ctx, int32_t enable) {
    return guard([&] {
        KRY_REQUIRE(ctx != nullptr, "NULL context");
        KRY_REQUIRE(enable == 0 || enable == 1, "enable must be 0 or 1");
        ctx->c.graphs = enable != 0;
    });
}

kry_status kry_set_tuning(kry_ctx* ctx, int32_t N1, int32_t N2, int32_t precision, const kry_tuning* t) {
    return guard([&] {
        KRY_REQUIRE(ctx != nullptr, "NULL context");
        KRY_REQUIRE(precision == KRY_FP64 || precision == KRY_FP32, "bad precision");
        KRY_REQUIRE(torus_side_ok(N1) && torus_side_ok(N2), "N1, N2 must be supported torus sides");
        const int rb = precision == KRY_FP32 ? 4 : 8;
        std::lock_guard<std::mutex> g(ctx->c.tune_mu);
        if (!t) {  // both batch classes
            for (int cls = 0; cls < 2; ++cls) ctx->c.tuning.erase(std::make_tuple((int)N1, (int)N2, rb, cls));
            return;
        }
        check_tuning(t);
        Tuning u;
        u.col_v = t->col_vectors;
        u.rt_scale = t->row_tile_scale;
        u.row_vt = t->row_vthreads;
        u.col_split = t->col_split;
        u.row_split = t->row_split;
        for (int cls = 0; cls < 2; ++cls) ctx->c.tuning[std::make_tuple((int)N1, (int)N2, rb, cls)] = u;
    });
}

kry_status kry_get_tuning(kry_ctx* ctx, int32_t N1, int32_t N2, int32_t precision, kry_tuning* out) {
    return guard([&] {
        KRY_REQUIRE(ctx && out, "NULL argument");
        KRY_REQUIRE(precision == KRY_FP64 || precision == KRY_FP32, "bad precision");
        const int rb = precision == KRY_FP32 ? 4 : 8;
        *out = to_abi(ctx->c.tuning_for(N1, N2, rb), rb);
    });
}

kry_status kry_loglik_multi(kry_problem* const* probs, const kry_matern* thetas, int32_t count, const kry_opts* opts,
                            kry_loglik_result* out) {
    bool noconv = false;
    kry_status s = guard([&] {
        KRY_REQUIRE(probs && thetas && out, "NULL argument");
        KRY_REQUIRE(count >= 1, "count must be >= 1");
        check_opts(opts);
        KRY_REQUIRE(opts->solver == KRY_SOLVER_CG, "kry_loglik_multi takes the CG quadratic form");
        KRY_REQUIRE(opts->shift_share == 0, "kry_loglik_multi does not share Krylov spaces across nuggets");
        for (int i = 0; i < count; ++i) {
            KRY_REQUIRE(probs[i] != nullptr, "NULL problem");
            KRY_REQUIRE(probs[i]->P.ctx == probs[0]->P.ctx, "problems of one call must share a context");
            KRY_REQUIRE(!probs[i]->P.irregular, "kry_loglik_multi takes gridded problems");
            check_theta(&thetas[i]);
        }
        Ctx& C = *probs[0]->P.ctx;
        bind(C);
        const int np = nprobes_of(opts);
        const size_t es = opts->precision == KRY_FP32 ? 4 : 8;
        size_t cap = (size_t)48e9;
        if (C.budget > 0) cap = std::min<size_t>(cap, C.budget / 2);
        // problems with equal embeddings go together, in order of first appearance
        std::vector<std::vector<int>> groups;
        std::vector<std::pair<int, int>> keys;
        for (int i = 0; i < count; ++i) {
            const std::pair<int, int> k{probs[i]->P.N1, probs[i]->P.N2};
            size_t g = 0;
            for (; g < keys.size() && keys[g] != k; ++g) {}
            if (g == keys.size()) {
                keys.push_back(k);
                groups.emplace_back();
            }
            groups[g].push_back(i);
        }
        // Tasks: each problem with covariates alone; the others in chunks of
        // one embedding group, whose products share every stage launch.
        // Tasks run concurrently on up to kWorkers streams, each worker with
        // one workspace that serves views of its tasks' problems; a task's
        // results do not depend on which worker runs it or what runs beside it.
        constexpr int kWorkers = 4;
        struct Task {
            std::vector<int> idx;
            bool cov = false;
            double cost = 0;
        };
        std::vector<Task> tasks;
        for (const auto& grp : groups) {
            std::vector<int> plain;
            for (int i : grp) {
                if (probs[i]->P.q > 0) tasks.push_back(Task{{i}, true, (double)probs[i]->P.N1 * probs[i]->P.N2});
                else plain.push_back(i);
            }
            if (plain.empty()) continue;
            int64_t pm = 0;
            for (int i : plain) pm = std::max(pm, probs[i]->P.p);
            // per problem: Lanczos block and CG / refinement vectors at the padded length
            const size_t per = (size_t)np * pm * es * (opts->reorth ? lanczos_cap(opts) + 3 : 5) + 12 * (size_t)pm * 8;
            const size_t chunk = std::max<size_t>(1, cap / kWorkers / std::max<size_t>(per, 1));
            for (size_t a = 0; a < plain.size(); a += chunk) {
                Task t;
                t.idx.assign(plain.begin() + a, plain.begin() + std::min(plain.size(), a + chunk));
                t.cost = (double)t.idx.size() * pm + (double)probs[plain[0]]->P.N1 * probs[plain[0]]->P.N2;
                tasks.push_back(t);
            }
        }
        // largest first, so that a worker's buffers reach their size early
        std::stable_sort(tasks.begin(), tasks.end(), [](const Task& a, const Task& b) { return a.cost > b.cost; });
        std::vector<kry_loglik_result> res(count);
        std::mutex mu;
        size_t next = 0;
        kry_status err = KRY_OK;
        std::string err_msg;
        auto worker = [&]() {
            hipStream_t ws = nullptr;
            Problem keep;  // the worker's workspace between tasks
            keep.ctx = &C;
            try {
                KRY_HIP(hipSetDevice(C.device));
                KRY_HIP(hipStreamCreateWithFlags(&ws, hipStreamNonBlocking));
                while (true) {
                    size_t ti;
                    {
                        std::lock_guard<std::mutex> g(mu);
                        if (next >= tasks.size() || err != KRY_OK) break;
                        ti = next++;
                    }
                    const Task& t = tasks[ti];
                    std::vector<Problem*> ps;
                    std::vector<kry_matern> th;
                    for (int i : t.idx) {
                        ps.push_back(&probs[i]->P);
                        th.push_back(thetas[i]);
                    }
                    std::vector<kry_loglik_result> r(ps.size());
                    Problem work = ps[0]->view();
                    work.no_graphs = true;  // several host threads: no stream capture
                    work.swap_work(keep);
                    try {
                        if (t.cov) loglik_points(work, th.data(), 1, opts, r.data(), ws);
                        else loglik_multi(work, ps, th.data(), opts, r.data(), ws);
                    } catch (...) {
                        (void)hipStreamSynchronize(ws);
                        work.swap_work(keep);
                        throw;
                    }
                    KRY_HIP(hipStreamSynchronize(ws));
                    work.swap_work(keep);
                    for (size_t j = 0; j < t.idx.size(); ++j) res[t.idx[j]] = r[j];
                }
            } catch (const Error& e) {
                std::lock_guard<std::mutex> g(mu);
                if (err == KRY_OK) {
                    err = e.status;
                    err_msg = e.what();
                }
            } catch (const std::exception& e) {
                std::lock_guard<std::mutex> g(mu);
                if (err == KRY_OK) {
                    err = KRY_EDEVICE;
                    err_msg = e.what();
                }
            }
            if (ws) {
                (void)hipStreamSynchronize(ws);
                (void)hipStreamDestroy(ws);
            }
            keep.release_work();
        };
        const int nw = (int)std::min<size_t>(kWorkers, tasks.size());
        std::vector<std::thread> pool;
        for (int w = 1; w < nw; ++w) pool.emplace_back(worker);
        worker();
        for (auto& t : pool) t.join();
        if (err != KRY_OK) throw Error(err, err_msg);
        std::copy(res.begin(), res.end(), out);
        noconv = any_not_converged(out, count, opts);
    });
    if (s == KRY_OK && noconv) {
        g_last_error = "CG reached cg_maxit before cg_rtol";
        return KRY_ENOCONV;
    }
    return s;
}

kry_status kry_loglik(kry_problem* prob, const kry_matern* theta, const kry_opts* opts, kry_loglik_result* out) {
    return kry_loglik_batch(prob, theta, 1, opts, out);
}

// ---- sampling -----------------------------------------------------------------------------
static void sample_fields(Problem& P, const Matern& th, int N1, int N2, uint64_t seed, int first_stream, int count,
                          double* d_out, double* lo, double* hi, hipStream_t st) {
    const int64_t nspec = (int64_t)(N2 / 2 + 1) * N1;
    DevBuf& sp = P.tmp4;
    sp.ensure(*P.ctx, nspec * sizeof(double));
    spectrum_device(P, N1, N2, th, sp.as<double>(), lo, hi, st);
    if (*lo < -1e-10 * *hi)
        throw Error(KRY_ENOTPSD, "embedding spectrum min/max = " + std::to_string(*lo / *hi) + " on a " +
                                     std::to_string(N1) + "x" + std::to_string(N2) + " torus");
    spectrum_scale(sp.as<double>(), nspec, 1.0 / ((double)N1 * N2), true, sp.as<double>(), nullptr, st);
    ConvSpec s;
    s.N1 = N1;
    s.N2 = N2;
    s.nvec = count;
    s.in_mode = IN_NOISE;
    s.in_rstride = N2;
    s.rows_in = N1;
    s.row_len = N2;
    s.seed = seed;
    s.stream0 = first_stream;
    s.out_mode = OUT_GRID;
    s.out = d_out;
    s.out_vstride = (int64_t)P.n1 * P.n2;
    s.rows_out = P.n1;
    s.cols_out = P.n2;
    s.scale = std::sqrt(th.sigma2);
    s.lam = sp.ptr;
    s.lam_tstride = 0;
    s.vecs_per_theta = count;
    conv_apply<double>(P, s, st);
    KRY_HIP(hipStreamSynchronize(st));
}

static void psd_torus(Problem& P, const Matern& th, int* N1, int* N2, hipStream_t st) {
    int a = P.N1, b = P.N2;
    const int64_t cap = 8192;
    DevBuf& sp = P.tmp4;
    while (true) {
        sp.ensure(*P.ctx, (size_t)(b / 2 + 1) * a * sizeof(double));
        double lo, hi;
        spectrum_device(P, a, b, th, sp.as<double>(), &lo, &hi, st);
        if (lo >= -1e-10 * hi) {
            *N1 = a;
            *N2 = b;
            return;
        }
        if (2 * a > cap || 2 * b > cap)
            throw Error(KRY_ENOTPSD, "no PSD embedding up to 8192 per axis (min/max = " + std::to_string(lo / hi) + ")");
        a *= 2;
        b *= 2;
    }
}

kry_status kry_psd_torus(kry_problem* prob, const kry_matern* theta, int32_t* N1, int32_t* N2) {
    return guard([&] {
        KRY_REQUIRE(prob && N1 && N2, "NULL argument");
        check_theta(theta);
        Problem& P = prob->P;
        bind(*P.ctx);
        int a, b;
        psd_torus(P, to_matern(theta), &a, &b, P.ctx->stream);
        *N1 = a;
        *N2 = b;
    });
}

kry_status kry_sample(kry_problem* prob, const kry_matern* theta, int32_t N1, int32_t N2, uint64_t seed,
                                 int32_t first_stream, int32_t count, double* out, double* minmax) {
    return guard([&] {
        KRY_REQUIRE(prob && out, "NULL argument");
        check_theta(theta);
        KRY_REQUIRE(count >= 1 && first_stream >= 0, "bad count or stream");
        Problem& P = prob->P;
        torus_args(P, N1, N2);
        KRY_REQUIRE(N1 >= 2 * P.n1 - 1 && N2 >= 2 * P.n2 - 1, "torus smaller than the embedding of the grid");
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        const size_t n = (size_t)P.n1 * P.n2 * count;
        DevBuf o;
        o.ensure(*P.ctx, n * sizeof(double));
        struct Free {
            Ctx& c;
            DevBuf& b;
            ~Free() { b.release(c); }
        } fr{*P.ctx, o};
        double lo, hi;
        sample_fields(P, to_matern(theta), N1, N2, seed, first_stream, count, o.as<double>(), &lo, &hi, st);
        KRY_HIP(hipMemcpy(out, o.ptr, n * sizeof(double), hipMemcpyDeviceToHost));
        if (minmax) {
            minmax[0] = lo;
            minmax[1] = hi;
        }
    });
}

// ---- kriging --------------------------------------------------------------------------------
void kry::krige_impl(Problem& P, const kry_matern* theta, const kry_opts* opts, const std::vector<int64_t>& tg,
                     double* mean_x, double* var_x, double* var_y, int32_t bootstrap_B, bool* noconv,
                     hipStream_t st) {
    const int64_t n = (int64_t)P.n1 * P.n2;
    const int64_t nt = (int64_t)tg.size();
    if (nt == 0) return;
    const Matern th = to_matern(theta);
    const double eta = th.tau2 / th.sigma2;
    const double tau = std::sqrt(th.tau2);
    Spectrum& S = problem_spectrum(P, th, st);
    // device scratch: eta, targets, w, full mean, target values
    const int64_t p = P.p;
    DevBuf& io = P.tmp1;
    io.ensure(*P.ctx, 512 + nt * sizeof(int64_t) + (size_t)p * 2 * sizeof(double) + (size_t)n * sizeof(double) +
                          (size_t)nt * 3 * sizeof(double) + 4096);
    Arena a;
    a.base = io.as<char>();
    double* d_eta = a.take<double>(1);
    int64_t* d_tg = a.take<int64_t>(nt);
    double* d_w = a.take<double>(p);
    double* d_full = a.take<double>(n);
    double* d_t1 = a.take<double>(nt);
    double* d_t2 = a.take<double>(nt);
    KRY_HIP(hipMemcpyAsync(d_eta, &eta, sizeof(double), hipMemcpyHostToDevice, st));
    KRY_HIP(hipMemcpyAsync(d_tg, tg.data(), nt * sizeof(int64_t), hipMemcpyHostToDevice, st));
    // mean: w = K^{-1} y, xhat = Sigma A^T w
    std::vector<double> beta;
    if (P.q == 0) {
        SolveStats ss;
        solve_device(P, opts->precision, S.s64.ptr, S.s32.ptr, 0, 1, d_eta, 1, P.y64.as<double>(), d_w,
                     opts->cg_rtol, opts->cg_maxit, ss, st);
        if (ss.relres[0] > opts->cg_rtol) *noconv = true;
    } else {
        if (P.irregular) throw Error(KRY_ENOTIMPL, "kriging with covariates needs them at the grid cells, which an irregular problem does not hold");
        // covariates: K^{-1} of the data and of every column in one solve,
        // beta_hat by GLS, then w = K^{-1} (y - X beta_hat) = K^{-1} yc - K^{-1} X delta
        beta = gls_beta(P, theta, opts, d_w, noconv, st);
    }
    cov_full<double>(P, S.s64.ptr, d_w, d_full, 1, st);
    hipLaunchKernelGGL(k_pick, grid1(nt), dim3(256), 0, st, d_full, d_tg, nt, d_t1);
    KRY_HIP(hipGetLastError());
    KRY_HIP(hipMemcpyAsync(mean_x, d_t1, nt * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < P.q; ++j) {  // + X_t beta_hat
        const double* xj = P.h_X->data() + (size_t)j * n;
        for (int64_t i = 0; i < nt; ++i) mean_x[i] += xj[tg[i]] * beta[j];
    }
    if (!var_x && !var_y) return;
    if (bootstrap_B == 0) {
        // exact: multi-RHS CG on the cross-correlation columns, in chunks
        P.lagtmp.ensure(*P.ctx, (size_t)P.N1 * P.N2 * sizeof(double));
        lag_grid_device(*P.ctx, P.N1, P.N2, P.dx1, P.dx2, th, P.lagtmp.as<double>(), st);
        const int chunk = (int)std::max<int64_t>(
            1, std::min<int64_t>(std::min<int64_t>(256, nt), (int64_t)(2e9 / (8.0 * p * 6))));
        DevBuf& cb = P.tmp2;
        cb.ensure(*P.ctx, (size_t)chunk * p * 2 * sizeof(double) + (size_t)chunk * 257 * sizeof(double) + 1024);
        double* Cc = cb.as<double>();
        double* Wc = Cc + (size_t)chunk * p;
        double* part = Wc + (size_t)chunk * p;
        double* dots = part + (size_t)chunk * 256;
        std::vector<double> q(chunk);
        for (int64_t t0 = 0; t0 < nt; t0 += chunk) {
            const int c = (int)std::min<int64_t>(chunk, nt - t0);
            if (P.irregular) {
                irr_cross_corr(P, P.lagtmp.as<double>(), d_tg + t0, c, Cc, st);
            } else {
                hipLaunchKernelGGL(k_cross_corr, grid1(p, c), dim3(256), 0, st, P.lagtmp.as<double>(), P.N1, P.N2,
                                   P.cell.as<int32_t>(), p, P.n2, d_tg + t0, Cc);
                KRY_HIP(hipGetLastError());
            }
            SolveStats s2;
            solve_device(P, opts->precision, S.s64.ptr, S.s32.ptr, 0, c, d_eta, c, Cc, Wc, opts->cg_rtol,
                         opts->cg_maxit, s2, st);
            for (int v = 0; v < c; ++v)
                if (s2.relres[v] > opts->cg_rtol) *noconv = true;
            dot_batched<double>(Cc, p, Wc, p, p, c, part, dots, st);
            KRY_HIP(hipMemcpyAsync(q.data(), dots, c * sizeof(double), hipMemcpyDeviceToHost, st));
            KRY_HIP(hipStreamSynchronize(st));
            for (int v = 0; v < c; ++v) {
                const double vx = th.sigma2 * (1.0 - q[v]);
                if (var_x) var_x[t0 + v] = vx;
                if (var_y) var_y[t0 + v] = vx + th.tau2;
            }
        }
        return;
    }
    // parametric bootstrap (eq. bootstrap_uq)
    int N1s, N2s;
    psd_torus(P, th, &N1s, &N2s, st);
    const int B = bootstrap_B;
    DevBuf& bb = P.tmp3;
    bb.ensure(*P.ctx, (size_t)B * n * 2 * sizeof(double) + (size_t)B * p * 2 * sizeof(double) + 1024);
    double* F = bb.as<double>();
    double* XH = F + (size_t)B * n;
    double* YB = XH + (size_t)B * n;
    double* WB = YB + (size_t)B * p;
    double lo, hi;
    sample_fields(P, th, N1s, N2s, opts->seed, 0, B, F, &lo, &hi, st);
    if (P.irregular) {
        irr_boot_obs(P, F, B, tau, opts->seed, YB, st);
    } else {
        hipLaunchKernelGGL(k_boot_obs, grid1(p, B), dim3(256), 0, st, F, n, P.cell.as<int32_t>(), p, tau, opts->seed,
                           YB);
        KRY_HIP(hipGetLastError());
    }
    SolveStats s3;
    solve_device(P, opts->precision, S.s64.ptr, S.s32.ptr, 0, B, d_eta, B, YB, WB, opts->cg_rtol, opts->cg_maxit, s3,
                 st);
    for (int v = 0; v < B; ++v)
        if (s3.relres[v] > opts->cg_rtol) *noconv = true;
    cov_full<double>(P, S.s64.ptr, WB, XH, B, st);
    hipLaunchKernelGGL(k_boot_acc, grid1(nt), dim3(256), 0, st, F, XH, n, B, d_tg, nt, tau, opts->seed, d_t1, d_t2);
    KRY_HIP(hipGetLastError());
    if (var_x) KRY_HIP(hipMemcpyAsync(var_x, d_t1, nt * sizeof(double), hipMemcpyDeviceToHost, st));
    if (var_y) KRY_HIP(hipMemcpyAsync(var_y, d_t2, nt * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
}

kry_status kry_krige(kry_problem* prob, const kry_matern* theta, const kry_opts* opts,
                     const int64_t* targets, int64_t ntargets, double* mean_x, double* var_x, double* var_y,
                     int32_t bootstrap_B) {
    bool noconv = false;
    kry_status s = guard([&] {
        KRY_REQUIRE(prob && mean_x, "NULL argument");
        check_theta(theta);
        check_opts(opts);
        KRY_REQUIRE(bootstrap_B >= 0 && bootstrap_B <= 4096, "bootstrap_B must be in [0, 4096]");
        Problem& P = prob->P;
        const int64_t n = (int64_t)P.n1 * P.n2;
        std::vector<int64_t> tg;
        if (targets) {
            KRY_REQUIRE(ntargets >= 1, "ntargets must be >= 1");
            tg.assign(targets, targets + ntargets);
            for (int64_t t : tg) KRY_REQUIRE(t >= 0 && t < n, "target cell id out of range");
        } else if (P.irregular) {  // every grid cell
            tg.resize(n);
            for (int64_t c = 0; c < n; ++c) tg[c] = c;
            KRY_REQUIRE(ntargets == n, "ntargets must equal the number of grid cells");
        } else {
            for (int64_t c = 0; c < n; ++c)
                if (!(*P.h_mask)[c]) tg.push_back(c);
            KRY_REQUIRE(ntargets == (int64_t)tg.size(), "ntargets must equal the number of unobserved cells");
        }
        bind(*P.ctx);
        krige_impl(P, theta, opts, tg, mean_x, var_x, var_y, bootstrap_B, &noconv, P.ctx->stream);
    });
    if (s == KRY_OK && noconv) {
        g_last_error = "CG reached cg_maxit before cg_rtol";
        return KRY_ENOCONV;
    }
    return s;
}

// ---- fit ----------------------------------------------------------------------------------------
static void fit_impl(Problem& P, const kry_matern* init, uint32_t free_mask, const kry_opts* opts, double xtol,
                     int32_t maxiter, kry_matern* est, kry_loglik_result* at_est) {
    {
        hipStream_t st = P.ctx->stream;
        // free coordinates: log range, log eta
        std::vector<int> which;
        if (free_mask & 1u) which.push_back(0);
        if (free_mask & 2u) which.push_back(1);
        const int d = (int)which.size();
        const double x0[2] = {std::log(init->range), std::log(init->tau2 / init->sigma2)};
        auto point = [&](const std::vector<double>& x) {
            double lr = x0[0], le = x0[1];
            for (int i = 0; i < d; ++i) (which[i] == 0 ? lr : le) = x[i];
            kry_matern t = *init;
            t.range = std::exp(lr);
            t.sigma2 = 1.0;
            t.tau2 = std::exp(le);
            return t;
        };
        // KRY_VERBOSE >= 1 in the environment: one line per evaluation on
        // stderr, so that a long fit reports its progress
        const char* vb = std::getenv("KRY_VERBOSE");
        const bool verbose = vb && std::atoi(vb) >= 1;
        int nev = 0;
        auto f = [&](const std::vector<double>& x) {
            kry_matern t = point(x);
            kry_loglik_result r;
            loglik_points(P, &t, 1, opts, &r, st);
            if (verbose)
                std::fprintf(stderr, "[kry] fit evaluation %d: range %.6g nugget ratio %.6g l_p %.6f (%d Lanczos steps, %d CG iterations)\n",
                             ++nev, t.range, t.tau2, r.loglik_profiled, r.lanczos_steps_used, r.cg_iters);
            return -r.loglik_profiled;
        };
        // Nelder-Mead (reflection 1, expansion 2, contraction 1/2, shrink 1/2)
        std::vector<std::vector<double>> sx(d + 1, std::vector<double>(d));
        for (int i = 0; i < d; ++i) sx[0][i] = x0[which[i]];
        for (int k = 1; k <= d; ++k) {
            sx[k] = sx[0];
            sx[k][k - 1] += 0.3;
        }
        std::vector<double> fx(d + 1);
        for (int k = 0; k <= d; ++k) fx[k] = f(sx[k]);
        for (int it = 0; it < maxiter; ++it) {
            std::vector<int> ord(d + 1);
            std::iota(ord.begin(), ord.end(), 0);
            std::sort(ord.begin(), ord.end(), [&](int a, int b) { return fx[a] < fx[b]; });
            std::vector<std::vector<double>> s2(d + 1);
            std::vector<double> f2(d + 1);
            for (int k = 0; k <= d; ++k) {
                s2[k] = sx[ord[k]];
                f2[k] = fx[ord[k]];
            }
            sx = s2;
            fx = f2;
            double size = 0;
            for (int k = 1; k <= d; ++k)
                for (int i = 0; i < d; ++i) size = std::max(size, std::fabs(sx[k][i] - sx[0][i]));
            if (size < xtol) break;
            std::vector<double> c(d, 0.0);
            for (int k = 0; k < d; ++k)
                for (int i = 0; i < d; ++i) c[i] += sx[k][i] / d;
            auto lerp = [&](double t) {
                std::vector<double> r(d);
                for (int i = 0; i < d; ++i) r[i] = c[i] + t * (sx[d][i] - c[i]);
                return r;
            };
            std::vector<double> xr = lerp(-1.0);
            const double fr = f(xr);
            if (fr < fx[0]) {
                std::vector<double> xe = lerp(-2.0);
                const double fe = f(xe);
                if (fe < fr) {
                    sx[d] = xe;
                    fx[d] = fe;
                } else {
                    sx[d] = xr;
                    fx[d] = fr;
                }
            } else if (fr < fx[d - 1]) {
                sx[d] = xr;
                fx[d] = fr;
            } else {
                const bool outside = fr < fx[d];
                std::vector<double> xc = lerp(outside ? -0.5 : 0.5);
                const double fc = f(xc);
                if (fc < (outside ? fr : fx[d])) {
                    sx[d] = xc;
                    fx[d] = fc;
                } else {
                    for (int k = 1; k <= d; ++k) {
                        for (int i = 0; i < d; ++i) sx[k][i] = sx[0][i] + 0.5 * (sx[k][i] - sx[0][i]);
                        fx[k] = f(sx[k]);
                    }
                }
            }
        }
        int best = 0;
        for (int k = 1; k <= d; ++k)
            if (fx[k] < fx[best]) best = k;
        kry_matern t = point(sx[best]);
        kry_loglik_result r;
        loglik_points(P, &t, 1, opts, &r, st);
        t.sigma2 = r.sigma2_hat;
        t.tau2 = std::exp(std::log(point(sx[best]).tau2)) * r.sigma2_hat;
        *est = t;
        if (at_est) {
            kry_matern t2 = t;
            loglik_points(P, &t2, 1, opts, at_est, st);
        }
    }
}

static void check_fit_args(const kry_matern* init, uint32_t free_mask, const kry_opts* opts, double xtol,
                           int32_t maxiter) {
    check_theta(init);
    check_opts(opts);
    KRY_REQUIRE((free_mask & 3u) != 0, "free_mask must free the range and/or the nugget ratio");
    KRY_REQUIRE(xtol > 0 && maxiter >= 1, "bad xtol or maxiter");
    KRY_REQUIRE(init->tau2 > 0, "the nugget ratio needs tau2 > 0 to be fitted on the log scale");
}

kry_status kry_fit(kry_problem* prob, const kry_matern* init, uint32_t free_mask, const kry_opts* opts,
                   double xtol, int32_t maxiter, kry_matern* est, kry_loglik_result* at_est) {
    return guard([&] {
        KRY_REQUIRE(prob && init && est, "NULL argument");
        check_fit_args(init, free_mask, opts, xtol, maxiter);
        Problem& P = prob->P;
        bind(*P.ctx);
        fit_impl(P, init, free_mask, opts, xtol, maxiter, est, at_est);
    });
}

kry_status kry_bootstrap_theta(kry_problem* prob, const kry_matern* theta_hat, uint32_t free_mask,
                               const kry_opts* opts, double xtol, int32_t maxiter, int32_t B, kry_matern* est,
                               double* sd) {
    return guard([&] {
        KRY_REQUIRE(prob && theta_hat && est, "NULL argument");
        check_fit_args(theta_hat, free_mask, opts, xtol, maxiter);
        KRY_REQUIRE(B >= 1 && B <= 4096, "B must be in [1, 4096]");
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        const Matern th = to_matern(theta_hat);
        const int64_t n = (int64_t)P.n1 * P.n2, p = P.p;
        // the mean at the estimates: X beta_hat (GLS at theta_hat)
        std::vector<double> mean(p, 0.0);
        if (P.q > 0) {
            const std::vector<double> beta = gls_beta(P, theta_hat, opts, nullptr, nullptr, st);
            for (int j = 0; j < P.q; ++j)
                for (int64_t i = 0; i < p; ++i)
                    mean[i] += beta[j] * (P.irregular ? (*P.h_X)[(size_t)j * p + (*P.h_obs_user)[i]]
                                                      : (*P.h_X)[(size_t)j * n + (*P.h_cell)[i]]);
        }
        // every simulated data set, as the prediction-variance bootstrap draws them
        int N1s, N2s;
        psd_torus(P, th, &N1s, &N2s, st);
        DevBuf& bb = P.tmp3;
        bb.ensure(*P.ctx, ((size_t)B * n + (size_t)B * p) * sizeof(double) + 512);
        double* F = bb.as<double>();
        double* YB = F + (size_t)B * n;
        double lo, hi;
        sample_fields(P, th, N1s, N2s, opts->seed, 0, B, F, &lo, &hi, st);
        const double tau = std::sqrt(th.tau2);
        if (P.irregular) {
            irr_boot_obs(P, F, B, tau, opts->seed, YB, st);
        } else {
            hipLaunchKernelGGL(k_boot_obs, grid1(p, B), dim3(256), 0, st, F, n, P.cell.as<int32_t>(), p, tau,
                               opts->seed, YB);
            KRY_HIP(hipGetLastError());
        }
        std::vector<double> ys((size_t)B * p), saved(p);
        KRY_HIP(hipMemcpyAsync(ys.data(), YB, ys.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipMemcpyAsync(saved.data(), P.y64.ptr, p * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        try {
            for (int b = 0; b < B; ++b) {
                std::vector<double> yb(ys.begin() + (size_t)b * p, ys.begin() + (size_t)(b + 1) * p);
                for (int64_t i = 0; i < p; ++i) yb[i] += mean[i];
                upload_compact(P, yb);
                fit_impl(P, theta_hat, free_mask, opts, xtol, maxiter, &est[b], nullptr);
            }
        } catch (...) {
            upload_compact(P, saved);
            throw;
        }
        upload_compact(P, saved);
        if (sd) {
            for (int c = 0; c < 2; ++c) {
                double m = 0, ss = 0;
                for (int b = 0; b < B; ++b) m += c == 0 ? std::log(est[b].range) : std::log(est[b].tau2 / est[b].sigma2);
                m /= B;
                for (int b = 0; b < B; ++b) {
                    const double v = (c == 0 ? std::log(est[b].range) : std::log(est[b].tau2 / est[b].sigma2)) - m;
                    ss += v * v;
                }
                sd[c] = B > 1 ? std::sqrt(ss / (B - 1)) : 0.0;
            }
        }
    });
}


// ---- the paper's objective, its trust-region fit and the low-rank posterior variance -----------
static std::vector<double> start_beta(Problem& P, const kry_matern* theta, const kry_opts* opts, const double* beta,
                                      hipStream_t st) {
    if (P.q == 0) return {};
    if (beta) {
        for (int j = 0; j < P.q; ++j) KRY_REQUIRE(std::isfinite(beta[j]), "beta has a non-finite entry");
        return std::vector<double>(beta, beta + P.q);
    }
    return gls_beta(P, theta, opts, nullptr, nullptr, st);
}

static void check_gk_opts(const kry_matern* theta, const kry_opts* opts) {
    check_theta(theta);
    check_opts(opts);
    KRY_REQUIRE(theta->tau2 > 0, "tau2 must be > 0 for Algorithm 1");
}

kry_status kry_plik(kry_problem* prob, const kry_matern* theta, const double* beta, const kry_opts* opts,
                    kry_plik_result* out) {
    return guard([&] {
        KRY_REQUIRE(prob && out, "NULL argument");
        check_gk_opts(theta, opts);
        Problem& P = prob->P;
        KRY_REQUIRE(P.q == 0 || beta != nullptr, "beta is NULL but the problem has covariates");
        bind(*P.ctx);
        const std::vector<double> b = start_beta(P, theta, opts, beta, P.ctx->stream);
        kry_plik_result r;
        plik_device(P, theta, b.data(), opts, &r, P.ctx->stream);
        *out = r;
    });
}

kry_status kry_plik_fit(kry_problem* prob, const kry_matern* init, const double* beta0, uint32_t free_mask,
                        const kry_opts* opts, double delta0, double gtol, int32_t maxiter, kry_matern* est,
                        double* beta_est, kry_plik_result* at_est, int32_t* iters) {
    return guard([&] {
        KRY_REQUIRE(prob && est, "NULL argument");
        check_gk_opts(init, opts);
        KRY_REQUIRE((free_mask & 15u) != 0 && (free_mask & ~15u) == 0, "free_mask must select from bits 0..3");
        KRY_REQUIRE(std::isfinite(delta0) && delta0 > 0, "delta0 must be > 0");
        KRY_REQUIRE(std::isfinite(gtol) && gtol >= 0, "gtol must be >= 0");
        KRY_REQUIRE(maxiter >= 1, "maxiter must be >= 1");
        Problem& P = prob->P;
        bind(*P.ctx);
        hipStream_t st = P.ctx->stream;
        const int q = P.q;
        const std::vector<double> b0 = start_beta(P, init, opts, beta0, st);
        // coordinates: log sigma2, log tau2, log range, beta
        std::vector<double> x0 = {std::log(init->sigma2), std::log(init->tau2), std::log(init->range)};
        x0.insert(x0.end(), b0.begin(), b0.end());
        std::vector<int> freec;
        if (free_mask & 2u) freec.push_back(0);
        if (free_mask & 4u) freec.push_back(1);
        if (free_mask & 1u) freec.push_back(2);
        if (free_mask & 8u)
            for (int j = 0; j < q; ++j) freec.push_back(3 + j);
        KRY_REQUIRE(!freec.empty(), "nothing to fit (bit 3 frees beta, which the problem does not have)");
        const int d = (int)freec.size();
        auto full_of = [&](const std::vector<double>& xf) {
            std::vector<double> x = x0;
            for (int i = 0; i < d; ++i) x[freec[i]] = xf[i];
            return x;
        };
        auto theta_of = [&](const std::vector<double>& x) {
            kry_matern t = *init;
            t.sigma2 = std::exp(x[0]);
            t.tau2 = std::exp(x[1]);
            t.range = std::exp(x[2]);
            return t;
        };
        auto eval = [&](const std::vector<double>& xf, double& f, std::vector<double>& g, kry_plik_result& r) {
            const std::vector<double> x = full_of(xf);
            const kry_matern t = theta_of(x);
            plik_device(P, &t, q ? x.data() + 3 : nullptr, opts, &r, st);
            std::vector<double> gf = {-r.grad_lam2 / t.sigma2, -r.grad_lame2 / t.tau2, t.range * r.grad_range};
            for (int j = 0; j < q; ++j) gf.push_back(r.grad_beta[j]);
            g.assign(d, 0.0);
            for (int i = 0; i < d; ++i) g[i] = gf[freec[i]];
            f = r.pl;
        };
        std::vector<double> x(d);
        for (int i = 0; i < d; ++i) x[i] = x0[freec[i]];
        double fx;
        std::vector<double> g;
        kry_plik_result rx;
        eval(x, fx, g, rx);
        double delta = delta0;
        int it = 0;
        for (it = 1; it <= maxiter; ++it) {
            double gn = 0;
            for (double v : g) gn += v * v;
            gn = std::sqrt(gn);
            if (gn <= gtol) break;
            // model gain t - t^2 / 2 in f with t = g^T s; largest at t = 1
            std::vector<double> s(d);
            bool boundary;
            if (1.0 / gn <= delta) {
                for (int i = 0; i < d; ++i) s[i] = g[i] / (gn * gn);
                boundary = false;
            } else {
                for (int i = 0; i < d; ++i) s[i] = delta * g[i] / gn;
                boundary = true;
            }
            double t = 0;
            for (int i = 0; i < d; ++i) t += g[i] * s[i];
            const double pred = t - 0.5 * t * t;
            std::vector<double> xn(d);
            for (int i = 0; i < d; ++i) xn[i] = x[i] + s[i];
            double fn;
            std::vector<double> gnew;
            kry_plik_result rn;
            eval(xn, fn, gnew, rn);
            const double ratio = (pred > 0 && std::isfinite(fn)) ? (fn - fx) / pred : -1.0;
            if (ratio < 0.25) delta *= 0.25;
            else if (ratio > 0.75 && boundary) delta *= 2.0;
            if (ratio > 0) {
                x = xn;
                fx = fn;
                g = gnew;
                rx = rn;
            }
            if (delta < 1e-8) break;
        }
        const std::vector<double> xf = full_of(x);
        *est = theta_of(xf);
        if (beta_est)
            for (int j = 0; j < q; ++j) beta_est[j] = xf[3 + j];
        if (at_est) *at_est = rx;
        if (iters) *iters = std::min(it, (int)maxiter);
    });
}

kry_status kry_posterior_variance(kry_problem* prob, const kry_matern* theta, const double* beta,
                                  const kry_opts* opts, double* var_x, double* var_y, double* mean_x) {
    return guard([&] {
        KRY_REQUIRE(prob && var_x, "NULL argument");
        check_gk_opts(theta, opts);
        Problem& P = prob->P;
        bind(*P.ctx);
        const std::vector<double> b = start_beta(P, theta, opts, beta, P.ctx->stream);
        posterior_variance_device(P, theta, b.data(), opts, var_x, var_y, mean_x, P.ctx->stream);
    });
}

kry_status kry_tridiag_eigen(int32_t k, const double* d, const double* e, double* theta, double* W) {
    return guard([&] {
        KRY_REQUIRE(k >= 1 && k <= 8192, "k must be in [1, 8192]");
        KRY_REQUIRE(d && theta && W && (k == 1 || e), "NULL argument");
        std::vector<double> dd(d, d + k), ee(e ? e : d, e ? e + (k - 1) : d), WW;
        for (double v : dd) KRY_REQUIRE(std::isfinite(v), "d has a non-finite entry");
        for (double v : ee) KRY_REQUIRE(std::isfinite(v), "e has a non-finite entry");
        tridiag_eigen(dd, ee, WW);
        std::copy(dd.begin(), dd.end(), theta);
        std::copy(WW.begin(), WW.end(), W);
    });
}
