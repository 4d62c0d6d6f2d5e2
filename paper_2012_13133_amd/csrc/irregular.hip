// Irregularly spaced observations (Sec. 2): the latent field lives on the
// grid and observation j is the Wendland-weighted convex combination of the
// grid values at the corners of its cell, y = A x + eps with at most four
// nonzeros per row of A.  The covariance of the observations is
// K = A Sigma A^T + eta I; its product runs as A^T (rows over the grid, so
// every cell sums its own observations in a fixed order), the
// circulant-embedding product on the full grid, and A (four slots per
// observation) with the nugget term.  All sums over A are in FP64, rounded
// once to the working precision.
#include "internal.hpp"
#include "krylov.hpp"

namespace kry {
namespace {

dim3 vgrid(int64_t n, int nvec) {
    int64_t b = (n + 255) / 256;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return dim3((unsigned)b, nvec);
}

// Up to IV vectors per thread, so every entry of A or A^T is read once per
// group of IV vectors rather than once per vector.
constexpr int IV = 8;

// out[v][c] = scale * sum_{e in row c of A^T} w_e x[v][obs_e]
template <typename RI, typename RO>
__global__ void k_irr_scatter(const RI* __restrict__ x, int64_t xs, const int32_t* __restrict__ off,
                              const int32_t* __restrict__ obs, const double* __restrict__ w, int64_t n, int nvec,
                              RO* __restrict__ out, int64_t os, double scale, const int* __restrict__ active) {
    const int v0 = blockIdx.y * IV;
    bool on[IV];
    bool any = false;
#pragma unroll
    for (int u = 0; u < IV; ++u) {
        on[u] = v0 + u < nvec && (!active || active[v0 + u]);
        any = any || on[u];
    }
    if (!any) return;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        double acc[IV];
#pragma unroll
        for (int u = 0; u < IV; ++u) acc[u] = 0.0;
        const int e1 = off[c + 1];
        for (int e = off[c]; e < e1; ++e) {
            const int64_t o = obs[e];
            const double we = w[e];
#pragma unroll
            for (int u = 0; u < IV; ++u)
                if (on[u]) acc[u] += we * (double)x[(int64_t)(v0 + u) * xs + o];
        }
#pragma unroll
        for (int u = 0; u < IV; ++u)
            if (on[u]) out[(int64_t)(v0 + u) * os + c] = (RO)(scale * acc[u]);
    }
}

// out[v][j] = sum_s w_js grid[v][cell_js] (+ eta[v / vpt] xin[v][j])
template <typename RI, typename RO>
__global__ void k_irr_gather(const RI* __restrict__ grid, int64_t gs, const int32_t* __restrict__ cell4,
                             const double* __restrict__ w4, int64_t p, int nvec, RO* __restrict__ out, int64_t os,
                             const RO* __restrict__ xin, const double* __restrict__ eta, int vpt,
                             const int* __restrict__ active) {
    const int v0 = blockIdx.y * IV;
    bool on[IV];
    double e[IV];
    bool any = false;
#pragma unroll
    for (int u = 0; u < IV; ++u) {
        on[u] = v0 + u < nvec && (!active || active[v0 + u]);
        e[u] = (on[u] && xin) ? eta[(v0 + u) / vpt] : 0.0;
        any = any || on[u];
    }
    if (!any) return;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        int c[4];
        double wv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            c[s] = cell4[4 * j + s];
            wv[s] = w4[4 * j + s];
        }
#pragma unroll
        for (int u = 0; u < IV; ++u) {
            if (!on[u]) continue;
            const RI* gv = grid + (int64_t)(v0 + u) * gs;
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (c[s] >= 0) acc += wv[s] * (double)gv[c[s]];
            if (xin) acc += e[u] * (double)xin[(int64_t)(v0 + u) * os + j];
            out[(int64_t)(v0 + u) * os + j] = (RO)acc;
        }
    }
}

// out[v * p + j] = sum_s w_js c(cell_js - t_v), lags wrapped on the N1 x N2 torus
__global__ void k_irr_cross_corr(const double* __restrict__ lag, int N1, int N2, const int32_t* __restrict__ cell4,
                                 const double* __restrict__ w4, int64_t p, int n2,
                                 const int64_t* __restrict__ targets, double* __restrict__ out) {
    const int v = blockIdx.y;
    const int64_t t = targets[v];
    const int tr = (int)(t / n2), tc = (int)(t % n2);
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int s = 0; s < 4; ++s) {
            const int c = cell4[4 * j + s];
            if (c < 0) continue;
            const int r = c / n2, cc = c - (c / n2) * n2;
            int l1 = (r - tr) % N1;
            if (l1 < 0) l1 += N1;
            int l2 = (cc - tc) % N2;
            if (l2 < 0) l2 += N2;
            acc += w4[4 * j + s] * lag[(int64_t)l1 * N2 + l2];
        }
        out[(int64_t)v * p + j] = acc;
    }
}

template <typename R>
__global__ void k_irr_permute(const R* __restrict__ src, R* __restrict__ dst, const int32_t* __restrict__ user,
                              int64_t p, int to_stored) {
    const int v = blockIdx.y;
    const R* s = src + (int64_t)v * p;
    R* d = dst + (int64_t)v * p;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x) {
        if (to_stored) d[i] = s[user[i]];
        else d[user[i]] = s[i];
    }
}

__global__ void k_irr_boot_obs(const double* __restrict__ fields, int64_t n, const int32_t* __restrict__ cell4,
                               const double* __restrict__ w4, const int32_t* __restrict__ user, int64_t p,
                               double tau, uint64_t seed, double* __restrict__ yb) {
    const int b = blockIdx.y;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int s = 0; s < 4; ++s) {
            const int c = cell4[4 * j + s];
            if (c >= 0) acc += w4[4 * j + s] * fields[(int64_t)b * n + c];
        }
        yb[(int64_t)b * p + j] = acc + tau * philox_normal((uint32_t)user[j], (uint32_t)b, DOMAIN_NOISE, seed);
    }
}

}  // namespace

template <typename RI, typename RO>
void irr_scatter(const Problem& P, const RI* x, int64_t xs, int nvec, RO* out, double scale, const int* active,
                 hipStream_t st) {
    const int64_t n = (int64_t)P.n1 * P.n2;
    hipLaunchKernelGGL((k_irr_scatter<RI, RO>), vgrid(n, (nvec + IV - 1) / IV), dim3(256), 0, st, x, xs,
                       P.at_off.as<int32_t>(), P.at_obs.as<int32_t>(), P.at_w.as<double>(), n, nvec, out, n, scale,
                       active);
    KRY_HIP(hipGetLastError());
}

template <typename RI, typename RO>
void irr_gather(const Problem& P, const RI* grid, int nvec, RO* out, const RO* xin, const double* eta, int vpt,
                const int* active, hipStream_t st) {
    const int64_t n = (int64_t)P.n1 * P.n2;
    hipLaunchKernelGGL((k_irr_gather<RI, RO>), vgrid(P.p, (nvec + IV - 1) / IV), dim3(256), 0, st, grid, n,
                       P.a_cell.as<int32_t>(), P.a_w.as<double>(), P.p, nvec, out, P.p, xin, eta, vpt, active);
    KRY_HIP(hipGetLastError());
}

template void irr_scatter<double, double>(const Problem&, const double*, int64_t, int, double*, double, const int*,
                                          hipStream_t);
template void irr_scatter<float, float>(const Problem&, const float*, int64_t, int, float*, double, const int*,
                                        hipStream_t);
template void irr_gather<double, double>(const Problem&, const double*, int, double*, const double*, const double*,
                                         int, const int*, hipStream_t);
template void irr_gather<float, float>(const Problem&, const float*, int, float*, const float*, const double*, int,
                                       const int*, hipStream_t);

template <typename R>
MatvecFn<R> irregular_op(Problem& P, const void* lam, int64_t lam_tstride, int vpt, const double* d_eta) {
    Problem* pp = &P;
    return [pp, lam, lam_tstride, vpt, d_eta](const R* x, R* y, int nvec, hipStream_t st, const int* active) {
        Problem& Q = *pp;
        const int64_t n = (int64_t)Q.n1 * Q.n2;
        // grid vectors: A^T x (FP64 sums rounded once, the dense input of the product) and the product
        const size_t gin = ((size_t)nvec * n * sizeof(R) + 255) & ~size_t(255);
        Q.irr.ensure(*Q.ctx, gin + (size_t)nvec * n * sizeof(R) + 256);
        R* Gin = Q.irr.as<R>();
        R* Gout = reinterpret_cast<R*>(Q.irr.as<char>() + gin);
        irr_scatter<R, R>(Q, x, Q.p, nvec, Gin, 1.0, active, st);
        ConvSpec s;
        s.N1 = Q.N1;
        s.N2 = Q.N2;
        s.nvec = nvec;
        s.in_mode = IN_DENSE;
        s.in = Gin;
        s.in_vstride = n;
        s.in_rstride = Q.n2;
        s.rows_in = Q.n1;
        s.row_len = Q.n2;
        s.out_mode = OUT_GRID;
        s.out = Gout;
        s.out_vstride = n;
        s.rows_out = Q.n1;
        s.cols_out = Q.n2;
        s.scale = 1.0;
        s.lam = lam;
        s.lam_tstride = lam_tstride;
        s.vecs_per_theta = vpt;
        s.active = active;
        conv_apply<R>(Q, s, st);
        irr_gather<R, R>(Q, Gout, nvec, y, x, d_eta, vpt, active, st);
    };
}
template MatvecFn<double> irregular_op<double>(Problem&, const void*, int64_t, int, const double*);
template MatvecFn<float> irregular_op<float>(Problem&, const void*, int64_t, int, const double*);

void irr_cross_corr(const Problem& P, const double* lag, const int64_t* targets, int nt, double* out,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_irr_cross_corr, vgrid(P.p, nt), dim3(256), 0, st, lag, P.N1, P.N2, P.a_cell.as<int32_t>(),
                       P.a_w.as<double>(), P.p, P.n2, targets, out);
    KRY_HIP(hipGetLastError());
}

void irr_boot_obs(const Problem& P, const double* fields, int B, double tau, uint64_t seed, double* yb,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_irr_boot_obs, vgrid(P.p, B), dim3(256), 0, st, fields, (int64_t)P.n1 * P.n2,
                       P.a_cell.as<int32_t>(), P.a_w.as<double>(), P.obs_user.as<int32_t>(), P.p, tau, seed, yb);
    KRY_HIP(hipGetLastError());
}

template <typename R>
void irr_permute(const Problem& P, const R* src, R* dst, int nvec, bool to_stored, hipStream_t st) {
    hipLaunchKernelGGL(k_irr_permute<R>, vgrid(P.p, nvec), dim3(256), 0, st, src, dst, P.obs_user.as<int32_t>(), P.p,
                       to_stored ? 1 : 0);
    KRY_HIP(hipGetLastError());
}
template void irr_permute<double>(const Problem&, const double*, double*, int, bool, hipStream_t);
template void irr_permute<float>(const Problem&, const float*, float*, int, bool, hipStream_t);

}  // namespace kry
