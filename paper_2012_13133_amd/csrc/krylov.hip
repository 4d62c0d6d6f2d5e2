// Batched Krylov building blocks: deterministic dot products, the Lanczos
// recurrence, Gauss quadrature of the Lanczos tridiagonals and conjugate
// gradients, all with scalars kept on the device so the host loop never waits
// on the GPU inside an iteration.
//
// Reductions are fixed-order trees: block b of vector v always sums the same
// elements in the same order, and the per-block partials are summed by one
// block in a fixed order.  The result for a vector therefore does not depend
// on which other vectors share the launch.  Accumulation is FP64 for both
// element types.
#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "krylov.hpp"

namespace kry {

constexpr int RB = 256;  // threads per reduction block

int dot_blocks(int64_t n) {
    int64_t b = (n + 8 * RB - 1) / (8 * RB);
    if (b < 1) b = 1;
    if (b > 256) b = 256;
    return (int)b;
}

// Sum over a 64-lane wavefront by shifts of 32, 16, ..., 1 lanes; lane 0
// holds the result, always added in the same order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a block of RB threads: wavefront sums, then the RB / 64 of them
// in wavefront order (two barriers; the second lets callers reuse sh).
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < RB / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// partial[v * nblk + b] = sum over block b's elements of a_v . b_v
template <typename R>
__global__ void __launch_bounds__(RB) k_dot_partial(const R* __restrict__ a, int64_t sa, const R* __restrict__ b,
                                                    int64_t sb, int64_t n, double* __restrict__ partial) {
    __shared__ double sh[RB];
    const int nblk = gridDim.x, vec = blockIdx.y;
    const R* av = a + vec * sa;
    const R* bv = b + vec * sb;
    double acc = 0.0;
#pragma unroll 8  // several loads in flight per thread
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)nblk * RB)
        acc += (double)av[i] * (double)bv[i];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[vec * nblk + blockIdx.x] = acc;
}

// out[v * ostride] = sum_b partial[v * nblk + b]
__global__ void __launch_bounds__(RB) k_reduce(const double* __restrict__ partial, int nblk,
                                               double* __restrict__ out, int64_t ostride) {
    __shared__ double sh[RB];
    const int vec = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RB) acc += partial[vec * nblk + i];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[vec * ostride] = acc;
}

template <typename R>
void dot_batched(const R* a, int64_t sa, const R* b, int64_t sb, int64_t n, int nvec, double* partial,
                 double* out, hipStream_t st) {
    const int nblk = dot_blocks(n);
    hipLaunchKernelGGL(k_dot_partial<R>, dim3(nblk, nvec), dim3(RB), 0, st, a, sa, b, sb, n, partial);
    KRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(nvec), dim3(RB), 0, st, partial, nblk, out, (int64_t)1);
    KRY_HIP(hipGetLastError());
}
template void dot_batched<double>(const double*, int64_t, const double*, int64_t, int64_t, int, double*, double*,
                                  hipStream_t);
template void dot_batched<float>(const float*, int64_t, const float*, int64_t, int64_t, int, double*, double*,
                                 hipStream_t);

// ---- element-wise helpers -----------------------------------------------------
template <typename R>
__global__ void k_scale_vec(const R* __restrict__ x, const double* __restrict__ s, R* __restrict__ y, int64_t n) {
    const int vec = blockIdx.y;
    const R f = (R)s[vec];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[vec * n + i] = x[vec * n + i] * f;
}

template <typename A, typename B>
__global__ void k_convert(const A* __restrict__ x, B* __restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (B)x[i];
}

static dim3 vec_grid(int64_t n, int nvec) {
    int64_t b = (n + 255) / 256;
    if (b > 1024) b = 1024;
    return dim3((unsigned)b, nvec);
}

template <typename A, typename B>
void convert(const A* x, B* y, int64_t n, hipStream_t st) {
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    hipLaunchKernelGGL((k_convert<A, B>), dim3((unsigned)b), dim3(256), 0, st, x, y, n);
    KRY_HIP(hipGetLastError());
}
template void convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void convert<float, double>(const float*, double*, int64_t, hipStream_t);
template void convert<double, double>(const double*, double*, int64_t, hipStream_t);

// ---- probes -----------------------------------------------------------------
// Rademacher sign of (compact index, probe); coloured probes keep the sign
// only on cells of colour k = (row mod c) + c (col mod c).
template <typename R>
__global__ void k_probes(const int32_t* __restrict__ cell, const int32_t* __restrict__ user, int64_t p, int n2,
                         int nprobe, uint64_t seed, int period, R* __restrict__ out, int64_t stride) {
    const int k = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x) {
        // the Philox index is the caller's observation index
        double v = rademacher((uint32_t)(user ? user[i] : i), (uint32_t)k, seed);
        if (period > 0) {
            const int c = cell[i];
            const int row = c / n2, col = c - (c / n2) * n2;
            const int colour = (row % period) + period * (col % period);
            if (colour != k) v = 0.0;
        }
        out[k * stride + i] = (R)v;
    }
}

template <typename R>
void make_probes(const Problem& P, int nprobe, uint64_t seed, int period, R* out, hipStream_t st, int64_t stride) {
    hipLaunchKernelGGL(k_probes<R>, vec_grid(P.p, nprobe), dim3(256), 0, st, P.cell.as<int32_t>(),
                       P.irregular ? P.obs_user.as<int32_t>() : nullptr, P.p, P.n2, nprobe, seed, period, out,
                       stride > 0 ? stride : P.p);
    KRY_HIP(hipGetLastError());
}
template void make_probes<double>(const Problem&, int, uint64_t, int, double*, hipStream_t, int64_t);
template void make_probes<float>(const Problem&, int, uint64_t, int, float*, hipStream_t, int64_t);

// ---- Lanczos ----------------------------------------------------------------------
// start: znorm2 known -> scale = 1/||z|| (0 for an all-zero probe)
__global__ void k_lanczos_init(const double* __restrict__ znorm2, double* __restrict__ scale,
                               int* __restrict__ active, int* __restrict__ steps, int nvec) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvec) return;
    const double z2 = znorm2[v];
    active[v] = z2 > 0.0;
    steps[v] = 0;
    scale[v] = z2 > 0.0 ? 1.0 / sqrt(z2) : 0.0;
}

// r = w - alpha_j q_j - beta_{j-1} q_{j-1} (in place in w); partial ||r||^2 if requested
template <typename R>
__global__ void __launch_bounds__(RB) k_lanczos_update(R* __restrict__ w, const R* __restrict__ q,
                                                       const R* __restrict__ qprev, const double* __restrict__ alpha,
                                                       const double* __restrict__ beta_prev, int64_t n,
                                                       double* __restrict__ partial) {
    __shared__ double sh[RB];
    const int nblk = gridDim.x, vec = blockIdx.y;
    const R a = (R)alpha[vec];
    const R b = beta_prev ? (R)beta_prev[vec] : (R)0;
    R* wv = w + vec * n;
    const R* qv = q + vec * n;
    const R* pv = qprev ? qprev + vec * n : nullptr;
    double acc = 0.0;
#pragma unroll 8
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)nblk * RB) {
        R r = wv[i] - a * qv[i];
        if (pv) r -= b * pv[i];
        wv[i] = r;
        acc += (double)r * (double)r;
    }
    if (partial) {
        acc = block_sum(acc, sh);
        if (threadIdx.x == 0) partial[vec * nblk + blockIdx.x] = acc;
    }
}

// beta_j = ||r||, breakdown test against the oracle's rule
// (beta <= tol * max(|alpha_j|, beta_{j-1})), step counts and 1/beta.
__global__ void __launch_bounds__(RB) k_lanczos_beta(const double* __restrict__ partial, int nblk, int j,
                                                     const double* __restrict__ alpha_j,
                                                     const double* __restrict__ beta_prev, double* __restrict__ beta_j,
                                                     double* __restrict__ scale, int* __restrict__ active,
                                                     int* __restrict__ steps, double tol) {
    __shared__ double sh[RB];
    const int vec = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RB) acc += partial[vec * nblk + i];
    acc = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    const double b = sqrt(acc);
    if (!active[vec]) {
        beta_j[vec] = 0.0;
        scale[vec] = 0.0;
        return;
    }
    steps[vec] = j + 1;
    const double bp = beta_prev ? beta_prev[vec] : 0.0;
    const double ref = fmax(fmax(fabs(alpha_j[vec]), bp), 1e-300);
    if (b <= tol * ref) {
        active[vec] = 0;
        beta_j[vec] = 0.0;
        scale[vec] = 0.0;
    } else {
        beta_j[vec] = b;
        scale[vec] = 1.0 / b;
    }
}

// NB dot products against one sweep of r: acc[k] += q_k[i] r[i] over the
// block's elements, each in the order a single dot product takes them.  The
// vector bases are uniform over the block; lanes add 32-bit byte offsets.
template <typename R, int NB>
__device__ __forceinline__ void multidot_sweep(const R* __restrict__ qv, int64_t qslot, const R* __restrict__ rv,
                                               uint32_t n, double* acc) {
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[k] = 0.0;
    const uint32_t step = gridDim.x * RB;
#pragma unroll 2
    for (uint32_t i = blockIdx.x * RB + threadIdx.x; i < n; i += step) {
        const double x = (double)at32(rv, i);
#pragma unroll
        for (int k = 0; k < NB; ++k) acc[k] += (double)at32(qv + k * qslot, i) * x;
    }
}

// Classical Gram-Schmidt against stored basis vectors: h[v][i] = q_i . r.
// Basis vectors go MDB at a time through one sweep of r (more loads in
// flight, one pair of barriers per group); every partial is the same sum, in
// the same order, as a block_sum of one dot product.  n * sizeof(R) < 2^32.
constexpr int MDB = 8;
template <typename R>
__global__ void __launch_bounds__(RB) k_multidot_partial(const R* __restrict__ Q, int64_t qslot, const R* __restrict__ r,
                                                         int nq, int64_t n, double* __restrict__ partial) {
    __shared__ double sh[MDB][RB / 64];
    const int nblk = gridDim.x, vec = blockIdx.y;
    const R* rv = r + vec * n;
    const R* qb = Q + vec * n;
    for (int q0 = 0; q0 < nq; q0 += MDB) {
        const int nb = min(MDB, nq - q0);
        const R* qv = qb + q0 * qslot;
        double acc[MDB] = {};
        switch (nb) {
            case 1: multidot_sweep<R, 1>(qv, qslot, rv, (uint32_t)n, acc); break;
            case 2: multidot_sweep<R, 2>(qv, qslot, rv, (uint32_t)n, acc); break;
            case 3: multidot_sweep<R, 3>(qv, qslot, rv, (uint32_t)n, acc); break;
            case 4: multidot_sweep<R, 4>(qv, qslot, rv, (uint32_t)n, acc); break;
            case 5: multidot_sweep<R, 5>(qv, qslot, rv, (uint32_t)n, acc); break;
            case 6: multidot_sweep<R, 6>(qv, qslot, rv, (uint32_t)n, acc); break;
            case 7: multidot_sweep<R, 7>(qv, qslot, rv, (uint32_t)n, acc); break;
            default: multidot_sweep<R, MDB>(qv, qslot, rv, (uint32_t)n, acc); break;
        }
#pragma unroll
        for (int k = 0; k < MDB; ++k) {
            if (k >= nb) break;
            const double v = wave_sum(acc[k]);
            if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x < nb) {
            double s = sh[threadIdx.x][0];
#pragma unroll
            for (int w = 1; w < RB / 64; ++w) s += sh[threadIdx.x][w];
            partial[((int64_t)vec * nq + q0 + threadIdx.x) * nblk + blockIdx.x] = s;
        }
        __syncthreads();
    }
}

// The first pass's update and the second pass's dots of CGS2 in one sweep of
// the basis: r <- r - sum_k h_k q_k element by element as k_multi_axpy forms
// it, then the partials of q_k . r as k_multidot_partial forms them (same
// block partition, same order), from the basis values already in registers.
// Slots past nq are loaded from slot nq - 1 (in range) and not used.
// nq <= NQ; n * sizeof(R) < 2^32; grid (dot_blocks(n), vectors).
template <typename R, int NQ>
__global__ void __launch_bounds__(RB) k_reorth_axpy_dot(const R* __restrict__ Q, int64_t qslot,
                                                        const double* __restrict__ h, int nq, R* __restrict__ r,
                                                        int64_t n, double* __restrict__ partial) {
    __shared__ double sh[NQ][RB / 64];
    const int nblk = gridDim.x, vec = blockIdx.y;
    const double* hv = h + (int64_t)vec * nq;
    R* rv = r + vec * n;
    const R* qb = Q + vec * n;
    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) acc[k] = 0.0;
    const uint32_t n32 = (uint32_t)n, step = nblk * RB;
    for (uint32_t i = blockIdx.x * RB + threadIdx.x; i < n32; i += step) {
        R qv[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) qv[k] = at32(qb + min(k, nq - 1) * qslot, i);
        double a = (double)at32(rv, i);
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            if (k < nq) a -= hv[k] * (double)qv[k];
        const R wn = (R)a;
        at32(rv, i) = wn;
        const double x = (double)wn;
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            if (k < nq) acc[k] += (double)qv[k] * x;
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        if (k < nq) {
            const double v = wave_sum(acc[k]);
            if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nq) {
        double s = sh[threadIdx.x][0];
#pragma unroll
        for (int w = 1; w < RB / 64; ++w) s += sh[threadIdx.x][w];
        partial[((int64_t)vec * nq + threadIdx.x) * nblk + blockIdx.x] = s;
    }
}

template <typename R, int NQ>
void launch_axpy_dot(dim3 grid, hipStream_t st, const R* Q, int64_t qslot, const double* h, int nq, R* r, int64_t n,
                     double* partial) {
    hipLaunchKernelGGL((k_reorth_axpy_dot<R, NQ>), grid, dim3(RB), 0, st, Q, qslot, h, nq, r, n, partial);
}

// launches k_reorth_axpy_dot for nq basis vectors (the smallest NQ, a
// multiple of 8, that holds them); false where nq is above the largest
// instantiation (64 FP32, 32 FP64 basis vectors)
template <typename R>
bool reorth_axpy_dot(const R* Q, int64_t qslot, const double* h, int nq, R* r, int64_t n, int nvec,
                     double* partial, hipStream_t st) {
    constexpr int cap = sizeof(R) == 4 ? 64 : 32;
    if (nq < 1 || nq > cap) return false;
    const dim3 grid(dot_blocks(n), nvec);
    switch ((nq + 7) / 8) {
        case 1: launch_axpy_dot<R, 8>(grid, st, Q, qslot, h, nq, r, n, partial); break;
        case 2: launch_axpy_dot<R, 16>(grid, st, Q, qslot, h, nq, r, n, partial); break;
        case 3: launch_axpy_dot<R, 24>(grid, st, Q, qslot, h, nq, r, n, partial); break;
        case 4: launch_axpy_dot<R, 32>(grid, st, Q, qslot, h, nq, r, n, partial); break;
        default:
            if constexpr (cap > 32) {
                switch ((nq + 7) / 8) {
                    case 5: launch_axpy_dot<R, 40>(grid, st, Q, qslot, h, nq, r, n, partial); break;
                    case 6: launch_axpy_dot<R, 48>(grid, st, Q, qslot, h, nq, r, n, partial); break;
                    case 7: launch_axpy_dot<R, 56>(grid, st, Q, qslot, h, nq, r, n, partial); break;
                    default: launch_axpy_dot<R, 64>(grid, st, Q, qslot, h, nq, r, n, partial); break;
                }
            }
            break;
    }
    KRY_HIP(hipGetLastError());
    return true;
}

// r -= sum_i h_i q_i (subtracted in order of i; loads issued eight at a time)
template <typename R>
__global__ void k_multi_axpy(const R* __restrict__ Q, int64_t qslot, const double* __restrict__ h, int nq,
                             R* __restrict__ r, int64_t n) {
    const int vec = blockIdx.y;
    const double* hv = h + (int64_t)vec * nq;
    const R* qb = Q + vec * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = (double)r[vec * n + i];
        int q = 0;
        for (; q + 8 <= nq; q += 8) {
            R qv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) qv[k] = qb[(int64_t)(q + k) * qslot + i];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc -= hv[q + k] * (double)qv[k];
        }
        for (; q < nq; ++q) acc -= hv[q] * (double)qb[(int64_t)q * qslot + i];
        r[vec * n + i] = (R)acc;
    }
}

// Points whose outputs all settled since the last check record the step and
// their values; done = every point settled.  One block, fixed order.
__global__ void k_lanczos_settle(const double* __restrict__ g_cur, const double* __restrict__ g_prev,
                                 double* __restrict__ g_final, int* __restrict__ stop, int nout, int per_point,
                                 double rtol, int step, int* __restrict__ done) {
    const int npoints = nout / per_point;
    for (int pt = threadIdx.x; pt < npoints; pt += blockDim.x) {
        if (stop[pt]) continue;
        bool settled = true;
        for (int o = pt * per_point; o < (pt + 1) * per_point; ++o)
            settled = settled && fabs(g_cur[o] - g_prev[o]) <= rtol * fabs(g_cur[o]);
        if (!settled) continue;
        stop[pt] = step;
        for (int o = pt * per_point; o < (pt + 1) * per_point; ++o) g_final[o] = g_cur[o];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int all = 1;
        for (int pt = 0; pt < npoints; ++pt) all = all && stop[pt] != 0;
        done[0] = all;
    }
}

template <typename R>
void lanczos_run(const MatvecFn<R>& A, int64_t n, int nvec, int m, bool reorth, const R* Z, LanczosBuffers<R>& B,
                 hipStream_t st, const LanczosAdaptive* ad) {
    const int nblk = dot_blocks(n);
    KRY_REQUIRE(!reorth || (uint64_t)n * sizeof(R) < (uint64_t(1) << 32), "vectors too long for reorthogonalisation");
    const double tol = sizeof(R) == 8 ? 1e-12 : 1e-6;
    const int64_t slot = (int64_t)nvec * n;
    const int nslots = reorth ? m + 1 : 3;
    auto Qs = [&](int j) { return B.Q + (int64_t)(reorth ? j : j % 3) * slot; };

    dot_batched<R>(Z, n, Z, n, n, nvec, B.partial, B.znorm2, st);
    hipLaunchKernelGGL(k_lanczos_init, dim3((nvec + 63) / 64), dim3(64), 0, st, B.znorm2, B.scale, B.active, B.steps,
                       nvec);
    KRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scale_vec<R>, vec_grid(n, nvec), dim3(256), 0, st, Z, B.scale, Qs(0), n);
    KRY_HIP(hipGetLastError());
    (void)nslots;
    double *g_prev = nullptr, *g_cur = nullptr;
    // checks after steps 5, 10, ..., 100, 110, ..., 150, 165, ...: every
    // 5 max(1, floor(j / 50)) steps, so that the quadratures, each O(j^2),
    // cost O(m^2) in all rather than O(m^3)
    int next_check = 5;
    if (ad) {
        KRY_HIP(hipMemsetAsync(ad->stop, 0, (ad->nout / ad->per_point) * sizeof(int), st));
        g_prev = ad->g_prev;
        g_cur = ad->g_cur;
    }
    for (int j = 0; j < m; ++j) {
        R* q = Qs(j);
        const R* qp = j > 0 ? Qs(j - 1) : nullptr;
        double* aj = B.alpha + (int64_t)j * nvec;
        double* bj = B.beta + (int64_t)j * nvec;
        const double* bprev = j > 0 ? B.beta + (int64_t)(j - 1) * nvec : nullptr;
        A(q, B.W, nvec, st, nullptr);
        dot_batched<R>(q, n, B.W, n, n, nvec, B.partial, aj, st);
        if (!reorth) {
            hipLaunchKernelGGL(k_lanczos_update<R>, dim3(nblk, nvec), dim3(RB), 0, st, B.W, q, qp, aj, bprev, n,
                               B.partial);
            KRY_HIP(hipGetLastError());
        } else {
            hipLaunchKernelGGL(k_lanczos_update<R>, dim3(nblk, nvec), dim3(RB), 0, st, B.W, q, qp, aj, bprev, n,
                               (double*)nullptr);
            KRY_HIP(hipGetLastError());
            // two classical Gram-Schmidt passes; where the basis fits one
            // fused sweep, the first update and the second pass's dots share it
            const int nq = j + 1;
            auto dots = [&] {
                hipLaunchKernelGGL(k_multidot_partial<R>, dim3(nblk, nvec), dim3(RB), 0, st, B.Q, slot, B.W, nq, n,
                                   B.partial);
                KRY_HIP(hipGetLastError());
            };
            auto coeffs = [&] {
                hipLaunchKernelGGL(k_reduce, dim3(nvec * nq), dim3(RB), 0, st, B.partial, nblk, B.h, (int64_t)1);
                KRY_HIP(hipGetLastError());
            };
            auto update = [&] {
                hipLaunchKernelGGL(k_multi_axpy<R>, vec_grid(n, nvec), dim3(256), 0, st, B.Q, slot, B.h, nq, B.W, n);
                KRY_HIP(hipGetLastError());
            };
            dots();
            coeffs();
            if (!reorth_axpy_dot<R>(B.Q, slot, B.h, nq, B.W, n, nvec, B.partial, st)) {
                update();
                dots();
            }
            coeffs();
            update();
            hipLaunchKernelGGL(k_dot_partial<R>, dim3(nblk, nvec), dim3(RB), 0, st, B.W, n, B.W, n, n, B.partial);
            KRY_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_lanczos_beta, dim3(nvec), dim3(RB), 0, st, B.partial, nblk, j, aj, bprev, bj, B.scale,
                           B.active, B.steps, tol);
        KRY_HIP(hipGetLastError());
        if (ad && j + 1 == next_check) {
            next_check += 5 * std::max(1, (j + 1) / 50);
            quadrature(B.alpha, B.beta, B.steps, B.znorm2, ad->nout, nvec, g_cur, st, ad->src, ad->shift);
            if (j + 1 >= 10) {
                hipLaunchKernelGGL(k_lanczos_settle, dim3(1), dim3(256), 0, st, g_cur, g_prev, ad->g_final, ad->stop,
                                   ad->nout, ad->per_point, ad->rtol, j + 1, ad->done);
                KRY_HIP(hipGetLastError());
                int done = 0;
                KRY_HIP(hipMemcpyAsync(&done, ad->done, sizeof(int), hipMemcpyDeviceToHost, st));
                KRY_HIP(hipStreamSynchronize(st));
                if (done) break;
            }
            std::swap(g_prev, g_cur);
        }
        if (j + 1 < m) {
            hipLaunchKernelGGL(k_scale_vec<R>, vec_grid(n, nvec), dim3(256), 0, st, B.W, B.scale, Qs(j + 1), n);
            KRY_HIP(hipGetLastError());
        }
    }
}
template void lanczos_run<double>(const MatvecFn<double>&, int64_t, int, int, bool, const double*,
                                  LanczosBuffers<double>&, hipStream_t, const LanczosAdaptive*);
template void lanczos_run<float>(const MatvecFn<float>&, int64_t, int, int, bool, const float*,
                                 LanczosBuffers<float>&, hipStream_t, const LanczosAdaptive*);

// ---- Gauss quadrature ---------------------------------------------------------------
// For each probe: eigen-decomposition of its Lanczos tridiagonal T (steps
// s <= m) by the implicit QL iteration with Wilkinson shifts (Bowdler,
// Martin, Reinsch & Wilkinson, 1968), tracking only the first component of
// every eigenvector (Golub & Welsch, 1969); then
//   gamma = ||z||^2 sum_i tau_i^2 log theta_i.
// Output v reads the tridiagonal of recurrence src[v] (v itself when src is
// NULL) shifted by shift[v] (none when NULL): T + shift I has the same
// eigenvectors and eigenvalues moved by the shift.
__global__ void k_quadrature(const double* __restrict__ alpha, const double* __restrict__ beta,
                             const int* __restrict__ steps, const double* __restrict__ znorm2, int nvec,
                             int64_t coef_stride /* distance between steps j and j+1 */, double* __restrict__ gamma,
                             const int* __restrict__ src, const double* __restrict__ shift) {
    // One output per workgroup; its first lane runs the (serial) QL sweeps
    // on the tridiagonal held in LDS: 24 KB at the step cap, where arrays in
    // private memory would ask the runtime for 24 KB of scratch per lane.
    __shared__ double d[KRY_MAX_LANCZOS], e[KRY_MAX_LANCZOS], z[KRY_MAX_LANCZOS];
    const int v = blockIdx.x;
    if (v >= nvec || threadIdx.x != 0) return;
    const int u = src ? src[v] : v;
    const double sh = shift ? shift[v] : 0.0;
    const int n = steps[u];
    if (n <= 0) {
        gamma[v] = 0.0;
        return;
    }
    for (int i = 0; i < n; ++i) {
        d[i] = alpha[i * coef_stride + u] + sh;
        e[i] = (i + 1 < n) ? beta[i * coef_stride + u] : 0.0;
        z[i] = (i == 0) ? 1.0 : 0.0;
    }
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 100; ++iter) {
            int mm = l;
            for (; mm < n - 1; ++mm) {
                const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
                if (fabs(e[mm]) <= eps * dd) break;
            }
            if (mm == l) break;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[mm] - d[l] + e[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            for (int i = mm - 1; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[mm] = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                const double zf = z[i + 1];
                z[i + 1] = s * z[i] + c * zf;
                z[i] = c * z[i] - s * zf;
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[mm] = 0.0;
        }
    }
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += z[i] * z[i] * log(d[i]);
    gamma[v] = znorm2[u] * acc;
}

void quadrature(const double* alpha, const double* beta, const int* steps, const double* znorm2, int nvec,
                int64_t coef_stride, double* gamma, hipStream_t st, const int* src, const double* shift) {
    if (nvec <= 0) return;
    hipLaunchKernelGGL(k_quadrature, dim3(nvec), dim3(64), 0, st, alpha, beta, steps, znorm2, nvec, coef_stride,
                       gamma, src, shift);
    KRY_HIP(hipGetLastError());
}

// ---- conjugate gradients ---------------------------------------------------------------
__global__ void k_cg_init(const double* __restrict__ rr, double* __restrict__ bnorm2, double* __restrict__ rr_state,
                          int* __restrict__ active, int* __restrict__ iters, const int* __restrict__ limit, int nvec) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvec) return;
    bnorm2[v] = rr[v];
    rr_state[v] = rr[v];
    active[v] = rr[v] > 0.0 && limit[v] > 0;
    iters[v] = 0;
}

// a = rr / (p . w); x += a p; r -= a w; partial r . r
template <typename R>
__global__ void __launch_bounds__(RB) k_cg_xr(R* __restrict__ x, R* __restrict__ r, const R* __restrict__ p,
                                              const R* __restrict__ w, const double* __restrict__ rr,
                                              const double* __restrict__ pw, const int* __restrict__ active, int64_t n,
                                              double* __restrict__ partial) {
    __shared__ double sh[RB];
    const int nblk = gridDim.x, vec = blockIdx.y;
    const bool on = active[vec] != 0;
    const double a = on ? rr[vec] / pw[vec] : 0.0;
    const R ar = (R)a;
    double acc = 0.0;
#pragma unroll 8
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)nblk * RB) {
        const int64_t k = vec * n + i;
        R ri = r[k];
        if (on) {
            x[k] += ar * p[k];
            ri -= ar * w[k];
            r[k] = ri;
        }
        acc += (double)ri * (double)ri;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[vec * nblk + blockIdx.x] = acc;
}

__global__ void __launch_bounds__(RB) k_cg_finish(const double* __restrict__ partial, int nblk,
                                                  double* __restrict__ rr, const double* __restrict__ bnorm2,
                                                  double* __restrict__ beta, int* __restrict__ active,
                                                  int* __restrict__ iters, const int* __restrict__ limit, double rtol) {
    __shared__ double sh[RB];
    const int vec = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RB) acc += partial[vec * nblk + i];
    acc = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    if (!active[vec]) {
        beta[vec] = 0.0;
        return;
    }
    beta[vec] = acc / rr[vec];
    rr[vec] = acc;
    iters[vec] += 1;
    if (!(sqrt(acc) > rtol * sqrt(bnorm2[vec])) || iters[vec] >= limit[vec]) active[vec] = 0;
}

template <typename R>
__global__ void k_cg_p(R* __restrict__ p, const R* __restrict__ r, const double* __restrict__ beta,
                       const int* __restrict__ active, int64_t n) {
    const int vec = blockIdx.y;
    if (!active[vec]) return;
    const R b = (R)beta[vec];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[vec * n + i] = r[vec * n + i] + b * p[vec * n + i];
}

// A block of stream work captured once into a HIP graph and replayed; the
// graph holds kernel launches only (no memset or copy nodes).
struct GraphBlock {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    template <typename F>
    void run(hipStream_t st, F&& body) {
        if (!exec) {
            KRY_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            try {
                body();
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(st, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            KRY_HIP(hipStreamEndCapture(st, &graph));
            KRY_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        }
        KRY_HIP(hipGraphLaunch(exec, st));
    }
    ~GraphBlock() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

template <typename R>
void cg_run(const MatvecFn<R>& A, int64_t n, int nvec, const R* b, R* x, double rtol, int maxit, CgBuffers<R>& B,
            std::vector<int>& iters, std::vector<double>& relres, hipStream_t st, const std::vector<int>* limits,
            bool graphs) {
    const int nblk = dot_blocks(n);
    std::vector<int> lim(nvec, maxit);
    if (limits) {
        for (int v = 0; v < nvec; ++v) lim[v] = std::min(maxit, (*limits)[v]);
    }
    int loop_max = 0;
    for (int v = 0; v < nvec; ++v) loop_max = std::max(loop_max, lim[v]);
    KRY_HIP(hipMemcpyAsync(B.limit, lim.data(), nvec * sizeof(int), hipMemcpyHostToDevice, st));
    const size_t vbytes = (size_t)nvec * n * sizeof(R);
    KRY_HIP(hipMemsetAsync(x, 0, vbytes, st));
    KRY_HIP(hipMemcpyAsync(B.r, b, vbytes, hipMemcpyDeviceToDevice, st));
    KRY_HIP(hipMemcpyAsync(B.p, b, vbytes, hipMemcpyDeviceToDevice, st));
    dot_batched<R>(b, n, b, n, n, nvec, B.partial, B.tmp, st);
    hipLaunchKernelGGL(k_cg_init, dim3((nvec + 63) / 64), dim3(64), 0, st, B.tmp, B.bnorm2, B.rr, B.active, B.iters,
                       B.limit, nvec);
    KRY_HIP(hipGetLastError());
    std::vector<int> act(nvec);
    const int check = 16;
    auto step = [&]() {
        A(B.p, B.w, nvec, st, B.active);
        dot_batched<R>(B.p, n, B.w, n, n, nvec, B.partial, B.pw, st);
        hipLaunchKernelGGL(k_cg_xr<R>, dim3(nblk, nvec), dim3(RB), 0, st, x, B.r, B.p, B.w, B.rr, B.pw, B.active, n,
                           B.partial);
        KRY_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_cg_finish, dim3(nvec), dim3(RB), 0, st, B.partial, nblk, B.rr, B.bnorm2, B.beta, B.active,
                           B.iters, B.limit, rtol);
        KRY_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_cg_p<R>, vec_grid(n, nvec), dim3(256), 0, st, B.p, B.r, B.beta, B.active, n);
        KRY_HIP(hipGetLastError());
    };
    // Iterations go in blocks of `check` between convergence reads.  The
    // first block runs eagerly (it also sizes every workspace the product
    // allocates); with graphs on, later full blocks replay one captured
    // graph of `check` iterations (same kernels, same arguments).
    GraphBlock gb;
    for (int it = 0; it < loop_max;) {
        const int blk = std::min(check, loop_max - it);
        if (graphs && it > 0 && blk == check) gb.run(st, [&] {
            for (int k = 0; k < check; ++k) step();
        });
        else
            for (int k = 0; k < blk; ++k) step();
        it += blk;
        KRY_HIP(hipMemcpyAsync(act.data(), B.active, nvec * sizeof(int), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        bool any = false;
        for (int v = 0; v < nvec; ++v) any = any || act[v];
        if (!any) break;
    }
    std::vector<double> rr(nvec), bn(nvec);
    iters.resize(nvec);
    relres.resize(nvec);
    KRY_HIP(hipMemcpyAsync(iters.data(), B.iters, nvec * sizeof(int), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipMemcpyAsync(rr.data(), B.rr, nvec * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipMemcpyAsync(bn.data(), B.bnorm2, nvec * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
    for (int v = 0; v < nvec; ++v) relres[v] = bn[v] > 0 ? std::sqrt(rr[v] / bn[v]) : 0.0;
}
template void cg_run<double>(const MatvecFn<double>&, int64_t, int, const double*, double*, double, int,
                             CgBuffers<double>&, std::vector<int>&, std::vector<double>&, hipStream_t,
                             const std::vector<int>*, bool);
template void cg_run<float>(const MatvecFn<float>&, int64_t, int, const float*, float*, double, int, CgBuffers<float>&,
                            std::vector<int>&, std::vector<double>&, hipStream_t, const std::vector<int>*, bool);

// ---- multi-shift conjugate gradients ---------------------------------------------------
// One CG recurrence per group on its base operator A; the shifted system
// (A + sigma I) x = b has, in the same Krylov space, the residual zeta r of the
// base residual r (Jegerlehner, hep-lat/9612014).  With the base's alpha_k,
// beta_k (alpha_{-1} = 1, beta_{-1} = 0, zeta_0 = zeta_{-1} = 1):
//   zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1} /
//                (alpha_k beta_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} alpha_{k-1} (1 + sigma alpha_k))
//   alpha^s_k = alpha_k zeta_{k+1} / zeta_k,    beta^s_k = beta_k (zeta_{k+1} / zeta_k)^2
//   x^s += alpha^s_k p^s,                       p^s = zeta_{k+1} r_{k+1} + beta^s_k p^s.
// Only Q^s = b . x^s is wanted, so the shifted vectors are never formed:
// with c_k = b . r_k and d^s = b . p^s,
//   Q^s += alpha^s_k d^s,                       d^s = zeta_{k+1} c_{k+1} + beta^s_k d^s,
// which leaves one base CG (vectors r, p, w) per group and scalars per shift.
// A shift stops once |zeta_{k+1}| ||r_{k+1}|| <= rtol ||b|| (or at its
// iteration cap); its values never depend on the other shifts or groups.

__global__ void k_ms_init(const double* __restrict__ gram, const int* __restrict__ rhs, int nd, int G, int S,
                          const int* __restrict__ pos, double* __restrict__ rr, double* __restrict__ bnorm2,
                          double* __restrict__ alpha_old, double* __restrict__ beta_old, double* __restrict__ beta,
                          double* __restrict__ zeta,
                          double* __restrict__ zeta_old, double* __restrict__ d, double* __restrict__ Q,
                          double* __restrict__ relres, int* __restrict__ active, int* __restrict__ iters,
                          const int* __restrict__ limit) {
    for (int q = threadIdx.x; q < G; q += blockDim.x) {
        const int a = rhs[q];
        const double b2 = gram[a * nd + a];
        rr[q] = b2;
        bnorm2[q] = b2;
        alpha_old[q] = 1.0;
        beta_old[q] = 0.0;
        beta[q] = 0.0;  // p_0 = r_0: a deferred direction update leaves it so
    }
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        const int a = rhs[pos[s]];
        const double b2 = gram[a * nd + a];
        zeta[s] = 1.0;
        zeta_old[s] = 1.0;
        for (int j = 0; j < nd; ++j) {  // p_0 = b: d_j = D_j^T b
            d[s * nd + j] = gram[a * nd + j];
            Q[s * nd + j] = 0.0;
        }
        relres[s] = b2 > 0.0 ? 1.0 : 0.0;
        active[s] = b2 > 0.0 && limit[s] > 0;
        iters[s] = 0;
    }
}

// out[row] for rows [0, nrows), one block of RB threads: the sums k_reduce
// forms (thread t adds partial t, then block_sum), in the same order.  Rows
// go sixteen at a time: their loads are in flight together and their
// wavefront sums are independent chains.  nblk <= RB.
__device__ __forceinline__ void reduce_rows_block(const double* __restrict__ partial, int nblk, int nrows,
                                                  double* __restrict__ out) {
    constexpr int RK = 16;
    __shared__ double sh[64][RB / 64];
    const int t = threadIdx.x;
    const int tc = min(t, nblk - 1);
    for (int r0 = 0; r0 < nrows; r0 += 64) {
        const int nr = min(64, nrows - r0);
        for (int k0 = 0; k0 < nr; k0 += RK) {
            // loads from clamped (in-range) addresses, issued unconditionally
            // so that they are in flight together; lanes past the row count
            // or the partial count then take 0
            double x[RK], v[RK];
#pragma unroll
            for (int k = 0; k < RK; ++k) x[k] = partial[(int64_t)(r0 + min(k0 + k, nr - 1)) * nblk + tc];
#pragma unroll
            for (int k = 0; k < RK; ++k) {
                double acc = 0.0;
                if (k0 + k < nr && t < nblk) acc += x[k];
                v[k] = acc;
            }
#pragma unroll
            for (int k = 0; k < RK; ++k) v[k] = wave_sum(v[k]);
            if ((t & 63) == 0) {
#pragma unroll
                for (int k = 0; k < RK; ++k)
                    if (k0 + k < nr) sh[k0 + k][t >> 6] = v[k];
            }
        }
        __syncthreads();
        if (t < nr) {
            double r = sh[t][0];
#pragma unroll
            for (int w = 1; w < RB / 64; ++w) r += sh[t][w];
            out[r0 + t] = r;
        }
        __syncthreads();
    }
}

// Base alpha per active position from p_q . w_q (published by the residual
// kernel), then zeta_{k+1} and alpha^s of the listed shifts.  One block of RB
// threads.
__device__ __forceinline__ void ms_alpha_step(int Gact, const double* __restrict__ rr, const double* __restrict__ pw,
                                              double* __restrict__ alpha, const double* __restrict__ alpha_old,
                                              const double* __restrict__ beta_old, const int* __restrict__ list,
                                              int nlist, const int* __restrict__ pos,
                                              const double* __restrict__ sigma, const double* __restrict__ zeta,
                                              const double* __restrict__ zeta_old, double* __restrict__ zeta_new,
                                              double* __restrict__ alpha_s, int* __restrict__ active) {
    for (int q = threadIdx.x; q < Gact; q += blockDim.x) alpha[q] = pw[q] > 0.0 ? rr[q] / pw[q] : 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < nlist; i += blockDim.x) {
        const int s = list[i];
        if (!active[s]) continue;
        const int q = pos[s];
        const double z = zeta[s];
        if (!(pw[q] > 0.0) || !(fabs(z) > 0.0)) {  // breakdown of the base, or a vanished shifted residual
            active[s] = 0;
            continue;
        }
        const double a = alpha[q], ao = alpha_old[q], bo = beta_old[q], zo = zeta_old[s];
        const double den = a * bo * (zo - z) + zo * ao * (1.0 + sigma[s] * a);
        const double zn = z * zo * ao / den;
        zeta_new[s] = zn;
        alpha_s[s] = a * zn / z;
    }
}

// The scalars of an iteration, after the residual update: first the alpha
// step (from the p . w the residual kernel published), then base beta and
// roll of the position scalars; Q^s and d^s,
// beta^s, the stopping test and the zeta roll of the listed shifts.  rc gets,
// from the residual kernel's partials, ||r_{k+1}||^2 (rows 0..Gact-1) and
// D_j . r_{k+1} (row Gact + q nd + j).  One block of RB threads.
__device__ void ms_scalar_step(const MsScalarArgs& a) {
    ms_alpha_step(a.Gact, a.rr, a.pw, a.alpha, a.alpha_old, a.beta_old, a.list, a.nlist, a.pos, a.sigma, a.zeta,
                  a.zeta_old, a.zeta_new, a.alpha_s, a.active);
    __syncthreads();
    const int Gact = a.Gact, nd = a.nd;
    reduce_rows_block(a.partial, a.nblk, (1 + nd) * Gact, a.rc);
    for (int i = threadIdx.x; i < a.nlist; i += blockDim.x) {
        const int s = a.list[i];
        if (!a.active[s]) continue;
        const int q = a.pos[s];
        const double rn = a.rc[q];
        const double b = a.rr[q] > 0.0 ? rn / a.rr[q] : 0.0;
        const double z = a.zeta[s], zn = a.zeta_new[s];
        const double ratio = zn / z;
        const double bs = b * ratio * ratio;
        const double as = a.alpha_s[s];
        for (int j = 0; j < nd; ++j) {
            double& dj = a.d[s * nd + j];
            a.Q[s * nd + j] += as * dj;
            dj = zn * a.rc[Gact + q * nd + j] + bs * dj;
        }
        const int it = a.iters[s] + 1;
        a.iters[s] = it;
        const double res = fabs(zn) * sqrt(rn);
        const double bn = sqrt(a.bnorm2[q]);
        a.relres[s] = res / bn;
        if (!(res > a.rtol * bn) || it >= a.limit[s]) a.active[s] = 0;
        a.zeta_old[s] = z;
        a.zeta[s] = zn;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < Gact; q += blockDim.x) {
        const double b = a.rr[q] > 0.0 ? a.rc[q] / a.rr[q] : 0.0;
        a.beta[q] = b;
        a.alpha_old[q] = a.alpha[q];
        a.beta_old[q] = b;
        a.rr[q] = a.rc[q];
    }
}

// r_q -= alpha_q w_q, with alpha_q formed in every block from the npw
// partials of p_q . w_q (thread t adding partials t, t + RB, ... in order,
// then block_sum: the same value in every block, which block 0 publishes to
// pw for the scalar step); partials of ||r_q||^2 and D_j . r_q.  The scalar
// step is a one-block launch of its own: publishing the partials to a last
// block within this launch would take a device-scope release per block,
// which writes back the XCD's L2 and cost more than the launch it saves.
template <int ND>
__global__ void __launch_bounds__(RB) k_ms_r(double* __restrict__ r, const double* __restrict__ w,
                                             const double* __restrict__ D, const double* __restrict__ partial_pw,
                                             int npw, const double* __restrict__ rr, double* __restrict__ pw,
                                             int Gact, int64_t n, double* __restrict__ partial) {
    __shared__ double sh[RB];
    const int nblk = gridDim.x, q = blockIdx.y;
    double x = 0.0;
    {
        // in index order; eight loads in flight at a time
        const double* pp = partial_pw + (int64_t)q * npw;
        int i = threadIdx.x;
        for (; i + 7 * RB < npw; i += 8 * RB) {
            double a[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = pp[i + k * RB];
#pragma unroll
            for (int k = 0; k < 8; ++k) x += a[k];
        }
        for (; i < npw; i += RB) x += pp[i];
    }
    const double pwq = block_sum(x, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) pw[q] = pwq;
    const double al = pwq > 0.0 ? rr[q] / pwq : 0.0;
    double acc = 0.0, accb[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) accb[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)nblk * RB) {
        const int64_t k = q * n + i;
        const double ri = r[k] - al * w[k];
        r[k] = ri;
        acc += ri * ri;
#pragma unroll
        for (int j = 0; j < ND; ++j) accb[j] += D[j * n + i] * ri;
    }
    acc = block_sum(acc, sh);
#pragma unroll
    for (int j = 0; j < ND; ++j) accb[j] = block_sum(accb[j], sh);
    if (threadIdx.x == 0) {
        partial[q * nblk + blockIdx.x] = acc;
#pragma unroll
        for (int j = 0; j < ND; ++j) partial[(Gact + q * ND + j) * nblk + blockIdx.x] = accb[j];
    }
}

__global__ void __launch_bounds__(RB) k_ms_scalar(MsScalarArgs a) { ms_scalar_step(a); }

// Rows of the two reductions that the one-pass scalar step keeps in LDS.
constexpr int MS_ONE_ROWS = 1024;

// ms_scalar_step when every shift and every position has a thread of its own
// (S <= RB, Gact <= RB) and the (1 + nd) Gact reduction rows fit LDS.  The
// step is a chain of dependent reads, each costing a trip to memory from
// whichever XCD the block lands on; here every load is issued at the start
// (the shift and position state beside the partials), the position values
// reach the shift threads through LDS, and the step waits on memory about
// once.  Same sums, in the same order, and the same arithmetic as
// ms_scalar_step; every shift is visited (a shift missing from the list has
// stopped, and stays stopped).
__global__ void __launch_bounds__(RB) k_ms_scalar_one(MsScalarArgs a) {
    constexpr int RK = 32;  // reduction rows in flight together
    __shared__ double red[MS_ONE_ROWS];  // ||r||^2 rows, then D_j . r rows
    __shared__ double wsum[RK][RB / 64];
    __shared__ double s_pw[RB], s_alpha[RB], s_ao[RB], s_bo[RB], s_rr[RB], s_bn[RB];
    const int t = threadIdx.x, Gact = a.Gact, nd = a.nd, nblk = a.nblk;
    const int nrows = (1 + nd) * Gact;
    // shift t's state
    const int s = t < a.nS ? t : 0;
    const int act = t < a.nS ? a.active[s] : 0;
    const int q = a.pos[s], it0 = a.iters[s], lim = a.limit[s];
    const double z = a.zeta[s], zo = a.zeta_old[s], sg = a.sigma[s];
    double dj[KRY_MS_MAX_ND], Qj[KRY_MS_MAX_ND];
#pragma unroll
    for (int j = 0; j < KRY_MS_MAX_ND; ++j) {
        dj[j] = j < nd ? a.d[s * nd + j] : 0.0;
        Qj[j] = j < nd ? a.Q[s * nd + j] : 0.0;
    }
    // position t's state
    const int qt = t < Gact ? t : 0;
    const double rr_t = a.rr[qt], ao_t = a.alpha_old[qt], bo_t = a.beta_old[qt], bn_t = a.bnorm2[qt];
    const double pw_t = a.pw[qt];
    // the reductions, as reduce_rows_block forms them: thread t adds partial
    // t, wavefront sums, then the RB / 64 of them in wavefront order
    const int tc = min(t, nblk - 1);
    for (int r0 = 0; r0 < nrows; r0 += RK) {
        const int nr = min(RK, nrows - r0);
        double x[RK];
#pragma unroll
        for (int k = 0; k < RK; ++k) x[k] = a.partial[(int64_t)(r0 + min(k, nr - 1)) * nblk + tc];
#pragma unroll
        for (int k = 0; k < RK; ++k) {
            if (k < nr) {  // uniform over the block
                double acc = 0.0;
                if (t < nblk) acc += x[k];
                acc = wave_sum(acc);
                if ((t & 63) == 0) wsum[k][t >> 6] = acc;
            }
        }
        __syncthreads();
        if (t < nr) {
            double r = wsum[t][0];
#pragma unroll
            for (int w = 1; w < RB / 64; ++w) r += wsum[t][w];
            red[r0 + t] = r;
        }
        __syncthreads();
    }
    if (t < Gact) {
        s_pw[t] = pw_t;
        s_alpha[t] = pw_t > 0.0 ? rr_t / pw_t : 0.0;
        s_ao[t] = ao_t;
        s_bo[t] = bo_t;
        s_rr[t] = rr_t;
        s_bn[t] = bn_t;
    }
    __syncthreads();
    if (act) {
        if (!(s_pw[q] > 0.0) || !(fabs(z) > 0.0)) {  // breakdown of the base, or a vanished shifted residual
            a.active[s] = 0;
        } else {
            const double al = s_alpha[q], ao = s_ao[q], bo = s_bo[q];
            const double den = al * bo * (zo - z) + zo * ao * (1.0 + sg * al);
            const double zn = z * zo * ao / den;
            a.zeta_new[s] = zn;
            const double as = al * zn / z;
            a.alpha_s[s] = as;
            const double rn = red[q];
            const double rrq = s_rr[q];
            const double b = rrq > 0.0 ? rn / rrq : 0.0;
            const double ratio = zn / z;
            const double bs = b * ratio * ratio;
#pragma unroll
            for (int j = 0; j < KRY_MS_MAX_ND; ++j) {
                if (j < nd) {
                    Qj[j] += as * dj[j];
                    dj[j] = zn * red[Gact + q * nd + j] + bs * dj[j];
                    a.Q[s * nd + j] = Qj[j];
                    a.d[s * nd + j] = dj[j];
                }
            }
            const int it = it0 + 1;
            a.iters[s] = it;
            const double res = fabs(zn) * sqrt(rn);
            const double bn = sqrt(s_bn[q]);
            a.relres[s] = res / bn;
            if (!(res > a.rtol * bn) || it >= lim) a.active[s] = 0;
            a.zeta_old[s] = z;
            a.zeta[s] = zn;
        }
    }
    if (t < Gact) {
        const double rcq = red[t];
        const double b = rr_t > 0.0 ? rcq / rr_t : 0.0;
        a.alpha[t] = s_alpha[t];
        a.beta[t] = b;
        a.alpha_old[t] = s_alpha[t];
        a.beta_old[t] = b;
        a.rr[t] = rcq;
    }
    for (int i = t; i < nrows; i += RB) a.rc[i] = red[i];
}

template <int ND>
void launch_ms_r(int nblk, int Gact, hipStream_t st, double* r, const double* w, const double* D, int64_t n,
                 const MsScalarArgs& a) {
    hipLaunchKernelGGL(k_ms_r<ND>, dim3(nblk, Gact), dim3(RB), 0, st, r, w, D, a.partial_pw, a.npw, a.rr, a.pw,
                       Gact, n, a.partial);
}

void ms_residual_and_scalars(int nd, int nblk, int Gact, hipStream_t st, double* r, const double* w, const double* D,
                             int64_t n, const MsScalarArgs& a) {
    switch (nd) {
        case 1: launch_ms_r<1>(nblk, Gact, st, r, w, D, n, a); break;
        case 2: launch_ms_r<2>(nblk, Gact, st, r, w, D, n, a); break;
        case 3: launch_ms_r<3>(nblk, Gact, st, r, w, D, n, a); break;
        case 4: launch_ms_r<4>(nblk, Gact, st, r, w, D, n, a); break;
        case 5: launch_ms_r<5>(nblk, Gact, st, r, w, D, n, a); break;
        case 6: launch_ms_r<6>(nblk, Gact, st, r, w, D, n, a); break;
        case 7: launch_ms_r<7>(nblk, Gact, st, r, w, D, n, a); break;
        case 8: launch_ms_r<8>(nblk, Gact, st, r, w, D, n, a); break;
        case 9: launch_ms_r<9>(nblk, Gact, st, r, w, D, n, a); break;
        default: KRY_REQUIRE(false, "multi-shift CG takes 1..9 dot vectors");
    }
    KRY_HIP(hipGetLastError());
    if (a.nS <= RB && Gact <= RB && (1 + nd) * Gact <= MS_ONE_ROWS)
        hipLaunchKernelGGL(k_ms_scalar_one, dim3(1), dim3(RB), 0, st, a);
    else
        hipLaunchKernelGGL(k_ms_scalar, dim3(1), dim3(RB), 0, st, a);
    KRY_HIP(hipGetLastError());
}

// p_q = r_q + beta_q p_q
__global__ void k_ms_p(double* __restrict__ p, const double* __restrict__ r, const double* __restrict__ beta,
                       int64_t n) {
    const int q = blockIdx.y;
    const double b = beta[q];
    double* pq = p + q * n;
    const double* rq = r + q * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pq[i] = rq[i] + b * pq[i];
}

template <typename T>
__global__ void k_swap_vec(T* __restrict__ base, int64_t stride, int a, int b, int64_t n) {
    T* pa = base + a * stride;
    T* pb = base + b * stride;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T t = pa[i];
        pa[i] = pb[i];
        pb[i] = t;
    }
}

template <typename T>
void swap_vectors(T* base, int64_t stride, int a, int b, int64_t n, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_swap_vec<T>, dim3((unsigned)blocks), dim3(256), 0, st, base, stride, a, b, n);
    KRY_HIP(hipGetLastError());
}
template void swap_vectors<double>(double*, int64_t, int, int, int64_t, hipStream_t);
template void swap_vectors<float>(float*, int64_t, int, int, int64_t, hipStream_t);

__global__ void k_ms_swap_scalars(double* rr, double* bnorm2, double* alpha_old, double* beta_old, double* beta,
                                  int a, int b) {
    if (threadIdx.x != 0) return;
    double* arr[5] = {rr, bnorm2, alpha_old, beta_old, beta};
    for (double* v : arr) {
        const double t = v[a];
        v[a] = v[b];
        v[b] = t;
    }
}

void mscg_run(const MatvecFn<double>& A, const MsFusedFn* fused, int fused_pw,
              const std::function<void(int, int)>& swap,
              int64_t n, int G,
              const std::vector<int>& group_of_shift, const std::vector<double>& sigma, const double* D, int nd,
              const std::vector<int>& rhs_of_group, double rtol, int maxit, MsCgBuffers& B, std::vector<int>& iters,
              std::vector<double>& relres, std::vector<double>& Q, hipStream_t st) {
    KRY_REQUIRE(nd >= 1 && nd <= KRY_MS_MAX_ND && (int)rhs_of_group.size() == G, "bad multi-shift right-hand sides");
    const int S = (int)group_of_shift.size();
    const int nblk = dot_blocks(n);
    KRY_REQUIRE(nblk <= RB, "dot partials exceed one reduction block");
    const size_t vb = (size_t)n * sizeof(double);
    for (int q = 0; q < G; ++q) {
        const double* b = D + (size_t)rhs_of_group[q] * n;
        KRY_HIP(hipMemcpyAsync(B.r + (size_t)q * n, b, vb, hipMemcpyDeviceToDevice, st));
        KRY_HIP(hipMemcpyAsync(B.p + (size_t)q * n, b, vb, hipMemcpyDeviceToDevice, st));
    }
    // host state: group -> position, position -> group, active shift list
    std::vector<int> pos_of(G), grp_at(G), pos(S), list(S), lim(S, maxit), act(S);
    for (int g = 0; g < G; ++g) pos_of[g] = grp_at[g] = g;
    for (int s = 0; s < S; ++s) {
        pos[s] = group_of_shift[s];
        list[s] = s;
    }
    KRY_HIP(hipMemcpyAsync(B.pos, pos.data(), S * sizeof(int), hipMemcpyHostToDevice, st));
    KRY_HIP(hipMemcpyAsync(B.list, list.data(), S * sizeof(int), hipMemcpyHostToDevice, st));
    KRY_HIP(hipMemcpyAsync(B.limit, lim.data(), S * sizeof(int), hipMemcpyHostToDevice, st));
    KRY_HIP(hipMemcpyAsync(B.sigma, sigma.data(), S * sizeof(double), hipMemcpyHostToDevice, st));
    KRY_HIP(hipMemcpyAsync(B.rhs, rhs_of_group.data(), G * sizeof(int), hipMemcpyHostToDevice, st));
    // gram[j][a] = D_j . D_a
    for (int j = 0; j < nd; ++j)
        dot_batched<double>(D + (size_t)j * n, 0, D, n, n, nd, B.partial, B.gram + (size_t)j * nd, st);
    hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(256), 0, st, B.gram, B.rhs, nd, G, S, B.pos, B.rr, B.bnorm2,
                       B.alpha_old, B.beta_old, B.beta, B.zeta, B.zeta_old, B.d, B.Q, B.relres, B.active, B.iters,
                       B.limit);
    KRY_HIP(hipGetLastError());
    MsScalarArgs sa;
    sa.nd = nd;
    sa.nblk = nblk;
    sa.partial_pw = B.partial_pw;
    sa.partial = B.partial;
    sa.rr = B.rr;
    sa.rc = B.rc;
    sa.pw = B.pw;
    sa.beta = B.beta;
    sa.alpha = B.alpha;
    sa.alpha_old = B.alpha_old;
    sa.beta_old = B.beta_old;
    sa.bnorm2 = B.bnorm2;
    sa.list = B.list;
    sa.pos = B.pos;
    sa.sigma = B.sigma;
    sa.zeta = B.zeta;
    sa.zeta_old = B.zeta_old;
    sa.zeta_new = B.zeta_new;
    sa.alpha_s = B.alpha_s;
    sa.d = B.d;
    sa.Q = B.Q;
    sa.relres = B.relres;
    sa.active = B.active;
    sa.iters = B.iters;
    sa.limit = B.limit;
    sa.rtol = rtol;
    sa.nS = S;
    const bool spectral_pw = fused && fused_pw > 0;
    sa.npw = spectral_pw ? fused_pw : nblk;
    int Gact = G, nlist = S;
    int64_t ublocks = (n + 255) / 256;
    if (ublocks > 1024) ublocks = 1024;
    const int check = 16;
    // An iteration: the product (with the previous iteration's direction
    // update folded in when `fused` is given, and the p . w partials formed
    // inside it when it can), else the p . w partials as a pass of their own,
    // the residual update and the one-block scalar step; without `fused`, the
    // direction update is a pass of its own at the end.
    for (int it = 0; it < maxit && Gact > 0; ++it) {
        if (fused) (*fused)(B.r, B.p, B.beta, B.w, Gact, spectral_pw ? B.partial_pw : nullptr, st);
        else A(B.p, B.w, Gact, st, nullptr);
        if (!spectral_pw) {
            hipLaunchKernelGGL(k_dot_partial<double>, dim3(nblk, Gact), dim3(RB), 0, st, B.p, n, B.w, n, n,
                               B.partial_pw);
            KRY_HIP(hipGetLastError());
        }
        sa.Gact = Gact;
        sa.nlist = nlist;
        ms_residual_and_scalars(nd, nblk, Gact, st, B.r, B.w, D, n, sa);
        if (!fused) {
            hipLaunchKernelGGL(k_ms_p, dim3((unsigned)ublocks, Gact), dim3(256), 0, st, B.p, B.r, B.beta, n);
            KRY_HIP(hipGetLastError());
        }
        if ((it + 1) % check != 0 && it + 1 != maxit) continue;
        KRY_HIP(hipMemcpyAsync(act.data(), B.active, S * sizeof(int), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        std::vector<char> alive(G, 0);
        nlist = 0;
        for (int s = 0; s < S; ++s)
            if (act[s]) {
                list[nlist++] = s;
                alive[group_of_shift[s]] = 1;
            }
        // move groups with no running shift behind the active positions
        bool moved = false;
        int q = 0;
        while (q < Gact) {
            if (alive[grp_at[q]]) {
                ++q;
                continue;
            }
            const int last = Gact - 1;
            if (last != q) {
                swap_vectors<double>(B.r, n, q, last, n, st);
                swap_vectors<double>(B.p, n, q, last, n, st);
                hipLaunchKernelGGL(k_ms_swap_scalars, dim3(1), dim3(64), 0, st, B.rr, B.bnorm2, B.alpha_old,
                                   B.beta_old, B.beta, q, last);
                KRY_HIP(hipGetLastError());
                swap(q, last);
                std::swap(grp_at[q], grp_at[last]);
                pos_of[grp_at[q]] = q;
                pos_of[grp_at[last]] = last;
                moved = true;
            }
            --Gact;
        }
        if (moved) {
            for (int s = 0; s < S; ++s) pos[s] = pos_of[group_of_shift[s]];
            KRY_HIP(hipMemcpyAsync(B.pos, pos.data(), S * sizeof(int), hipMemcpyHostToDevice, st));
        }
        if (nlist > 0) KRY_HIP(hipMemcpyAsync(B.list, list.data(), nlist * sizeof(int), hipMemcpyHostToDevice, st));
    }
    iters.resize(S);
    relres.resize(S);
    Q.resize((size_t)S * nd);
    KRY_HIP(hipMemcpyAsync(iters.data(), B.iters, S * sizeof(int), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipMemcpyAsync(relres.data(), B.relres, S * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipMemcpyAsync(Q.data(), B.Q, (size_t)S * nd * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
}

// y = a x + b y  (FP64 coefficients per vector)
template <typename R>
__global__ void k_axpby(const R* __restrict__ x, R* __restrict__ y, double a, double b, int64_t n) {
    const int vec = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[vec * n + i] = (R)(a * (double)x[vec * n + i] + b * (double)y[vec * n + i]);
}

template <typename R>
void axpby(const R* x, R* y, double a, double b, int64_t n, int nvec, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby<R>, vec_grid(n, nvec), dim3(256), 0, st, x, y, a, b, n);
    KRY_HIP(hipGetLastError());
}
template void axpby<double>(const double*, double*, double, double, int64_t, int, hipStream_t);
template void axpby<float>(const float*, float*, double, double, int64_t, int, hipStream_t);

// x64 += (double) d32
__global__ void k_add_f32(const float* __restrict__ d, double* __restrict__ x, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += (double)d[i];
}
void add_f32(const float* d, double* x, int64_t n, hipStream_t st) {
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    hipLaunchKernelGGL(k_add_f32, dim3((unsigned)b), dim3(256), 0, st, d, x, n);
    KRY_HIP(hipGetLastError());
}

}  // namespace kry
