// The paper's own objective and its companions on the device:
//  - the quadrant block-circulant log-determinant of Sec. 3.3 and its range
//    derivative (eq. circ_diag, eq. trace_approx), as two dense DFT
//    contractions per lag grid (FP64 tiled products against twiddle tables);
//  - pl~ of eq. prof_lik with the genGK terms of Sec. 3.2 and the
//    approximate gradient of eq. approx_grad;
//  - the low-rank posterior variance of eq. bgamma_approx;
//  - the host symmetric tridiagonal eigen-solver these use.
//
// The (2 n - 1)-point DFT has no power-of-two structure, and only n of its
// 2 n - 1 frequencies per axis are needed, so it is written as a product
// with cos / sin tables: T = c F2 over the column lags (both grids at once),
// then lam = G1 T_cos + H1 T_sin over the row lags (G1 = cos, H1 = -sin);
// the lag grid is even, so the DFT is real and this is its real part.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "krylov.hpp"

namespace kry {
namespace {

constexpr int PB = 256;

// ---- dense products (row-major): C = A B, or C += A B -------------------------------------
// A is m x k (row stride lda), B is k x n (ldb), C is m x n (ldc).  A
// workgroup of 256 threads computes a 64 x 64 tile of C, each thread a 4 x 4
// block, over k in steps of 16 staged through LDS (A transposed there, so a
// thread's four rows are adjacent); fused multiply-adds in a fixed order, so
// results do not depend on the launch.  Edges are zero-filled.
constexpr int GT = 64, GK = 16;

template <typename R>
__global__ void __launch_bounds__(256) k_gemm_rm(int m, int n, int k, const R* __restrict__ A, int64_t lda,
                                                  const R* __restrict__ B, int64_t ldb, R* __restrict__ C,
                                                  int64_t ldc, int accumulate) {
    __shared__ R As[GK][GT + 4];
    __shared__ R Bs[GK][GT + 4];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const int64_t row0 = (int64_t)blockIdx.y * GT, col0 = (int64_t)blockIdx.x * GT;
    R acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (R)0;
    // loader positions: A tile 64 rows x 16 k (4 consecutive k per thread),
    // B tile 16 k x 64 columns (4 consecutive columns per thread)
    const int ar = tid / 4, ak = (tid % 4) * 4;
    const int bk = tid / 16, bc = (tid % 16) * 4;
    for (int k0 = 0; k0 < k; k0 += GK) {
        R av[4], bv[4];
        const int64_t gr = row0 + ar;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = k0 + ak + q;
            av[q] = (gr < m && kk < k) ? A[gr * lda + kk] : (R)0;
        }
        const int kb = k0 + bk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gc = col0 + bc + q;
            bv[q] = (kb < k && gc < n) ? B[(int64_t)kb * ldb + gc] : (R)0;
        }
        __syncthreads();  // the previous step's reads are done
#pragma unroll
        for (int q = 0; q < 4; ++q) As[ak + q][ar] = av[q];
#pragma unroll
        for (int q = 0; q < 4; ++q) Bs[bk][bc + q] = bv[q];
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            R a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma_rn(a[i], b[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t r = row0 + ty * 4 + i;
        if (r >= m) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t c = col0 + tx * 4 + j;
            if (c >= n) continue;
            R& o = C[r * ldc + c];
            o = accumulate ? o + acc[i][j] : acc[i][j];
        }
    }
}

template <typename R>
void gemm_rm(int m, int n, int k, const R* A, int64_t lda, const R* B, int64_t ldb, R* C, int64_t ldc,
             bool accumulate, hipStream_t st) {
    if (m <= 0 || n <= 0) return;
    const dim3 grid((unsigned)((n + GT - 1) / GT), (unsigned)((m + GT - 1) / GT));
    KRY_REQUIRE(grid.y <= 65535u, "product too tall for one launch");
    hipLaunchKernelGGL(k_gemm_rm<R>, grid, dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc, accumulate ? 1 : 0);
    KRY_HIP(hipGetLastError());
}

// out[l * 2 nf + j]: cos(2 pi l j / M) for j < nf, sin(2 pi l (j - nf) / M)
// after (rows l < rows); the angle is reduced exactly in integers first.
__global__ void k_twiddle_lag_major(double* __restrict__ out, int rows, int nf, int M) {
    const int64_t total = (int64_t)rows * 2 * nf;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(i / (2 * nf));
        const int j = (int)(i - (int64_t)l * 2 * nf);
        const int f = j < nf ? j : j - nf;
        const int64_t r = ((int64_t)l * f) % M;
        double s, c;
        sincospi(2.0 * (double)r / (double)M, &s, &c);
        out[i] = j < nf ? c : s;
    }
}

// G[p * M + l] = cos(2 pi l p / M), H[p * M + l] = -sin(2 pi l p / M), p < nf.
__global__ void k_twiddle_freq_major(double* __restrict__ G, double* __restrict__ H, int nf, int M) {
    const int64_t total = (int64_t)nf * M;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(i / M);
        const int l = (int)(i - (int64_t)p * M);
        const int64_t r = ((int64_t)l * p) % M;
        double s, c;
        sincospi(2.0 * (double)r / (double)M, &s, &c);
        G[i] = c;
        H[i] = -s;
    }
}

__device__ double block_reduce_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = PB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ double block_reduce_min(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = PB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Per block: sum log lam, sum dlam / lam (when dlam), min lam.
__global__ void __launch_bounds__(PB) k_quadrant_partial(const double* __restrict__ lam,
                                                         const double* __restrict__ dlam, int64_t n,
                                                         double* __restrict__ part) {
    __shared__ double sh[PB];
    double sl = 0.0, sd = 0.0, mn = INFINITY;
    for (int64_t i = blockIdx.x * (int64_t)PB + threadIdx.x; i < n; i += (int64_t)gridDim.x * PB) {
        const double v = lam[i];
        mn = fmin(mn, v);
        sl += log(v);
        if (dlam) sd += dlam[i] / v;
    }
    sl = block_reduce_sum(sl, sh);
    sd = block_reduce_sum(sd, sh);
    mn = block_reduce_min(mn, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = sl;
        part[3 * blockIdx.x + 1] = sd;
        part[3 * blockIdx.x + 2] = mn;
    }
}

// out[c] = sum_i z_i * base[i * n + c] (FP64), k vectors of n.
template <typename R>
__global__ void k_combine(const R* __restrict__ base, int64_t n, int k, const double* __restrict__ z,
                          double* __restrict__ out) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < k; ++i) acc += z[i] * (double)base[(int64_t)i * n + c];
        out[c] = acc;
    }
}

// psi[j] = b[j] - x[cell[j]]
__global__ void k_residual(const double* __restrict__ b, const double* __restrict__ x,
                           const int32_t* __restrict__ cell, int64_t p, double* __restrict__ psi) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x)
        psi[j] = b[j] - x[cell[j]];
}

// var[i] = s2 * (1 - sum_j delta_j Z[i + j ld]^2) for c cells.
template <typename R>
__global__ void k_postvar(const R* __restrict__ Z, int64_t c, int64_t ld, int k, const double* __restrict__ delta,
                          double s2, double* __restrict__ var) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) {
            const double v = (double)Z[i + (int64_t)j * ld];
            acc += delta[j] * v * v;
        }
        var[i] = s2 * (1.0 - acc);
    }
}

dim3 grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

// Workspace carved from one buffer.
struct Carve {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + off);
        off += (count * sizeof(T) + 255) & ~size_t(255);
        return p;
    }
};

}  // namespace

// ---- quadrant log-determinant (Sec. 3.3, eq. trace_approx) ---------------------------------
struct Quadrant {
    double logdet = 0, dlogdet = 0, lam_min = 0;
};

Quadrant quadrant_device(Problem& P, const Matern& th, bool deriv, hipStream_t st) {
    Ctx& C = *P.ctx;
    const int n1 = P.n1, n2 = P.n2, M1 = 2 * n1 - 1, M2 = 2 * n2 - 1;
    const int ng = deriv ? 2 : 1;
    const int64_t nq = (int64_t)n1 * n2;
    const int nb = (int)std::min<int64_t>(1024, (nq + PB - 1) / PB);
    auto layout = [&](Carve& w, double** c, double** F2, double** T, double** G1, double** H1, double** lam,
                      double** part) {
        *c = w.take<double>((size_t)ng * M1 * M2);
        *F2 = w.take<double>((size_t)M2 * 2 * n2);
        *T = w.take<double>((size_t)ng * M1 * 2 * n2);
        *G1 = w.take<double>((size_t)n1 * M1);
        *H1 = w.take<double>((size_t)n1 * M1);
        *lam = w.take<double>((size_t)ng * nq);
        *part = w.take<double>((size_t)3 * nb);
    };
    double *c, *F2, *T, *G1, *H1, *lam, *part;
    Carve probe{nullptr};
    layout(probe, &c, &F2, &T, &G1, &H1, &lam, &part);
    P.tmp1.ensure(C, probe.off + 256);
    Carve w{P.tmp1.as<char>()};
    layout(w, &c, &F2, &T, &G1, &H1, &lam, &part);
    lag_grid_device(C, M1, M2, P.dx1, P.dx2, th, c, st, false);
    if (deriv) lag_grid_device(C, M1, M2, P.dx1, P.dx2, th, c + (size_t)M1 * M2, st, true);
    hipLaunchKernelGGL(k_twiddle_lag_major, grid_for((int64_t)M2 * 2 * n2), dim3(256), 0, st, F2, M2, n2, M2);
    KRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_twiddle_freq_major, grid_for((int64_t)n1 * M1), dim3(256), 0, st, G1, H1, n1, M1);
    KRY_HIP(hipGetLastError());
    // T (ng M1 x 2 n2) = c (ng M1 x M2) F2 (M2 x 2 n2): the column lags, both grids
    gemm_rm<double>(ng * M1, 2 * n2, M2, c, M2, F2, 2 * n2, T, 2 * n2, false, st);
    for (int gi = 0; gi < ng; ++gi) {
        const double* Tg = T + (size_t)gi * M1 * 2 * n2;
        double* lg = lam + (size_t)gi * nq;
        // lam (n1 x n2) = G1 (n1 x M1) T_cos (M1 x n2) + H1 T_sin: the row lags
        gemm_rm<double>(n1, n2, M1, G1, M1, Tg, 2 * n2, lg, n2, false, st);
        gemm_rm<double>(n1, n2, M1, H1, M1, Tg + n2, 2 * n2, lg, n2, true, st);
    }
    hipLaunchKernelGGL(k_quadrant_partial, dim3(nb), dim3(PB), 0, st, lam, deriv ? lam + nq : nullptr, nq, part);
    KRY_HIP(hipGetLastError());
    std::vector<double> h((size_t)3 * nb);
    KRY_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
    Quadrant q;
    q.lam_min = INFINITY;
    for (int b = 0; b < nb; ++b) {
        q.logdet += h[3 * b];
        q.dlogdet += h[3 * b + 1];
        q.lam_min = std::min(q.lam_min, h[3 * b + 2]);
    }
    if (!(q.lam_min > 0)) throw Error(KRY_ENOTPSD, "an eigenvalue of the block-circulant quadrant is not positive");
    return q;
}

// ---- symmetric tridiagonal eigen-decomposition (host) -------------------------------------
// Implicit QL with a shift from the leading 2 x 2 block (Golub and Van Loan,
// Sec. 8.3, in the QL orientation): d (k) and e (k - 1, e[i] couples i and
// i + 1) in; eigenvalues ascending in d and the rotations accumulated into W
// (column-major, column j the eigenvector of d[j]).
void tridiag_eigen(std::vector<double>& d, std::vector<double> e, std::vector<double>& W) {
    const int k = (int)d.size();
    W.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) W[(size_t)i * k + i] = 1.0;
    e.resize(k, 0.0);
    if (k > 0) e[k - 1] = 0.0;
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < k; ++l) {
        for (int iter = 0;; ++iter) {
            int m = l;
            for (; m < k - 1; ++m)
                if (std::fabs(e[m]) <= eps * (std::fabs(d[m]) + std::fabs(d[m + 1]))) break;
            if (m == l) break;
            KRY_REQUIRE(iter < 100, "tridiagonal eigen-solver did not converge");
            // shift: the eigenvalue of the leading 2 x 2 block nearer d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, shift = 0.0;
            bool split = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {  // the rotation vanished: the matrix splits here
                    d[i + 1] -= shift;
                    e[m] = 0.0;
                    split = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - shift;
                r = (d[i] - g) * s + 2.0 * c * b;
                shift = s * r;
                d[i + 1] = g + shift;
                g = c * r - b;
                double* wi = W.data() + (size_t)i * k;
                double* wj = W.data() + (size_t)(i + 1) * k;
                for (int q = 0; q < k; ++q) {
                    const double t = wj[q];
                    wj[q] = s * wi[q] + c * t;
                    wi[q] = c * wi[q] - s * t;
                }
            }
            if (split) continue;
            d[l] -= shift;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    // ascending order
    std::vector<int> ord(k);
    for (int i = 0; i < k; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] < d[b]; });
    std::vector<double> d2(k), W2((size_t)k * k);
    for (int j = 0; j < k; ++j) {
        d2[j] = d[ord[j]];
        std::copy(W.begin() + (size_t)ord[j] * k, W.begin() + (size_t)(ord[j] + 1) * k, W2.begin() + (size_t)j * k);
    }
    d = d2;
    W = W2;
}

// ---- low-rank posterior variance (eq. bgamma_approx) --------------------------------------
// From a genGK run in the unit-variance form (B' = sigma B, so
// B'^T B' = W Theta' W^T with Theta' = sigma2 Theta and the same W), the
// weights Theta (Theta + I / sigma2)^{-1} = Theta' (Theta' + I)^{-1}.
void postvar_device(Problem& P, const GkRun& G, double sigma2, double* d_var, hipStream_t st) {
    Ctx& C = *P.ctx;
    const int k = (int)G.z.size();
    const int64_t n = (int64_t)P.n1 * P.n2;
    std::vector<double> d(k), e(k > 1 ? k - 1 : 0), W;
    for (int i = 0; i < k; ++i) d[i] = G.alpha[i] * G.alpha[i] + G.beta[i + 1] * G.beta[i + 1];
    for (int i = 0; i + 1 < k; ++i) e[i] = G.alpha[i + 1] * G.beta[i + 1];
    tridiag_eigen(d, e, W);
    std::vector<double> delta(k);
    for (int j = 0; j < k; ++j) {
        const double t = std::max(d[j], 0.0);
        delta[j] = t / (t + 1.0);
    }
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(1 << 28) / std::max(k, 1)));
    const size_t rb = (size_t)G.real_bytes;
    auto layout = [&](Carve& w, void** Wd, double** dd, void** Z) {
        *Wd = w.take<char>((size_t)k * k * rb);
        *dd = w.take<double>(k);
        *Z = w.take<char>((size_t)chunk * k * rb);
    };
    void *Wd, *Z;
    double* dd;
    Carve probe{nullptr};
    layout(probe, &Wd, &dd, &Z);
    P.tmp1.ensure(C, probe.off + 256);
    Carve w{P.tmp1.as<char>()};
    layout(w, &Wd, &dd, &Z);
    if (rb == 8) {
        KRY_HIP(hipMemcpyAsync(Wd, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice, st));
    } else {
        std::vector<float> Wf(W.begin(), W.end());
        KRY_HIP(hipMemcpyAsync(Wd, Wf.data(), Wf.size() * sizeof(float), hipMemcpyHostToDevice, st));
    }
    KRY_HIP(hipMemcpyAsync(dd, delta.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
    for (int64_t i0 = 0; i0 < n; i0 += chunk) {
        const int c = (int)std::min<int64_t>(chunk, n - i0);
        // Z[j][i] = sum_l W[l][j] (Sigma v_l)[i0 + i]: with the basis stored
        // vector by vector (k rows of n), Z (k x c, row-major) = W^T Sv; W is
        // held column by column, so row j of W^T is W's column j, contiguous
        if (rb == 8) {
            gemm_rm<double>(k, c, k, static_cast<const double*>(Wd), k, static_cast<const double*>(G.Sv) + i0, n,
                            static_cast<double*>(Z), c, false, st);
            hipLaunchKernelGGL(k_postvar<double>, grid_for(c), dim3(256), 0, st, static_cast<const double*>(Z),
                               (int64_t)c, (int64_t)c, k, dd, sigma2, d_var + i0);
        } else {
            gemm_rm<float>(k, c, k, static_cast<const float*>(Wd), k, static_cast<const float*>(G.Sv) + i0, n,
                           static_cast<float*>(Z), c, false, st);
            hipLaunchKernelGGL(k_postvar<float>, grid_for(c), dim3(256), 0, st, static_cast<const float*>(Z),
                               (int64_t)c, (int64_t)c, k, dd, sigma2, d_var + i0);
        }
        KRY_HIP(hipGetLastError());
    }
    KRY_HIP(hipStreamSynchronize(st));
}

// b = y - X beta (compact FP64) into dst.
void residual_data(Problem& P, const double* beta, double* dst, hipStream_t st) {
    KRY_HIP(hipMemcpyAsync(dst, P.y64.ptr, P.p * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int j = 0; j < P.q; ++j) axpby<double>(P.X64.as<double>() + (size_t)j * P.p, dst, -beta[j], 1.0, P.p, 1, st);
}

// x_k* = Sigma V_k z (and optionally w = V_k z) on every cell, FP64.
void gk_fields(const GkRun& G, int64_t n, double* d_z, double* xs, double* wv, hipStream_t st) {
    const int k = (int)G.z.size();
    KRY_HIP(hipMemcpyAsync(d_z, G.z.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
    if (G.real_bytes == 8) {
        hipLaunchKernelGGL(k_combine<double>, grid_for(n), dim3(256), 0, st, static_cast<const double*>(G.Sv), n, k,
                           d_z, xs);
        if (wv)
            hipLaunchKernelGGL(k_combine<double>, grid_for(n), dim3(256), 0, st, static_cast<const double*>(G.V), n,
                               k, d_z, wv);
    } else {
        hipLaunchKernelGGL(k_combine<float>, grid_for(n), dim3(256), 0, st, static_cast<const float*>(G.Sv), n, k,
                           d_z, xs);
        if (wv)
            hipLaunchKernelGGL(k_combine<float>, grid_for(n), dim3(256), 0, st, static_cast<const float*>(G.V), n, k,
                               d_z, wv);
    }
    KRY_HIP(hipGetLastError());
}

// ---- pl~ and its approximate gradient (eq. prof_lik, eq. approx_grad) ----------------------
void plik_device(Problem& P, const kry_matern* theta, const double* beta, const kry_opts* o, kry_plik_result* r,
                 hipStream_t st) {
    Ctx& C = *P.ctx;
    const Matern th = to_matern_abi(theta);
    const int64_t p = P.p, n = (int64_t)P.n1 * P.n2;
    const int q = P.q;
    const int nblk = dot_blocks(std::max(p, n));
    // scratch: b, psi (p); x*, w, dSigma w (n); z; dots
    auto layout = [&](Carve& w, double** b, double** psi, double** xs, double** wv, double** dw, double** dz,
                      double** part, double** dots) {
        *b = w.take<double>(p);
        *psi = w.take<double>(p);
        *xs = w.take<double>(n);
        *wv = w.take<double>(n);
        *dw = w.take<double>(n);
        *dz = w.take<double>(o->gk_steps + 8);
        *part = w.take<double>((size_t)(q + 2) * nblk);
        *dots = w.take<double>(q + 8);
    };
    double *b, *psi, *xs, *wv, *dw, *dz, *part, *dots;
    Carve probe{nullptr};
    layout(probe, &b, &psi, &xs, &wv, &dw, &dz, &part, &dots);
    P.tmp4.ensure(C, probe.off + 256);
    Carve w{P.tmp4.as<char>()};
    layout(w, &b, &psi, &xs, &wv, &dw, &dz, &part, &dots);
    residual_data(P, beta, b, st);
    GkRun G;
    gengk_run(P, th, o, G, b, st);
    const int k = (int)G.z.size();
    gk_fields(G, n, dz, xs, wv, st);
    if (P.irregular) {  // psi = b - A x*
        irr_gather<double, double>(P, xs, 1, psi, nullptr, nullptr, 1, nullptr, st);
        axpby<double>(b, psi, 1.0, -1.0, p, 1, st);
    } else {
        hipLaunchKernelGGL(k_residual, grid_for(p), dim3(256), 0, st, b, xs, P.cell.as<int32_t>(), p, psi);
        KRY_HIP(hipGetLastError());
    }
    // psi . psi and X_j . psi
    dot_batched<double>(psi, 0, psi, 0, p, 1, part, dots, st);
    if (q > 0) dot_batched<double>(P.X64.as<double>(), p, psi, 0, p, q, part, dots + 1, st);
    // dSigma w: the range derivative's spectrum on the product's embedding
    const int64_t nspec = (int64_t)(P.N2 / 2 + 1) * P.N1;
    P.spec_multi64.ensure(C, (size_t)nspec * sizeof(double));
    double lo, hi;
    spectrum_device(P, P.N1, P.N2, th, P.spec_multi64.as<double>(), &lo, &hi, st, true);
    spectrum_scale(P.spec_multi64.as<double>(), nspec, 1.0 / ((double)P.N1 * P.N2), false,
                   P.spec_multi64.as<double>(), nullptr, st);
    ConvSpec s;
    s.N1 = P.N1;
    s.N2 = P.N2;
    s.nvec = 1;
    s.in_mode = IN_DENSE;
    s.in = wv;
    s.in_vstride = n;
    s.in_rstride = P.n2;
    s.rows_in = P.n1;
    s.row_len = P.n2;
    s.out_mode = OUT_GRID;
    s.out = dw;
    s.out_vstride = n;
    s.rows_out = P.n1;
    s.cols_out = P.n2;
    s.scale = 1.0;
    s.lam = P.spec_multi64.ptr;
    s.lam_tstride = 0;
    s.vecs_per_theta = 1;
    conv_apply<double>(P, s, st);
    dot_batched<double>(wv, 0, dw, 0, n, 1, part, dots + 1 + q, st);
    std::vector<double> h(q + 2);
    KRY_HIP(hipMemcpyAsync(h.data(), dots, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
    const Quadrant qd = quadrant_device(P, th, true, st);
    double zz = 0;
    for (int i = 0; i < k; ++i) zz += G.z[i] * G.z[i];
    const double s2 = th.sigma2, t2 = th.tau2, pp = h[0], wdw = h[1 + q];
    std::memset(r, 0, sizeof(*r));
    r->pl = -0.5 * (double)p * std::log(t2) - pp / (2.0 * t2) - 0.5 * (double)n * std::log(s2) - 0.5 * qd.logdet -
            zz / (2.0 * s2);
    r->logdet_bccb = qd.logdet;
    r->dlogdet_bccb = qd.dlogdet;
    r->psi2 = pp;
    r->z2 = zz;
    r->grad_lam2 = 0.5 * (double)n * s2 - 0.5 * zz;
    r->grad_range = -0.5 * qd.dlogdet + 0.5 * wdw / s2;
    r->grad_lame2 = 0.5 * (double)p * t2 - 0.5 * pp;
    for (int j = 0; j < q; ++j) r->grad_beta[j] = h[1 + j] / t2;
    r->ncov = q;
    r->gk_steps = k;
}

// Posterior variance at every cell and, optionally, x_k* + X beta.
void posterior_variance_device(Problem& P, const kry_matern* theta, const double* beta, const kry_opts* o,
                               double* var_x, double* var_y, double* mean_x, hipStream_t st) {
    Ctx& C = *P.ctx;
    const Matern th = to_matern_abi(theta);
    const int64_t p = P.p, n = (int64_t)P.n1 * P.n2;
    P.tmp4.ensure(C, ((size_t)p + 3 * (size_t)n + (size_t)o->gk_steps + 64) * sizeof(double) + 1024);
    Carve w{P.tmp4.as<char>()};
    double* b = w.take<double>(p);
    double* var = w.take<double>(n);
    double* xs = w.take<double>(n);
    double* dz = w.take<double>(o->gk_steps + 8);
    residual_data(P, beta, b, st);
    GkRun G;
    gengk_run(P, th, o, G, b, st);
    postvar_device(P, G, th.sigma2, var, st);
    std::vector<double> hv(n);
    KRY_HIP(hipMemcpyAsync(hv.data(), var, n * sizeof(double), hipMemcpyDeviceToHost, st));
    if (mean_x) gk_fields(G, n, dz, xs, nullptr, st);
    KRY_HIP(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) {
        var_x[i] = hv[i];
        if (var_y) var_y[i] = hv[i] + th.tau2;
    }
    if (mean_x) {
        KRY_HIP(hipMemcpyAsync(mean_x, xs, n * sizeof(double), hipMemcpyDeviceToHost, st));
        KRY_HIP(hipStreamSynchronize(st));
        for (int j = 0; j < P.q; ++j) {
            const double* xj = P.h_X->data() + (size_t)j * n;
            for (int64_t i = 0; i < n; ++i) mean_x[i] += xj[i] * beta[j];
        }
    }
}


}  // namespace kry
