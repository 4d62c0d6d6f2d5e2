// Circulant-embedding transforms: Matern lag grid, spectrum and the fused
// three-stage masked BTTB product.
//
// The product follows the paper's fast route for Sigma v on a grid (Sec. 3
// and 3.2: the symmetric BTTB Sigma is embedded in a block-circulant matrix
// diagonalised by the 2-D DFT).  With lam = DFT2(c) of the embedding lag grid,
//   Sigma v = [ IDFT2( lam * DFT2( zero-pad(v) ) ) ]_corner,
// and the masked product scatters the compact vector into the grid first and
// gathers observed cells at the end.  Layout of the transform intermediate:
// column-major over the half spectrum, Y[vec][k2][row], k2 in [0, N2/2], so
// the column pass reads contiguous columns.
//
//  stage A  rows:    scatter -> real FFT of length N2 (as a complex FFT of
//                    length N2/2 plus the even/odd split), written transposed
//                    in tiles of RT rows (contiguous runs of RT entries)
//  stage B  columns: forward FFT of length N1 (zero rows below the input),
//                    multiply by lam, inverse FFT, keep the output rows
//  stage C  rows:    read RT-row tiles, merge the split, inverse FFT of length
//                    N2/2, gather observed cells (+ eta v) or write the grid
#include <cmath>
#include <mutex>
#include <unordered_map>

#include "fft.hpp"
#include "internal.hpp"

namespace kry {

// ---------------------------------------------------------------------------
// Matern correlation (Sec. 2) on the device
// ---------------------------------------------------------------------------
struct MaternDev {
    double range, nu, ratio, ca, sa, dx1, dx2;
};

// e^x K_nu(x) by the trapezoidal rule on the integral representation
// K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt (e.g. DLMF 10.32.9), with
// cosh t - 1 = 2 sinh^2(t/2) so the exponent stays small.  The integrand is
// analytic and decays doubly exponentially, so the rule converges
// geometrically in 1/h; the step shrinks like 1/sqrt(x) as the integrand
// narrows for large x.
__device__ double bessel_k_scaled(double nu, double x) {
    const double h = fmin(0.15, 0.7 / sqrt(x));
    double s = 0.5;
    for (int k = 1; k < 4000; ++k) {
        const double t = k * h;
        const double sh = sinh(0.5 * t);
        const double term = exp(-2.0 * x * sh * sh) * cosh(nu * t);
        s += term;
        if (term < 1e-17 * s) break;
    }
    return h * s;
}

// Matern correlation at scaled distance t = d / range.
__device__ double matern_t(double t, double nu) {
    if (t <= 0.0) return 1.0;
    if (nu == 0.5) return exp(-t);
    if (nu == 1.5) {
        const double u = 1.7320508075688772935274463415058723669 * t;
        return (1.0 + u) * exp(-u);
    }
    if (nu == 2.5) {
        const double u = 2.2360679774997896964091736687312762354 * t;
        return (1.0 + u + u * u / 3.0) * exp(-u);
    }
    const double x = sqrt(2.0 * nu) * t;
    const double lg = (1.0 - nu) * 0.69314718055994530941723212145817656808 - lgamma(nu) + nu * log(x) - x;
    return exp(lg) * bessel_k_scaled(nu, x);
}

__device__ double corr_lag(const MaternDev& m, double h1, double h2) {
    const double dx = h2 * m.dx2, dy = h1 * m.dx1;  // column (x), row (y) displacements
    const double a = dx * m.ca + dy * m.sa;
    const double b = -dx * m.sa + dy * m.ca;
    const double d = sqrt(a * a + (m.ratio * b) * (m.ratio * b));
    return matern_t(d / m.range, m.nu);
}

// c[l1][l2] at the wrapped lags; mean over both aliases on a Nyquist line.
__global__ void k_lag_grid(double* __restrict__ c, int N1, int N2, MaternDev m) {
    const int64_t n = (int64_t)N1 * N2;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int l1 = (int)(idx / N2), l2 = (int)(idx - (int64_t)l1 * N2);
        const bool ny1 = (N1 % 2 == 0) && (2 * l1 == N1);
        const bool ny2 = (N2 % 2 == 0) && (2 * l2 == N2);
        const double h1 = (2 * l1 <= N1) ? l1 : l1 - N1;
        const double h2 = (2 * l2 <= N2) ? l2 : l2 - N2;
        double v;
        if (!ny1 && !ny2) {
            v = corr_lag(m, h1, h2);
        } else if (ny1 && !ny2) {
            v = 0.5 * (corr_lag(m, h1, h2) + corr_lag(m, -h1, h2));
        } else if (!ny1 && ny2) {
            v = 0.5 * (corr_lag(m, h1, h2) + corr_lag(m, h1, -h2));
        } else {
            v = 0.25 * (corr_lag(m, h1, h2) + corr_lag(m, h1, -h2) + corr_lag(m, -h1, h2) +
                        corr_lag(m, -h1, -h2));
        }
        c[idx] = v;
    }
}

// ---------------------------------------------------------------------------
// Stage kernels
// ---------------------------------------------------------------------------
struct StageAArgs {
    const void* in;
    int64_t in_vstride;
    int in_rstride;
    MaskView mask;
    int rows_in, row_len;
    int log2M;
    int RT, log2RT;
    void* Y;
    int ldY;
    int64_t Y_vstride;
    uint64_t seed;
    int stream0;
};

template <typename R, int VPT, int IN>
__global__ void __launch_bounds__(1024) k_stage_a(StageAArgs a, const cpx<R>* __restrict__ tw) {
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    R* ldsr = reinterpret_cast<R*>(smem_raw);
    const int M = 1 << a.log2M;
    const int S = M + 1;  // LDS row stride (complex elements)
    const int tid = threadIdx.x, nt = blockDim.x;
    const int row0 = blockIdx.x * a.RT;
    const int vec = blockIdx.y;

    for (int i = tid; i < a.RT * S; i += nt) lds[i] = cpx<R>{(R)0, (R)0};
    __syncthreads();
    const int total = a.RT * a.row_len;
    for (int idx = tid; idx < total; idx += nt) {
        const int rr = idx / a.row_len;
        const int j = idx - rr * a.row_len;
        const int row = row0 + rr;
        if (row >= a.rows_in) continue;
        R val;
        if constexpr (IN == IN_COMPACT) {
            int64_t c;
            if (!mask_lookup(a.mask, row, j, c)) continue;
            val = reinterpret_cast<const R*>(a.in)[vec * a.in_vstride + c];
        } else if constexpr (IN == IN_DENSE) {
            val = (R) reinterpret_cast<const double*>(a.in)[vec * a.in_vstride + (int64_t)row * a.in_rstride + j];
        } else {
            val = (R)philox_normal((uint32_t)(row * a.in_rstride + j), (uint32_t)(a.stream0 + vec),
                                   DOMAIN_FIELD, a.seed);
        }
        ldsr[2 * rr * S + j] = val;
    }
    __syncthreads();
    fft_lds<R, false, VPT>(lds, a.log2M, S, tid, nt, tw);

    cpx<R>* Y = reinterpret_cast<cpx<R>*>(a.Y) + vec * a.Y_vstride;
    const int nout = a.RT * (M + 1);
    for (int o = tid; o < nout; o += nt) {
        const int rr = o & (a.RT - 1);
        const int k = o >> a.log2RT;
        const cpx<R> zk = lds[rr * S + (k & (M - 1))];
        const cpx<R> zc = cconj(lds[rr * S + ((M - k) & (M - 1))]);
        const cpx<R> w = twiddle<R, false>(tw, k, a.log2M + 1);
        const cpx<R> s = cadd(zk, zc);
        const cpx<R> wd = cmul(w, csub(zk, zc));
        // X[k] = (s - i w d) / 2
        Y[(int64_t)k * a.ldY + row0 + rr] = cpx<R>{(R)0.5 * (s.x + wd.y), (R)0.5 * (s.y - wd.x)};
    }
}

enum { B_CONV = 0, B_SPEC = 1 };

struct StageBArgs {
    void* Y;
    int ldY;
    int64_t Y_vstride;
    int ncols;
    int rows_in, rows_out;
    int log2N1;
    int CB;
    const void* lam;
    int64_t lam_tstride;
    int vecs_per_theta;
    double* spec_out;
};

template <typename R, int VPT, int MODE>
__global__ void __launch_bounds__(1024) k_stage_b(StageBArgs a, const cpx<R>* __restrict__ tw) {
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int N1 = 1 << a.log2N1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int col0 = blockIdx.x * a.CB;
    const int vec = blockIdx.y;
    cpx<R>* Y = reinterpret_cast<cpx<R>*>(a.Y) + vec * a.Y_vstride;
    const int n = a.CB * N1;

    for (int i = tid; i < n; i += nt) {
        const int c = i >> a.log2N1, r = i & (N1 - 1);
        const int col = col0 + c;
        cpx<R> v{(R)0, (R)0};
        if (col < a.ncols && r < a.rows_in) v = Y[(int64_t)col * a.ldY + r];
        lds[i] = v;
    }
    __syncthreads();
    fft_lds<R, false, VPT>(lds, a.log2N1, N1, tid, nt, tw);
    if constexpr (MODE == B_SPEC) {
        for (int i = tid; i < n; i += nt) {
            const int c = i >> a.log2N1, r = i & (N1 - 1);
            const int col = col0 + c;
            if (col < a.ncols) a.spec_out[(int64_t)col * N1 + r] = (double)lds[i].x;
        }
        return;
    } else {
        const R* lam = reinterpret_cast<const R*>(a.lam) + (int64_t)(vec / a.vecs_per_theta) * a.lam_tstride;
        for (int i = tid; i < n; i += nt) {
            const int c = i >> a.log2N1, r = i & (N1 - 1);
            const int col = col0 + c;
            const R l = (col < a.ncols) ? lam[(int64_t)col * N1 + r] : (R)0;
            lds[i] = cscale(lds[i], l);
        }
        __syncthreads();
        fft_lds<R, true, VPT>(lds, a.log2N1, N1, tid, nt, tw);
        for (int i = tid; i < n; i += nt) {
            const int c = i >> a.log2N1, r = i & (N1 - 1);
            const int col = col0 + c;
            if (col < a.ncols && r < a.rows_out) Y[(int64_t)col * a.ldY + r] = lds[i];
        }
    }
}

struct StageCArgs {
    const void* Y;
    int ldY;
    int64_t Y_vstride;
    int rows_out, cols_out;
    int log2M;
    int RT, log2RT;
    MaskView mask;
    const void* vin;
    int64_t vin_vstride;
    const double* eta;
    int vecs_per_theta;
    void* out;
    int64_t out_vstride;
    double scale;
};

template <typename R, int VPT, int OUT>
__global__ void __launch_bounds__(1024) k_stage_c(StageCArgs a, const cpx<R>* __restrict__ tw) {
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const R* ldsr = reinterpret_cast<const R*>(smem_raw);
    const int M = 1 << a.log2M;
    const int S = M + 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int row0 = blockIdx.x * a.RT;
    const int vec = blockIdx.y;
    const cpx<R>* Y = reinterpret_cast<const cpx<R>*>(a.Y) + vec * a.Y_vstride;

    const int nin = a.RT * (M + 1);
    for (int o = tid; o < nin; o += nt) {
        const int rr = o & (a.RT - 1);
        const int k = o >> a.log2RT;
        const int row = row0 + rr;
        lds[rr * S + k] = (row < a.rows_out) ? Y[(int64_t)k * a.ldY + row] : cpx<R>{(R)0, (R)0};
    }
    __syncthreads();
    // merge the even/odd split: Z[k] = (X[k] + X*[M-k]) + i W^{-k} (X[k] - X*[M-k]),
    // done for k and M - k together so the update is in place.
    const int half = M / 2;
    const int npair = a.RT * (half + 1);
    for (int o = tid; o < npair; o += nt) {
        const int rr = o & (a.RT - 1);
        const int k = o >> a.log2RT;
        cpx<R>* rowp = lds + rr * S;
        const cpx<R> xk = rowp[k];
        const cpx<R> xm = rowp[M - k];
        {
            const cpx<R> s = cadd(xk, cconj(xm));
            const cpx<R> d = cmul(twiddle<R, true>(tw, k, a.log2M + 1), csub(xk, cconj(xm)));
            rowp[k] = cpx<R>{s.x - d.y, s.y + d.x};
        }
        if (k > 0 && k < M - k) {
            const cpx<R> s = cadd(xm, cconj(xk));
            const cpx<R> d = cmul(twiddle<R, true>(tw, M - k, a.log2M + 1), csub(xm, cconj(xk)));
            rowp[M - k] = cpx<R>{s.x - d.y, s.y + d.x};
        }
    }
    __syncthreads();
    fft_lds<R, true, VPT>(lds, a.log2M, S, tid, nt, tw);

    const int total = a.RT * a.cols_out;
    const int theta = vec / a.vecs_per_theta;
    for (int idx = tid; idx < total; idx += nt) {
        const int rr = idx / a.cols_out;
        const int j = idx - rr * a.cols_out;
        const int row = row0 + rr;
        if (row >= a.rows_out) continue;
        const R x = ldsr[2 * rr * S + j];
        if constexpr (OUT == OUT_COMPACT) {
            int64_t c;
            if (!mask_lookup(a.mask, row, j, c)) continue;
            const R vi = reinterpret_cast<const R*>(a.vin)[vec * a.vin_vstride + c];
            reinterpret_cast<R*>(a.out)[vec * a.out_vstride + c] = x + (R)a.eta[theta] * vi;
        } else {
            reinterpret_cast<R*>(a.out)[vec * a.out_vstride + (int64_t)row * a.cols_out + j] = (R)a.scale * x;
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

struct RowTiling {
    int RT, VPT, threads;
    size_t lds;
};

// Rows per tile: transposed writes in runs of RT * sizeof(cpx) = 64 bytes
// where LDS allows, at most 1024 threads per workgroup.
template <typename R>
static RowTiling row_tiling(int M) {
    const int cs = (int)sizeof(cpx<R>);
    int RT = 64 / cs;
    while (RT > 1 && (size_t)RT * (M + 1) * cs > 131072) RT /= 2;
    int VPT = 8;
    while (RT * M / VPT > 1024) VPT *= 2;
    while (RT * M / VPT < 256 && RT < 64) RT *= 2;
    RowTiling t;
    t.RT = RT;
    t.VPT = VPT;
    t.threads = RT * M / VPT;
    t.lds = (size_t)RT * (M + 1) * cs;
    return t;
}

template <typename R>
static int col_batch(int N1) {
    // 256 threads (VPT = 8) per workgroup where the column is short
    int CB = 2048 / N1;
    return CB < 1 ? 1 : CB;
}

// Raise a kernel's dynamic LDS limit once per kernel (and size).
template <typename K>
static void set_lds(K kernel, size_t bytes) {
    static std::mutex mu;
    static std::unordered_map<const void*, size_t> done;
    const void* key = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> g(mu);
    auto it = done.find(key);
    if (it != done.end() && it->second >= bytes) return;
    KRY_HIP(hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done[key] = bytes;
}

template <typename R>
static const cpx<R>* twiddles(Ctx& c);
template <>
const cpx<double>* twiddles<double>(Ctx& c) { return c.tw64; }
template <>
const cpx<float>* twiddles<float>(Ctx& c) { return c.tw32; }

template <typename R, int VPT, int IN>
static void launch_a(const StageAArgs& a, dim3 grid, int threads, size_t lds, const cpx<R>* tw, hipStream_t st) {
    auto k = k_stage_a<R, VPT, IN>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads), lds, st, a, tw);
    KRY_HIP(hipGetLastError());
}

template <typename R, int VPT, int OUT>
static void launch_c(const StageCArgs& a, dim3 grid, int threads, size_t lds, const cpx<R>* tw, hipStream_t st) {
    auto k = k_stage_c<R, VPT, OUT>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads), lds, st, a, tw);
    KRY_HIP(hipGetLastError());
}

template <typename R, int MODE>
static void launch_b(const StageBArgs& a, dim3 grid, int threads, size_t lds, const cpx<R>* tw, hipStream_t st) {
    auto k = k_stage_b<R, 8, MODE>;
    set_lds(k, lds);
    hipLaunchKernelGGL(k, grid, dim3(threads), lds, st, a, tw);
    KRY_HIP(hipGetLastError());
}

template <typename R>
static void run_stage_a(Problem& P, const ConvSpec& s, cpx<R>* Y, int ldY, int64_t Yvs, hipStream_t st) {
    const int M = s.N2 / 2;
    const RowTiling t = row_tiling<R>(M);
    StageAArgs a;
    a.in = s.in;
    a.in_vstride = s.in_vstride;
    a.in_rstride = s.in_rstride;
    a.mask = P.mask_view();
    a.rows_in = s.rows_in;
    a.row_len = s.row_len;
    a.log2M = ilog2(M);
    a.RT = t.RT;
    a.log2RT = ilog2(t.RT);
    a.Y = Y;
    a.ldY = ldY;
    a.Y_vstride = Yvs;
    a.seed = s.seed;
    a.stream0 = s.stream0;
    dim3 grid((s.rows_in + t.RT - 1) / t.RT, s.nvec);
    const cpx<R>* tw = twiddles<R>(*P.ctx);
#define KRY_A(V, I) launch_a<R, V, I>(a, grid, t.threads, t.lds, tw, st)
    if (t.VPT == 8) {
        if (s.in_mode == IN_COMPACT) KRY_A(8, IN_COMPACT);
        else if (s.in_mode == IN_DENSE) KRY_A(8, IN_DENSE);
        else KRY_A(8, IN_NOISE);
    } else {
        if (s.in_mode == IN_COMPACT) KRY_A(16, IN_COMPACT);
        else if (s.in_mode == IN_DENSE) KRY_A(16, IN_DENSE);
        else KRY_A(16, IN_NOISE);
    }
#undef KRY_A
}

template <typename R>
static void run_stage_b(Problem& P, int N1, int M, int nvec, cpx<R>* Y, int ldY, int64_t Yvs, int rows_in,
                        int rows_out, const void* lam, int64_t lam_tstride, int vpt, double* spec_out,
                        hipStream_t st) {
    const int CB = col_batch<R>(N1);
    StageBArgs b;
    b.Y = Y;
    b.ldY = ldY;
    b.Y_vstride = Yvs;
    b.ncols = M + 1;
    b.rows_in = rows_in;
    b.rows_out = rows_out;
    b.log2N1 = ilog2(N1);
    b.CB = CB;
    b.lam = lam;
    b.lam_tstride = lam_tstride;
    b.vecs_per_theta = vpt;
    b.spec_out = spec_out;
    const int threads = CB * N1 / 8;
    const size_t lds = (size_t)CB * N1 * sizeof(cpx<R>);
    dim3 grid((M + 1 + CB - 1) / CB, nvec);
    const cpx<R>* tw = twiddles<R>(*P.ctx);
    if (spec_out) launch_b<R, B_SPEC>(b, grid, threads, lds, tw, st);
    else launch_b<R, B_CONV>(b, grid, threads, lds, tw, st);
}

template <typename R>
void conv_apply(Problem& P, const ConvSpec& s, hipStream_t st) {
    KRY_REQUIRE(s.N1 >= 16 && s.N2 >= 16 && s.N1 <= 8192 && s.N2 <= 8192, "torus size out of range");
    KRY_REQUIRE((s.N1 & (s.N1 - 1)) == 0 && (s.N2 & (s.N2 - 1)) == 0, "torus sizes must be powers of two");
    KRY_REQUIRE(s.rows_in <= s.N1 && s.row_len <= s.N2 && s.rows_out <= s.N1 && s.cols_out <= s.N2,
                "block larger than the torus");
    if (s.nvec <= 0) return;
    const int M = s.N2 / 2;
    const RowTiling ta = row_tiling<R>(M);
    const int rows_max = s.rows_in > s.rows_out ? s.rows_in : s.rows_out;
    const int ldY = ((rows_max + ta.RT - 1) / ta.RT) * ta.RT;
    const int64_t Yvs = (int64_t)(M + 1) * ldY;
    P.Y.ensure(*P.ctx, (size_t)Yvs * s.nvec * sizeof(cpx<R>));
    cpx<R>* Y = P.Y.as<cpx<R>>();

    StageProfile& pr = P.ctx->prof;
    std::array<int, 5> rec{};
    auto mark = [&](int slot) {
        if (!pr.on) return;
        if (pr.next == pr.pool.size()) {
            hipEvent_t e;
            KRY_HIP(hipEventCreate(&e));
            pr.pool.push_back(e);
        }
        rec[slot] = (int)pr.next;
        KRY_HIP(hipEventRecord(pr.pool[pr.next++], st));
    };
    mark(0);
    run_stage_a<R>(P, s, Y, ldY, Yvs, st);
    mark(1);
    run_stage_b<R>(P, s.N1, M, s.nvec, Y, ldY, Yvs, s.rows_in, s.rows_out, s.lam, s.lam_tstride,
                   s.vecs_per_theta, nullptr, st);
    mark(2);

    StageCArgs c;
    c.Y = Y;
    c.ldY = ldY;
    c.Y_vstride = Yvs;
    c.rows_out = s.rows_out;
    c.cols_out = s.cols_out;
    c.log2M = ilog2(M);
    c.RT = ta.RT;
    c.log2RT = ilog2(ta.RT);
    c.mask = P.mask_view();
    c.vin = s.vin;
    c.vin_vstride = s.vin_vstride;
    c.eta = s.eta;
    c.vecs_per_theta = s.vecs_per_theta;
    c.out = s.out;
    c.out_vstride = s.out_vstride;
    c.scale = s.scale;
    dim3 grid((s.rows_out + ta.RT - 1) / ta.RT, s.nvec);
    const cpx<R>* tw = twiddles<R>(*P.ctx);
    if (ta.VPT == 8) {
        if (s.out_mode == OUT_COMPACT) launch_c<R, 8, OUT_COMPACT>(c, grid, ta.threads, ta.lds, tw, st);
        else launch_c<R, 8, OUT_GRID>(c, grid, ta.threads, ta.lds, tw, st);
    } else {
        if (s.out_mode == OUT_COMPACT) launch_c<R, 16, OUT_COMPACT>(c, grid, ta.threads, ta.lds, tw, st);
        else launch_c<R, 16, OUT_GRID>(c, grid, ta.threads, ta.lds, tw, st);
    }
    mark(3);
    if (pr.on) {
        rec[4] = s.nvec;
        pr.recs.push_back(rec);
    }
}

template void conv_apply<double>(Problem&, const ConvSpec&, hipStream_t);
template void conv_apply<float>(Problem&, const ConvSpec&, hipStream_t);

// ---------------------------------------------------------------------------
// Lag grid and spectrum
// ---------------------------------------------------------------------------
void lag_grid_device(Ctx& c, int N1, int N2, double dx1, double dx2, const Matern& th, double* d_c,
                     hipStream_t st) {
    (void)c;
    MaternDev m;
    m.range = th.range;
    m.nu = th.nu;
    m.ratio = th.ratio;
    m.ca = std::cos(th.angle);
    m.sa = std::sin(th.angle);
    m.dx1 = dx1;
    m.dx2 = dx2;
    const int64_t n = (int64_t)N1 * N2;
    const int threads = 256;
    int64_t blocks = (n + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_lag_grid, dim3((unsigned)blocks), dim3(threads), 0, st, d_c, N1, N2, m);
    KRY_HIP(hipGetLastError());
}

// min / max over n doubles: per-block partials, then one block.
__global__ void k_minmax_partial(const double* __restrict__ x, int64_t n, double* __restrict__ part) {
    __shared__ double smin[256], smax[256];
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        lo = fmin(lo, x[i]);
        hi = fmax(hi, x[i]);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = smin[0];
        part[2 * blockIdx.x + 1] = smax[0];
    }
}

__global__ void k_minmax_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double lo = INFINITY, hi = -INFINITY;
    for (int b = 0; b < nb; ++b) {
        lo = fmin(lo, part[2 * b]);
        hi = fmax(hi, part[2 * b + 1]);
    }
    out[0] = lo;
    out[1] = hi;
}

void spectrum_device(Problem& P, int N1, int N2, const Matern& th, double* d_lam, double* lam_min,
                     double* lam_max, hipStream_t st) {
    Ctx& C = *P.ctx;
    const int M = N2 / 2;
    P.lagtmp.ensure(C, (size_t)N1 * N2 * sizeof(double));
    lag_grid_device(C, N1, N2, P.dx1, P.dx2, th, P.lagtmp.as<double>(), st);
    // stage A over every row of the lag grid, then the forward column pass
    const RowTiling ta = row_tiling<double>(M);
    const int ldY = ((N1 + ta.RT - 1) / ta.RT) * ta.RT;
    const int64_t Yvs = (int64_t)(M + 1) * ldY;
    P.spectmp.ensure(C, (size_t)Yvs * sizeof(cpx<double>) + 1024 * 2 * sizeof(double));
    cpx<double>* Y = P.spectmp.as<cpx<double>>();
    ConvSpec s;
    s.N1 = N1;
    s.N2 = N2;
    s.nvec = 1;
    s.in_mode = IN_DENSE;
    s.in = P.lagtmp.ptr;
    s.in_vstride = 0;
    s.in_rstride = N2;
    s.rows_in = N1;
    s.row_len = N2;
    run_stage_a<double>(P, s, Y, ldY, Yvs, st);
    run_stage_b<double>(P, N1, M, 1, Y, ldY, Yvs, N1, N1, nullptr, 0, 1, d_lam, st);
    // min / max
    double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(P.spectmp.ptr) + (size_t)Yvs * sizeof(cpx<double>));
    const int64_t n = (int64_t)(M + 1) * N1;
    int nb = (int)((n + 255) / 256);
    if (nb > 512) nb = 512;
    hipLaunchKernelGGL(k_minmax_partial, dim3(nb), dim3(256), 0, st, d_lam, n, part);
    KRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(64), 0, st, part, nb, part + 2 * nb);
    KRY_HIP(hipGetLastError());
    double mm[2];
    KRY_HIP(hipMemcpyAsync(mm, part + 2 * nb, sizeof(mm), hipMemcpyDeviceToHost, st));
    KRY_HIP(hipStreamSynchronize(st));
    *lam_min = mm[0];
    *lam_max = mm[1];
}

__global__ void k_spectrum_scale(const double* __restrict__ lam, int64_t n, double s, int sqrt_clip,
                                 double* __restrict__ o64, float* __restrict__ o32) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = lam[i];
        if (sqrt_clip) v = sqrt(fmax(v, 0.0));
        v *= s;
        if (o64) o64[i] = v;
        if (o32) o32[i] = (float)v;
    }
}

void spectrum_scale(const double* lam, int64_t n, double s, bool sqrt_clip, double* out64, float* out32,
                    hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_spectrum_scale, dim3((unsigned)blocks), dim3(256), 0, st, lam, n, s, sqrt_clip ? 1 : 0,
                       out64, out32);
    KRY_HIP(hipGetLastError());
}

static bool same_theta(const Matern& a, const Matern& b) {
    return a.range == b.range && a.nu == b.nu && a.ratio == b.ratio && a.angle == b.angle;
}

Spectrum& problem_spectrum(Problem& P, const Matern& th, hipStream_t st) {
    Spectrum& S = P.spec;
    if (S.valid && same_theta(S.theta, th)) return S;
    S.valid = false;
    const int64_t n = (int64_t)(P.N2 / 2 + 1) * P.N1;
    S.s64.ensure(*P.ctx, n * sizeof(double));
    S.s32.ensure(*P.ctx, n * sizeof(float));
    double lo, hi;
    spectrum_device(P, P.N1, P.N2, th, S.s64.as<double>(), &lo, &hi, st);
    spectrum_scale(S.s64.as<double>(), n, 1.0 / ((double)P.N1 * P.N2), false, S.s64.as<double>(), S.s32.as<float>(),
                   st);
    S.theta = th;
    S.lam_min = lo;
    S.lam_max = hi;
    S.valid = true;
    return S;
}

}  // namespace kry
