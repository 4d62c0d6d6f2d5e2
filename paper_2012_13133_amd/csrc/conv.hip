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
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "fftk.hpp"
#include "fftm.hpp"
#include "internal.hpp"

namespace kry {

// ---------------------------------------------------------------------------
// Matern correlation (Sec. 2) on the device
// ---------------------------------------------------------------------------
struct MaternDev {
    double range, nu, ratio, ca, sa, dx1, dx2;
    int drange;  // 1: the derivative with respect to the range instead
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

// Derivative of the Matern correlation with respect to the range at scaled
// distance t = d / range: with x = sqrt(2 nu) t, d/dx [x^nu K_nu(x)] =
// -x^nu K_{nu-1}(x) and dx/drange = -x / range, so the derivative is
// 2^(1-nu) / Gamma(nu) x^(nu+1) K_{nu-1}(x) / range (K of order |nu - 1|);
// elementary forms for nu = 1/2, 3/2, 5/2.
__device__ double matern_drange_t(double t, double nu, double range) {
    if (t <= 0.0) return 0.0;
    if (nu == 0.5) return t * exp(-t) / range;
    if (nu == 1.5) {
        const double u = 1.7320508075688772935274463415058723669 * t;
        return u * u * exp(-u) / range;
    }
    if (nu == 2.5) {
        const double u = 2.2360679774997896964091736687312762354 * t;
        return u * u * (1.0 + u) * exp(-u) / (3.0 * range);
    }
    const double x = sqrt(2.0 * nu) * t;
    const double lg = (1.0 - nu) * 0.69314718055994530941723212145817656808 - lgamma(nu) + nu * log(x) - x;
    return exp(lg) * x * bessel_k_scaled(fabs(nu - 1.0), x) / range;
}

__device__ double corr_lag(const MaternDev& m, double h1, double h2) {
    const double dx = h2 * m.dx2, dy = h1 * m.dx1;  // column (x), row (y) displacements
    const double a = dx * m.ca + dy * m.sa;
    const double b = -dx * m.sa + dy * m.ca;
    const double d = sqrt(a * a + (m.ratio * b) * (m.ratio * b));
    return m.drange ? matern_drange_t(d / m.range, m.nu, m.range) : matern_t(d / m.range, m.nu);
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
// Stage kernels (compile-time plans, register hand-off; see fftk.hpp)
// ---------------------------------------------------------------------------

// Largest workgroup of a row-stage kernel: rows of 8 VT values per thread;
// FP32 kernels with two values sets per thread take tiles of 16 rows (128-byte
// runs of the transposed intermediate) in 1024 threads, FP64 ones 512.
template <typename R>
constexpr int row_threads_max(int vt) { return vt > 1 && sizeof(R) == 8 ? 512 : 1024; }
// (mixed-radix rows: FP64 passes hold more values per thread than radix 8)
template <typename R>
constexpr int row_threads_mixed() { return sizeof(R) == 8 ? 512 : 1024; }
struct StageAArgs {
    const void* in;
    int64_t in_vstride;
    int in_rstride;
    MaskView mask;
    int rows_in, row_len;
    int RT, log2RT;
    void* Y;
    int ldY;
    int64_t Y_vstride;
    uint64_t seed;
    int stream0;
    int vec0;
    const ProbDesc* tab;  // several problems: per-vector mask and block
    int tab_vpp;
    const int* active;    // per-vector skip flags (nullable)
    const void* upd_r;    // direction update of the compact input (nullable; see ConvSpec)
    const double* upd_beta;
};

// Value of input column c of a row (0 beyond the data or off the mask).
template <typename R, int IN>
__device__ __forceinline__ void load_pair(const StageAArgs& a, const MaskView& mask, int row_len, int vec, int row,
                                          int c0, cpx<R>& out) {
    out = cpx<R>{(R)0, (R)0};
    if (c0 >= row_len) return;
    if constexpr (IN == IN_COMPACT) {
        const int w = row * mask.words_per_row + (c0 >> 5);
        const uint32_t word = mask.bits[w];
        const uint32_t b0 = 1u << (c0 & 31);
        const uint32_t pair = word & (b0 | (b0 << 1));
        if (!pair) return;
        const R* vin = reinterpret_cast<const R*>(a.in) + vec * a.in_vstride;
        int64_t ci = (int64_t)mask.base[w] + __popc(word & (b0 - 1u));
        if (word & b0) out.x = vin[ci++];
        if (word & (b0 << 1)) out.y = vin[ci];
    } else if constexpr (IN == IN_DENSE) {
        const R* src = reinterpret_cast<const R*>(a.in) + vec * a.in_vstride + (int64_t)row * a.in_rstride;
        out.x = src[c0];
        if (c0 + 1 < row_len) out.y = src[c0 + 1];
    } else {
        const uint32_t idx = (uint32_t)(row * a.in_rstride + c0);
        const uint32_t stream = (uint32_t)(a.stream0 + a.vec0 + vec);
        out.x = (R)philox_normal(idx, stream, DOMAIN_FIELD, a.seed);
        if (c0 + 1 < row_len) out.y = (R)philox_normal(idx + 1u, stream, DOMAIN_FIELD, a.seed);
    }
}

// The inputs of a row-forward thread: 8 VT values of row `row` at columns
// 2 (t + u TR + r T) and the next one (pairs packed as complex values), 0
// beyond the data or off the mask; with a compact input and a direction
// update (StageAArgs::upd_r), the input is updated and written back first.
template <typename R, int IN, int VT, bool LOW>
__device__ __forceinline__ void row_inputs(const StageAArgs& a, const MaskView& mask, int vec, int row, int rows_in,
                                           int row_len, int t, int TR, int T, cpx<R>* v) {
    if constexpr (IN == IN_COMPACT) {
        // every mask word and offset first, then every value: two rounds of
        // independent loads instead of a dependent chain per pair.  Pairs
        // outside the row read word 0 and element 0 and are discarded.
        constexpr int NP = LOW ? 4 : 8;
        const R* vin = reinterpret_cast<const R*>(a.in) + vec * a.in_vstride;
        uint32_t wd[VT * NP], bs[VT * NP];
#pragma unroll
        for (int u = 0; u < VT; ++u)
#pragma unroll
            for (int r = 0; r < NP; ++r) {
                const int c0 = 2 * (t + u * TR + r * T);
                const bool ok = row < rows_in && c0 < row_len;
                const uint32_t w = ok ? (uint32_t)(row * mask.words_per_row + (c0 >> 5)) : 0u;
                const uint32_t word = at32(mask.bits, w);
                bs[u * NP + r] = at32(mask.base, w);
                wd[u * NP + r] = ok ? word : 0u;
            }
        if (sizeof(R) == 8 && a.upd_r) {
            // p = r + beta p on the fly, written back: both vectors' values
            // are loaded together, then the updated ones stored
            const R* rin = reinterpret_cast<const R*>(a.upd_r) + vec * a.in_vstride;
            R* pio = const_cast<R*>(vin);
            const R b = (R)a.upd_beta[a.vec0 + vec];
            uint32_t cx[VT * NP], cy[VT * NP];
            R px[VT * NP], py[VT * NP], rx[VT * NP], ry[VT * NP];
#pragma unroll
            for (int q = 0; q < VT * NP; ++q) {
                const int u = q / NP, r = q % NP;
                const int c0 = 2 * (t + u * TR + r * T);
                const uint32_t word = wd[q];
                const uint32_t b0 = 1u << (c0 & 31);
                const bool lo = (word & b0) != 0u, hi = (word & (b0 << 1)) != 0u;
                const uint32_t ci = bs[q] + (uint32_t)__popc(word & (b0 - 1u));
                cx[q] = lo ? ci : 0u;
                cy[q] = hi ? ci + (lo ? 1u : 0u) : 0u;
                px[q] = at32(vin, cx[q]);
                py[q] = at32(vin, cy[q]);
                rx[q] = at32(rin, cx[q]);
                ry[q] = at32(rin, cy[q]);
            }
#pragma unroll
            for (int u = 0; u < VT; ++u)
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    v[u * 8 + r] = cpx<R>{(R)0, (R)0};
                    if (r >= NP) continue;
                    const int q = u * NP + r;
                    const int c0 = 2 * (t + u * TR + r * T);
                    const uint32_t word = wd[q];
                    const uint32_t b0 = 1u << (c0 & 31);
                    const bool lo = (word & b0) != 0u, hi = (word & (b0 << 1)) != 0u;
                    const R x = rx[q] + b * px[q];
                    const R y = ry[q] + b * py[q];
                    if (lo) at32(pio, cx[q]) = x;
                    if (hi) at32(pio, cy[q]) = y;
                    v[u * 8 + r] = cpx<R>{lo ? x : (R)0, hi ? y : (R)0};
                }
        } else {
#pragma unroll
        for (int u = 0; u < VT; ++u)
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                v[u * 8 + r] = cpx<R>{(R)0, (R)0};
                if (r >= NP) continue;
                const int c0 = 2 * (t + u * TR + r * T);
                const uint32_t word = wd[u * NP + r];
                const uint32_t b0 = 1u << (c0 & 31);
                const bool lo = (word & b0) != 0u, hi = (word & (b0 << 1)) != 0u;
                const uint32_t ci = bs[u * NP + r] + (uint32_t)__popc(word & (b0 - 1u));
                const R x = at32(vin, lo ? ci : 0u);
                const R y = at32(vin, hi ? ci + (lo ? 1u : 0u) : 0u);
                v[u * 8 + r] = cpx<R>{lo ? x : (R)0, hi ? y : (R)0};
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < VT; ++u)
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                v[u * 8 + r] = cpx<R>{(R)0, (R)0};
                if (LOW && r >= 4) continue;
                if (row < rows_in) load_pair<R, IN>(a, mask, row_len, vec, row, 2 * (t + u * TR + r * T), v[u * 8 + r]);
            }
    }
}

// Stage A: per row, z[m] = x[2m] + i x[2m+1] -> FFT of length M -> split into
// the real transform X[k], k = 0..M, written as Y[k][row] in RT-row runs.
// A row is transformed by TR = M / (8 VT) threads holding 8 VT values each;
// when those lie in one wavefront the passes need no workgroup barrier, and
// the only barrier is the one before the split, which mixes rows.
template <typename R, int LOG2M, int IN, int VT, bool SPLIT>
__global__ void __launch_bounds__(row_threads_max<R>(VT), (VT > 1 ? 2 : (sizeof(R) == 4 && IN == IN_COMPACT ? 8 : 4))) k_row_fwd(StageAArgs a, const cpx<R>* __restrict__ twp,
                                                                   const cpx<R>* __restrict__ twb) {
    using S = Sched<LOG2M>;
    constexpr int M = S::L, T = M / 8, PM = lpadded<cpx<R>>(M) + 1;
    constexpr int TR = T / VT;
    constexpr bool WAVE = TR <= 64;
    constexpr bool LOW = (IN == IN_COMPACT);  // row_len <= M: z[m] = 0 for m >= M/2
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x;
    const int rr = tid / TR, t = tid % TR;
    // row tiles of one vector run consecutively on one XCD, so the halves of
    // a cache line written by neighbouring tiles merge in its L2
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int row0 = (lid % gridDim.x) * a.RT;
    const int row = row0 + rr;
    const int vec = lid / gridDim.x;
    if (a.active && !a.active[vec]) return;
    MaskView mask = a.mask;
    int rows_in = a.rows_in, row_len = a.row_len;
    if (a.tab) {
        const ProbDesc& d = a.tab[(a.vec0 + vec) / a.tab_vpp];
        mask = MaskView{d.bits, d.base, d.wpr};
        rows_in = d.n1;
        row_len = d.n2;
        if (row0 >= rows_in) return;  // rows the column transform never reads
    }
    cpx<R>* buf = lds + rr * PM;
    const int nt = blockDim.x;
    cpx<R> v[8 * VT];
    row_inputs<R, IN, VT, LOW>(a, mask, vec, row, rows_in, row_len, t, TR, T, v);
    cpx<R>* Y = reinterpret_cast<cpx<R>*>(a.Y) + vec * a.Y_vstride;
    if constexpr (SPLIT) {
        // exchanges of reals (half the LDS per row); the split below reads
        // the transform's real parts, then its imaginary parts
        R* rl = reinterpret_cast<R*>(smem_raw);
        R* rbuf = rl + rr * PM;
#pragma unroll
        for (int u = 0; u < VT; ++u) pass_compute<R, LOG2M, false, 0, LOW>(v + u * 8, t + u * TR, twp);
        SplitPassesVT<R, LOG2M, false, 1, S::npass - 1, VT, WAVE>::run(v, rbuf, t, twp);
        constexpr int PF = S::npass - 1;
        constexpr int NO = 8 * VT;
        // output i of this thread: row r2 = tid mod RT, k = k0 + i TR (the
        // workgroup has RT TR threads); z_0 is copied to position M so that
        // z_{M-k} needs no wrap.  s = z_k + conj(z_{M-k}), d = z_k - conj(z_{M-k})
        // in parts; the Nyquist column k = M (s = 2 Re z_0 ...) by thread r2 < RT.
        const int r2 = tid & (a.RT - 1), k0 = tid >> a.log2RT;
        // padded positions: lpad(k0 + i TR) = lpad(k0) + i PTR and
        // lpad(M - k0 - i TR) = lpad(M - k0) - i PTR, TR being a multiple of the pad group
        constexpr int PTR = lpad_off<R>(TR);
        static_assert(TR % pad_group<R>() == 0, "row threads must be a multiple of the pad group");
        const R* bk = rl + r2 * PM + lpad<R>(k0);
        const R* bc = rl + r2 * PM + lpad<R>(M - k0);
        R sx[NO], dx[NO], nyx = (R)0, nydx = (R)0;
        lds_sync<WAVE>();
#pragma unroll
        for (int u = 0; u < VT; ++u) pass_write_part<R, LOG2M, false, PF, 0>(v + u * 8, rbuf, t + u * TR);
        if (t == 0) rbuf[lpad<R>(M)] = v[0].x;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NO; ++i) {
            const R zk = bk[i * PTR], zc = bc[-i * PTR];
            sx[i] = zk + zc;
            dx[i] = zk - zc;
        }
        if (tid < a.RT) {
            const R z0 = rl[tid * PM];
            nyx = z0 + z0;
            nydx = z0 - z0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < VT; ++u) pass_write_part<R, LOG2M, false, PF, 1>(v + u * 8, rbuf, t + u * TR);
        if (t == 0) rbuf[lpad<R>(M)] = v[0].y;
        __syncthreads();
        cpx<R>* Yr = Y + row0 + r2;
#pragma unroll
        for (int i = 0; i < NO; ++i) {
            const int k = k0 + i * TR;
            const R zk = bk[i * PTR], zc = bc[-i * PTR];
            const R sy = zk - zc, dy = zk + zc;
            const cpx<R> wd = cmul(twiddle<R, false>(twb, k, LOG2M + 1), cpx<R>{dx[i], dy});
            at32(Y, (uint32_t)(k * a.ldY + row0 + r2)) = cpx<R>{(R)0.5 * (sx[i] + wd.y), (R)0.5 * (sy - wd.x)};
        }
        if (tid < a.RT) {
            const R z0 = rl[tid * PM];
            const R sy = z0 - z0, dy = z0 + z0;
            const cpx<R> wd = cmul(twiddle<R, false>(twb, M, LOG2M + 1), cpx<R>{nydx, dy});
            at32(Y, (uint32_t)(M * a.ldY + row0 + tid)) = cpx<R>{(R)0.5 * (nyx + wd.y), (R)0.5 * (sy - wd.x)};
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < VT; ++u) {
        pass_compute<R, LOG2M, false, 0, LOW>(v + u * 8, t + u * TR, twp);
        pass_write<R, LOG2M, false, 0>(v + u * 8, buf, t + u * TR);
    }
    lds_sync<WAVE>();
    LdsPassesVT<R, LOG2M, false, 1, S::npass, VT, WAVE>::run(v, buf, t, twp);
    if constexpr (WAVE) __syncthreads();

    // split Z into the real transform X[k] = (s - i w d) / 2, k = 0..M:
    // 8 VT outputs per thread for k < M plus the Nyquist column k = M
    auto split = [&](int r2, int k, cpx<R> w) {
        const cpx<R>* bp = lds + r2 * PM;
        const cpx<R> zk = bp[lpad<cpx<R>>(k & (M - 1))];
        const cpx<R> zc = cconj(bp[lpad<cpx<R>>((M - k) & (M - 1))]);
        const cpx<R> s = cadd(zk, zc);
        const cpx<R> wd = cmul(w, csub(zk, zc));
        at32(Y, (uint32_t)(k * a.ldY + row0 + r2)) = cpx<R>{(R)0.5 * (s.x + wd.y), (R)0.5 * (s.y - wd.x)};
    };
#pragma unroll
    for (int i = 0; i < 8 * VT; ++i) {
        const int o = tid + i * nt;
        split(o & (a.RT - 1), o >> a.log2RT, twiddle<R, false>(twb, o >> a.log2RT, LOG2M + 1));
    }
    if (tid < a.RT) split(tid, M, twiddle<R, false>(twb, M, LOG2M + 1));
}

enum { B_LOW = 0, B_FULL = 1, B_SPEC = 2 };

struct StageBArgs {
    void* Y;
    int ldY;
    int64_t Y_vstride;
    int nvec;
    int ncols;
    int rows_in, rows_out;
    int CB;
    const void* lam;
    int64_t lam_tstride;
    int vecs_per_theta;
    int lam_even;         // lam even in k1 (power-of-two columns read the lower half)
    int vec0;
    double* spec_out;
    double* pw_out;       // FP64 power-of-two columns (nullable): per (vector, column) partials of p . lam p
    const ProbDesc* tab;  // several problems: per-vector rows and spectrum
    int tab_vpp;
    const int* active;    // per-vector skip flags (nullable)
};

// The quadratic form of the product, read off the spectrum: for a real x
// zero outside the observed cells, with X its forward transform on the torus
// and lam the spectrum scaled by 1 / (N1 N2), x . (Sigma_oo x) = sum over the
// whole torus of lam |X|^2; over the half spectrum, columns 0 and M once and
// the others twice (Hermitian symmetry).  All terms are non-negative (a PSD
// spectrum), so the sum has no cancellation.  A thread sums its eight values
// before the multiplication (col_qf_thread) and, once its column is written,
// the column's lanes of each wavefront are summed by a butterfly
// (col_qf_write): one partial per (column, wavefront), written to
// pw_out[vector][column][wavefront].  The order depends on the column length
// only -- not on the batch, the vectors per workgroup or the exchange form --
// and no barrier is needed.
__host__ __device__ constexpr int col_qf_waves(int log2l) { return (1 << log2l) / 8 > 64 ? (1 << log2l) / 512 : 1; }

template <int V>
__device__ __forceinline__ void col_qf_thread(const cpx<double>* v, const double* lamv, double* acc) {
#pragma unroll
    for (int u = 0; u < V; ++u) {
        acc[u] = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {  // explicit fused multiply-adds: one rounding each, the same everywhere
            const cpx<double> z = v[u * 8 + k];
            acc[u] = fma(lamv[u * 8 + k], fma(z.x, z.x, z.y * z.y), acc[u]);
        }
    }
}

template <int LOG2L, int V>
__device__ __forceinline__ void col_qf_write(const StageBArgs& a, double* acc, int t, int col, bool valid,
                                             int vbase) {
    constexpr int T = (1 << LOG2L) / 8;
    constexpr int SEG = T < 64 ? T : 64;  // lanes of one column in a wavefront
    constexpr int NW = col_qf_waves(LOG2L);
#pragma unroll
    for (int u = 0; u < V; ++u)
#pragma unroll
        for (int off = SEG / 2; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off, 64);
    if (t % SEG == 0 && valid) {
        const double wt = (col == 0 || col == a.ncols - 1) ? 1.0 : 2.0;
#pragma unroll
        for (int u = 0; u < V; ++u)
            if (vbase + u < a.nvec)
                a.pw_out[((int64_t)(a.vec0 + vbase + u) * a.ncols + col) * NW + t / SEG] = wt * acc[u];
    }
}

// Stage B: per column of the half spectrum, forward FFT of length L (rows
// beyond rows_in are zero), multiply by lam in registers, inverse FFT, keep
// rows_out rows.  Each thread carries the same column of V consecutive
// vectors, sharing twiddle and spectrum loads.  B_SPEC: forward only, real
// part to spec_out.
template <typename R, int LOG2L, int MODE, int V, bool SPLIT>
__global__ void __launch_bounds__(((1 << LOG2L) / 8 > 256 ? (1 << LOG2L) / 8 : 256)) k_col(StageBArgs a, const cpx<R>* __restrict__ twp) {
    using S = Sched<LOG2L>;
    constexpr int L = S::L, T = L / 8, PL = lpadded<cpx<R>>(L);  // per transform (complex or reals)
    constexpr bool LOW = (MODE == B_LOW);
    constexpr int LRF = S::lr(false, S::npass - 1);  // last forward radix = first inverse radix
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x;
    // (one column per workgroup when a transform has 256 or more threads: the
    // column, and with it every base address, is then uniform over the workgroup)
    const int cl = T >= 256 ? 0 : tid / T, t = T >= 256 ? tid : tid % T;
    // the vectors of one column block run consecutively on one XCD, so the
    // spectrum columns they share stay in its L2
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int col = (lid / gridDim.y) * a.CB + cl;
    const bool valid = col < a.ncols;
    const int vbase = (lid % gridDim.y) * V;  // first vector of this workgroup (within the launch)
    cpx<R>* buf = lds + cl * V * PL;
    R* rbuf = reinterpret_cast<R*>(smem_raw) + cl * V * PL;  // split exchanges: reals
    cpx<R>* Ycol = reinterpret_cast<cpx<R>*>(a.Y) + (int64_t)(valid ? col : 0) * a.ldY;
    cpx<R> v[V * 8];
    // spectrum values for this column, fetched up front so their latency
    // overlaps the forward transform (an unused slot, vbase + u >= nvec,
    // reads the last vector's spectrum, never past the end)
    R lamv[MODE == B_SPEC ? 1 : V * 8];
    if (a.active) {
        bool any = false;
#pragma unroll
        for (int u = 0; u < V; ++u) any = any || (vbase + u < a.nvec && a.active[vbase + u]);
        if (!any) return;
    }
    int rows_in[V], rows_out[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
        rows_in[u] = a.rows_in;
        rows_out[u] = a.rows_out;
        if (a.tab) {
            const ProbDesc& d = a.tab[(a.vec0 + min(vbase + u, a.nvec - 1)) / a.tab_vpp];
            rows_in[u] = d.n1;
            rows_out[u] = d.n1;
        }
    }
    if constexpr (MODE != B_SPEC) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int vl = min(vbase + u, a.nvec - 1);
            const R* lam;
            if (a.tab) {
                const ProbDesc& d = a.tab[(a.vec0 + vl) / a.tab_vpp];
                lam = reinterpret_cast<const R*>(sizeof(R) == 8 ? (const void*)d.lam64 : (const void*)d.lam32);
            } else {
                lam = reinterpret_cast<const R*>(a.lam) + (int64_t)((a.vec0 + vl) / a.vecs_per_theta) * a.lam_tstride;
            }
            lam += (int64_t)(valid ? col : 0) * L;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                // an even table is read at min(k1, N1 - k1): half the bytes
                // from memory, the mirrored reads served by the caches
                const int e = edge_pos<LOG2L, LRF>(t, k);
                lamv[u * 8 + k] = lam[a.lam_even && e > L / 2 ? L - e : e];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < V; ++u) {
        const bool vu = valid && (vbase + u < a.nvec);
        const cpx<R>* Yv = Ycol + (vbase + u) * a.Y_vstride;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int idx = t + r * T;
            v[u * 8 + r] = cpx<R>{(R)0, (R)0};
            if (LOW && r >= 4) continue;
            if (vu && idx < rows_in[u]) v[u * 8 + r] = Yv[idx];
        }
    }
    pass_compute<R, LOG2L, false, 0, LOW, V>(v, t, twp);
    if constexpr (SPLIT) {
        SplitPasses<R, LOG2L, false, 1, S::npass - 1, V>::run(v, rbuf, PL, t, twp);
    } else {
#pragma unroll
        for (int u = 0; u < V; ++u) pass_write<R, LOG2L, false, 0>(v + u * 8, buf + u * PL, t);
        __syncthreads();
        LdsPasses<R, LOG2L, false, 1, S::npass - 1, V>::run(v, buf, PL, t, twp);
#pragma unroll
        for (int u = 0; u < V; ++u) pass_read<R, LOG2L, false, S::npass - 1>(v + u * 8, buf + u * PL, t);
        pass_compute<R, LOG2L, false, S::npass - 1, false, V>(v, t, twp);
    }
    if constexpr (MODE == B_SPEC) {
        if (valid) {
#pragma unroll
            for (int k = 0; k < 8; ++k) a.spec_out[(int64_t)col * L + edge_pos<LOG2L, LRF>(t, k)] = (double)v[k].x;
        }
        return;
    } else {
        double qf[V];  // quadratic-form partials of this thread (FP64 with pw_out)
        if constexpr (sizeof(R) == 8) {
            if (a.pw_out) col_qf_thread<V>(v, lamv, qf);
        }
#pragma unroll
        for (int k = 0; k < V * 8; ++k) v[k] = cscale(v[k], lamv[k]);
        if constexpr (SPLIT) {
            pass_compute<R, LOG2L, true, 0, false, V>(v, t, twp);
            SplitPasses<R, LOG2L, true, 1, S::npass - 1, V>::run(v, rbuf, PL, t, twp);
        } else {
            __syncthreads();
            pass_compute<R, LOG2L, true, 0, false, V>(v, t, twp);
#pragma unroll
            for (int u = 0; u < V; ++u) pass_write<R, LOG2L, true, 0>(v + u * 8, buf + u * PL, t);
            __syncthreads();
            LdsPasses<R, LOG2L, true, 1, S::npass - 1, V>::run(v, buf, PL, t, twp);
#pragma unroll
            for (int u = 0; u < V; ++u) pass_read<R, LOG2L, true, S::npass - 1>(v + u * 8, buf + u * PL, t);
            pass_compute<R, LOG2L, true, S::npass - 1, false, V>(v, t, twp);
        }
#pragma unroll
        for (int u = 0; u < V; ++u) {
            if (!(valid && vbase + u < a.nvec)) continue;
            cpx<R>* Yv = Ycol + (vbase + u) * a.Y_vstride;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int idx = t + k * T;
                if (idx < rows_out[u]) Yv[idx] = v[u * 8 + k];
            }
        }
        if constexpr (sizeof(R) == 8) {
            if (a.pw_out) col_qf_write<LOG2L, V>(a, qf, t, col, valid, vbase);
        }
    }
}

struct StageCArgs {
    const void* Y;
    int ldY;
    int64_t Y_vstride;
    int rows_out, cols_out;
    int RT, log2RT;
    MaskView mask;
    const void* vin;
    int64_t vin_vstride;
    const double* eta;
    int vecs_per_theta;
    int vec0;
    void* out;
    int64_t out_vstride;
    double scale;
    const ProbDesc* tab;  // several problems: per-vector mask and block;
    int tab_vpp;          // compact outputs are zero from the problem's count
                          // up to out_vstride
    const int* active;    // per-vector skip flags (nullable)
};

// Compact indices of a row-inverse thread's output cells (columns 2 m and
// 2 m + 1 for its values, m = pos(k)), looked up before the transform so the
// loads overlap it; 2 bits per value in obits: which of the two is observed.
template <int OUT, int NV, typename PosF>
__device__ __forceinline__ void row_output_cells(const MaskView& mask, int row, int rows_out, int cols_out,
                                                 int32_t* oci, uint64_t& obits, PosF pos) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        oci[k] = 0;
        if constexpr (OUT == OUT_COMPACT) {
            const int c0 = 2 * pos(k);
            if (row < rows_out && c0 < cols_out) {
                const uint32_t w = (uint32_t)(row * mask.words_per_row + (c0 >> 5));
                const uint32_t word = at32(mask.bits, w);
                const uint32_t b0 = 1u << (c0 & 31);
                obits |= (uint64_t)((word & b0 ? 1u : 0u) | (word & (b0 << 1) ? 2u : 0u)) << (2 * k);
                oci[k] = (int32_t)(at32(mask.base, w) + __popc(word & (b0 - 1u)));
            }
        }
    }
}

// A row-inverse thread's outputs: x[2m], x[2m+1] = Re, Im of value k (m =
// pos(k)) to the observed cells plus eta v, or to the grid row scaled.
template <typename R, int OUT, int NV, typename PosF>
__device__ __forceinline__ void row_outputs(const StageCArgs& a, int row, int cols_out, int vec, const int32_t* oci,
                                            uint64_t obits, const cpx<R>* v, PosF pos) {
    const int theta = (a.vec0 + vec) / a.vecs_per_theta;
    // outputs in groups of two values: the group's nugget-term inputs are
    // loaded together (none when eta = 0), then its stores go out
    constexpr int GK = 2;
    const R e = (OUT == OUT_COMPACT && a.vin) ? (R)a.eta[theta] : (R)0;
    const R* vi = reinterpret_cast<const R*>(a.vin) + vec * a.vin_vstride;
    R* oc = reinterpret_cast<R*>(a.out) + vec * a.out_vstride;
#pragma unroll
    for (int k0 = 0; k0 < NV; k0 += GK) {
        R vx[GK], vy[GK];
#pragma unroll
        for (int g = 0; g < GK; ++g) {
            vx[g] = (R)0;
            vy[g] = (R)0;
        }
        if constexpr (OUT == OUT_COMPACT) {
            if (e != (R)0) {
#pragma unroll
                for (int g = 0; g < GK; ++g) {
                    const uint32_t b = (uint32_t)(obits >> (2 * (k0 + g))) & 3u;
                    const uint32_t ci = (uint32_t)oci[k0 + g];
                    const R x = at32(vi, (b & 1u) ? ci : 0u);
                    const R y = at32(vi, (b & 2u) ? ci + (b & 1u) : 0u);
                    vx[g] = (b & 1u) ? x : (R)0;
                    vy[g] = (b & 2u) ? y : (R)0;
                }
            }
        }
#pragma unroll
        for (int g = 0; g < GK; ++g) {
            const int k = k0 + g;
            const int m = pos(k);
            const int c0 = 2 * m;
            if (c0 >= cols_out) continue;
            if constexpr (OUT == OUT_COMPACT) {
                const uint32_t b = (uint32_t)(obits >> (2 * k)) & 3u;
                if (!b) continue;
                uint32_t ci = (uint32_t)oci[k];
                if (b & 1u) {
                    at32(oc, ci) = v[k].x + e * vx[g];
                    ++ci;
                }
                if (b & 2u) at32(oc, ci) = v[k].y + e * vy[g];
            } else {
                R* o = reinterpret_cast<R*>(a.out) + vec * a.out_vstride;
                const uint32_t g0 = (uint32_t)(row * cols_out + c0);
                at32(o, g0) = (R)a.scale * v[k].x;
                if (c0 + 1 < cols_out) at32(o, g0 + 1) = (R)a.scale * v[k].y;
            }
        }
    }
}

// Stage C: read RT-row runs of X[k], k = 0..M, merge the even/odd split into
// Z[k] = (X[k] + X*[M-k]) + i W^{-k} (X[k] - X*[M-k]), inverse FFT of length M,
// then x[2m], x[2m+1] = Re, Im z[m] go to the observed cells (+ eta v) or the
// grid.  Row threads as in stage A: one workgroup barrier after the tile
// load; the merge is folded into the first pass's reads.
template <typename R, int LOG2M, int OUT, int VT, bool SPLIT>
__global__ void __launch_bounds__(row_threads_max<R>(VT), (VT > 1 ? 2 : (sizeof(R) == 4 ? 8 : 4))) k_row_inv(StageCArgs a, const cpx<R>* __restrict__ twp,
                                                                   const cpx<R>* __restrict__ twb) {
    using S = Sched<LOG2M>;
    constexpr int M = S::L, T = M / 8, PM = lpadded<cpx<R>>(M) + 1;
    constexpr int TR = T / VT;
    constexpr bool WAVE = TR <= 64;
    constexpr int NV = 8 * VT;  // values per thread
    constexpr int LRL = S::lr(true, S::npass - 1);
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x;
    // neighbouring row tiles on one XCD share the cache lines of their runs
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int tile = lid % gridDim.x;
    const int row0 = tile * a.RT;
    const int vec = lid / gridDim.x;
    const cpx<R>* Y = reinterpret_cast<const cpx<R>*>(a.Y) + vec * a.Y_vstride;
    const int rr = tid / TR, t = tid % TR;
    const int row = row0 + rr;
    if (a.active && !a.active[vec]) return;
    MaskView mask = a.mask;
    int rows_out = a.rows_out, cols_out = a.cols_out;
    if (a.tab) {
        const ProbDesc& d = a.tab[(a.vec0 + vec) / a.tab_vpp];
        mask = MaskView{d.bits, d.base, d.wpr};
        rows_out = d.n1;
        cols_out = d.n2;
        if constexpr (OUT == OUT_COMPACT) {
            // this tile's share of the zero padding [p, out_vstride)
            const int64_t len = a.out_vstride - d.p;
            const int64_t per = (len + gridDim.x - 1) / gridDim.x;
            const int64_t b = d.p + tile * per, e = min(b + per, a.out_vstride);
            R* o = reinterpret_cast<R*>(a.out) + vec * a.out_vstride;
            for (int64_t i = b + tid; i < e; i += blockDim.x) o[i] = (R)0;
        }
        if (row0 >= rows_out) return;  // rows past this problem's block
    }
    // Output cells of this thread (columns 2m, 2m+1 for its values m) do not
    // depend on the transform: look up their compact indices now, so the
    // loads overlap the transform.
    int32_t oci[NV];
    uint64_t obits = 0u;  // 2 bits per value: columns 2m and 2m+1 observed
    row_output_cells<OUT, NV>(mask, row, rows_out, cols_out, oci, obits,
                              [&](int k) { return edge_pos<LOG2M, LRL>(t + (k / 8) * TR, k % 8); });
    cpx<R> v[NV];
    if constexpr (SPLIT) {
        // the tile through a buffer of reals (half the LDS per row): real
        // parts, then imaginary parts, each merged as it is read; the passes
        // exchange reals the same way
        R* rl = reinterpret_cast<R*>(smem_raw);
        R* rbuf = rl + rr * PM;
        // tile value i of this thread: row r2 = tid mod RT, k = k0 + i TR
        // (the workgroup has RT TR threads)
        const int r2 = tid & (a.RT - 1), k0 = tid >> a.log2RT;
        // padded positions lpad(k0 + i TR) = lpad(k0) + i PTR (TR a multiple of the pad group)
        constexpr int PTR = lpad_off<R>(TR);
        static_assert(TR % pad_group<R>() == 0, "row threads must be a multiple of the pad group");
        R* tl = rl + r2 * PM + lpad<R>(k0);
        const bool rin = row0 + r2 < rows_out;
        const cpx<R>* Yr = Y + row0 + r2;
        cpx<R> tv[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            tv[i] = rin ? at32(Y, (uint32_t)((k0 + i * TR) * a.ldY + row0 + r2)) : cpx<R>{(R)0, (R)0};
        const cpx<R> ny = (tid < a.RT && row0 + tid < rows_out) ? at32(Y, (uint32_t)(M * a.ldY + row0 + tid))
                                                                 : cpx<R>{(R)0, (R)0};
#pragma unroll
        for (int i = 0; i < NV; ++i) tl[i * PTR] = tv[i].x;
        if (tid < a.RT) rl[tid * PM + lpad<R>(M)] = ny.x;
        __syncthreads();
        // Z[k] = (X[k] + X*[M-k]) + i W^{-k} (X[k] - X*[M-k]) at the first
        // inverse pass's input positions: s = X[k] + X*[M-k], e = X[k] - X*[M-k]
        constexpr int R0 = 1 << S::lr(true, 0);
        constexpr int Q0 = M / R0;
        // positions k = t + c with c = u TR + b T + r Q0 a multiple of the pad group:
        // lpad(t + c) = lpad(t) + lpad_off(c), lpad(M - t - c) = lpad(M - t) - lpad_off(c)
        constexpr int G = pad_group<R>();
        static_assert(TR % G == 0 && T % G == 0 && Q0 % G == 0, "merge offsets must be multiples of the pad group");
        const R* rk = rbuf + lpad<R>(t);
        const R* rm = rbuf + lpad<R>(M - t);
        R sx[NV], ex[NV];
#pragma unroll
        for (int u = 0; u < VT; ++u)
#pragma unroll
            for (int b = 0; b < 8 / R0; ++b)
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    const int c = u * TR + b * T + r * Q0, q = u * 8 + b * R0 + r;
                    const R xk = rk[lpad_off<R>(c)], xm = rm[-lpad_off<R>(c)];
                    sx[q] = xk + xm;
                    ex[q] = xk - xm;
                }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) tl[i * PTR] = tv[i].y;
        if (tid < a.RT) rl[tid * PM + lpad<R>(M)] = ny.y;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < VT; ++u)
#pragma unroll
            for (int b = 0; b < 8 / R0; ++b)
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    const int c = u * TR + b * T + r * Q0, q = u * 8 + b * R0 + r;
                    const int k = t + c;
                    const R xk = rk[lpad_off<R>(c)], xm = rm[-lpad_off<R>(c)];
                    const R sy = xk - xm, ey = xk + xm;
                    const cpx<R> d = cmul(twiddle<R, true>(twb, k, LOG2M + 1), cpx<R>{ex[q], ey});
                    v[q] = cpx<R>{sx[q] - d.y, sy + d.x};
                }
#pragma unroll
        for (int u = 0; u < VT; ++u) pass_compute<R, LOG2M, true, 0>(v + u * 8, t + u * TR, twp);
        SplitPassesVT<R, LOG2M, true, 1, S::npass - 1, VT, WAVE>::run(v, rbuf, t, twp);
    } else {
        // the tile holds RT x (M + 1) values: exactly NV per thread for k < M (all
        // loads issued before any is used) plus the Nyquist column k = M
        {
            const int nt = blockDim.x;  // = RT * M / NV
            cpx<R> tv[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int o = tid + i * nt;
                const int r2 = o & (a.RT - 1);
                const int k = o >> a.log2RT;
                const int row = row0 + r2;
                tv[i] = (row < rows_out) ? at32(Y, (uint32_t)(k * a.ldY + row)) : cpx<R>{(R)0, (R)0};
            }
            // the Nyquist column, taken as the tile values are (a value
            // assigned under a branch was kept in scratch memory)
            const cpx<R> ny = (tid < a.RT && row0 + tid < rows_out)
                                  ? at32(Y, (uint32_t)(M * a.ldY + row0 + tid))
                                  : cpx<R>{(R)0, (R)0};
            if (tid < a.RT) lds[tid * PM + lpad<cpx<R>>(M)] = ny;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int o = tid + i * nt;
                lds[(o & (a.RT - 1)) * PM + lpad<cpx<R>>(o >> a.log2RT)] = tv[i];
            }
        }
        __syncthreads();
        // The first inverse pass reads its inputs merged from the split half
        // spectrum X of its row: Z[k] = (X[k] + X*[M-k]) + i W^{-k} (X[k] - X*[M-k])
        // (X[M] is the Nyquist column), so no separate merge pass is needed.
        cpx<R>* buf = lds + rr * PM;
        auto merged = [&](int k) {
            const cpx<R> xk = buf[lpad<cpx<R>>(k)];
            const cpx<R> xm = buf[lpad<cpx<R>>(M - k)];
            const cpx<R> s = cadd(xk, cconj(xm));
            const cpx<R> d = cmul(twiddle<R, true>(twb, k, LOG2M + 1), csub(xk, cconj(xm)));
            return cpx<R>{s.x - d.y, s.y + d.x};
        };
        {
            constexpr int R0 = 1 << S::lr(true, 0);
            constexpr int Q0 = M / R0;
#pragma unroll
            for (int u = 0; u < VT; ++u)
#pragma unroll
                for (int b = 0; b < 8 / R0; ++b) {
                    const int j = t + u * TR + b * T;
#pragma unroll
                    for (int r = 0; r < R0; ++r) v[u * 8 + b * R0 + r] = merged(j + r * Q0);
                }
        }
        if constexpr (S::npass == 1) {
#pragma unroll
            for (int u = 0; u < VT; ++u) pass_compute<R, LOG2M, true, 0>(v + u * 8, t + u * TR, twp);
        } else {
            lds_sync<WAVE>();  // every read of X before the pass overwrites it
#pragma unroll
            for (int u = 0; u < VT; ++u) {
                pass_compute<R, LOG2M, true, 0>(v + u * 8, t + u * TR, twp);
                pass_write<R, LOG2M, true, 0>(v + u * 8, buf, t + u * TR);
            }
            lds_sync<WAVE>();
            LdsPassesVT<R, LOG2M, true, 1, S::npass - 1, VT, WAVE>::run(v, buf, t, twp);
#pragma unroll
            for (int u = 0; u < VT; ++u) pass_read<R, LOG2M, true, S::npass - 1>(v + u * 8, buf, t + u * TR);
#pragma unroll
            for (int u = 0; u < VT; ++u) pass_compute<R, LOG2M, true, S::npass - 1>(v + u * 8, t + u * TR, twp);
        }
    }
    if (row >= rows_out) return;
    row_outputs<R, OUT, NV>(a, row, cols_out, vec, oci, obits, v,
                            [&](int k) { return edge_pos<LOG2M, LRL>(t + (k / 8) * TR, k % 8); });
}

// ---------------------------------------------------------------------------
// Mixed-radix stage kernels with compile-time plans (3 2^a, 5 2^a and 7 2^a
// lengths; fftm.hpp).  The data flow and layouts are those of the kernels
// above, with one value set per thread, complex exchanges, and every pass
// through LDS.  The last forward pass of a column leaves the spectrum in
// natural order in LDS, where the first inverse pass reads it multiplied by
// lam.
// ---------------------------------------------------------------------------
template <typename R, int M, int IN>
__global__ void __launch_bounds__(row_threads_mixed<R>()) k_row_fwd_c(StageAArgs a, const cpx<R>* __restrict__ twp) {
    using S = MSched<M>;
    constexpr int T = M / 8, PM = lpadded<cpx<R>>(M) + 1;
    constexpr bool LOW = (IN == IN_COMPACT);
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x;
    const int rr = tid / T, t = tid % T;
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int row0 = (lid % gridDim.x) * a.RT;
    const int row = row0 + rr;
    const int vec = lid / gridDim.x;
    if (a.active && !a.active[vec]) return;
    MaskView mask = a.mask;
    int rows_in = a.rows_in, row_len = a.row_len;
    if (a.tab) {
        const ProbDesc& d = a.tab[(a.vec0 + vec) / a.tab_vpp];
        mask = MaskView{d.bits, d.base, d.wpr};
        rows_in = d.n1;
        row_len = d.n2;
        if (row0 >= rows_in) return;
    }
    cpx<R>* buf = lds + rr * PM;
    cpx<R> v[MVMAX];
#pragma unroll
    for (int k = 0; k < MVMAX; ++k) v[k] = cpx<R>{(R)0, (R)0};
    row_inputs<R, IN, 1, LOW>(a, mask, vec, row, rows_in, row_len, t, T, T, v);
    mpass_compute_tw<R, M, false, 0, LOW>(v, MPassTw<R, M, false, 0>{});
    mpass_write<R, M, false, 0>(v, buf, t);
    __syncthreads();
    MLdsPasses<R, M, false, 1, S::npass>::run(v, buf, 0, t, twp);
    // split Z into the real transform X[k] = (s - i w d) / 2, k = 0..M, with
    // w = W_{2M}^k from the plan table
    cpx<R>* Y = reinterpret_cast<cpx<R>*>(a.Y) + vec * a.Y_vstride;
    const cpx<R>* ws = twp + S::split_off;
    auto split = [&](int r2, int k) {
        const cpx<R>* bp = lds + r2 * PM;
        const cpx<R> zk = bp[lpad<cpx<R>>(k == M ? 0 : k)];
        const cpx<R> zc = cconj(bp[lpad<cpx<R>>(k == 0 ? 0 : M - k)]);
        const cpx<R> s2 = cadd(zk, zc);
        const cpx<R> wd = cmul(ws[k], csub(zk, zc));
        at32(Y, (uint32_t)(k * a.ldY + row0 + r2)) = cpx<R>{(R)0.5 * (s2.x + wd.y), (R)0.5 * (s2.y - wd.x)};
    };
    const int nt = blockDim.x;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int o = tid + i * nt;
        split(o & (a.RT - 1), o >> a.log2RT);
    }
    if (tid < a.RT) split(tid, M);
}

template <typename R, int L, int MODE, int V>
__global__ void __launch_bounds__((L / 8 > 256 ? L / 8 : 256)) k_col_c(StageBArgs a, const cpx<R>* __restrict__ twp) {
    using S = MSched<L>;
    constexpr int T = L / 8, PL = lpadded<cpx<R>>(L);
    constexpr bool LOW = (MODE == B_LOW);
    constexpr int RI = S::radix(true, 0), BI = S::bpt(true, 0), QI = L / RI;
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x;
    const int cl = T >= 256 ? 0 : tid / T, t = T >= 256 ? tid : tid % T;
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int col = (lid / gridDim.y) * a.CB + cl;
    const bool valid = col < a.ncols;
    const int vbase = (lid % gridDim.y) * V;
    cpx<R>* buf = lds + cl * V * PL;
    if (a.active) {
        bool any = false;
#pragma unroll
        for (int u = 0; u < V; ++u) any = any || (vbase + u < a.nvec && a.active[vbase + u]);
        if (!any) return;
    }
    int rows_in[V], rows_out[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
        rows_in[u] = a.rows_in;
        rows_out[u] = a.rows_out;
        if (a.tab) {
            const ProbDesc& d = a.tab[(a.vec0 + min(vbase + u, a.nvec - 1)) / a.tab_vpp];
            rows_in[u] = d.n1;
            rows_out[u] = d.n1;
        }
    }
    // spectrum values at the first inverse pass's input positions, fetched
    // up front (unused slots read position 0 of the last vector's spectrum)
    R lamv[MODE == B_SPEC ? 1 : V * BI * RI];
    if constexpr (MODE != B_SPEC) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int vl = min(vbase + u, a.nvec - 1);
            const R* lam;
            if (a.tab) {
                const ProbDesc& d = a.tab[(a.vec0 + vl) / a.tab_vpp];
                lam = reinterpret_cast<const R*>(sizeof(R) == 8 ? (const void*)d.lam64 : (const void*)d.lam32);
            } else {
                lam = reinterpret_cast<const R*>(a.lam) + (int64_t)((a.vec0 + vl) / a.vecs_per_theta) * a.lam_tstride;
            }
            lam += (int64_t)(valid ? col : 0) * L;
#pragma unroll
            for (int b = 0; b < BI; ++b) {
                const int j = t + b * T;
#pragma unroll
                for (int r = 0; r < RI; ++r) lamv[(u * BI + b) * RI + r] = lam[j < QI ? j + r * QI : 0];
            }
        }
    }
    cpx<R>* Ycol = reinterpret_cast<cpx<R>*>(a.Y) + (int64_t)(valid ? col : 0) * a.ldY;
    cpx<R> v[V * MVMAX];
#pragma unroll
    for (int u = 0; u < V; ++u) {
        const bool vu = valid && (vbase + u < a.nvec);
        const cpx<R>* Yv = Ycol + (vbase + u) * a.Y_vstride;
#pragma unroll
        for (int r = 0; r < MVMAX; ++r) {
            const int idx = t + r * T;
            v[u * MVMAX + r] = cpx<R>{(R)0, (R)0};
            if (r >= 8 || (LOW && r >= 4)) continue;
            if (vu && idx < rows_in[u]) v[u * MVMAX + r] = Yv[idx];
        }
    }
#pragma unroll
    for (int u = 0; u < V; ++u) {
        mpass_compute_tw<R, L, false, 0, LOW>(v + u * MVMAX, MPassTw<R, L, false, 0>{});
        mpass_write<R, L, false, 0>(v + u * MVMAX, buf + u * PL, t);
    }
    __syncthreads();
    MLdsPasses<R, L, false, 1, S::npass, V>::run(v, buf, PL, t, twp);
    if constexpr (MODE == B_SPEC) {
        if (valid) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int pos = t + k * T;
                a.spec_out[(int64_t)col * L + pos] = (double)buf[lpad<cpx<R>>(pos)].x;
            }
        }
        return;
    } else {
        // first inverse pass: its inputs times lam
#pragma unroll
        for (int u = 0; u < V; ++u)
#pragma unroll
            for (int b = 0; b < BI; ++b) {
                const int j = t + b * T;
                if (j < QI) {
#pragma unroll
                    for (int r = 0; r < RI; ++r)
                        v[u * MVMAX + b * RI + r] =
                            cscale(buf[u * PL + lpad<cpx<R>>(j + r * QI)], lamv[(u * BI + b) * RI + r]);
                }
            }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < V; ++u) {
            mpass_compute_tw<R, L, true, 0>(v + u * MVMAX, MPassTw<R, L, true, 0>{});
            mpass_write<R, L, true, 0>(v + u * MVMAX, buf + u * PL, t);
        }
        __syncthreads();
        MLdsPasses<R, L, true, 1, S::npass - 1, V>::run(v, buf, PL, t, twp);
        {
            constexpr int PLAST = S::npass - 1;  // radix 8: outputs at t + k T
            const auto w = mpass_twiddles<R, L, true, PLAST>(t, twp);
#pragma unroll
            for (int u = 0; u < V; ++u) {
                mpass_read<R, L, true, PLAST>(v + u * MVMAX, buf + u * PL, t);
                mpass_compute_tw<R, L, true, PLAST>(v + u * MVMAX, w);
            }
        }
#pragma unroll
        for (int u = 0; u < V; ++u) {
            if (!(valid && vbase + u < a.nvec)) continue;
            cpx<R>* Yv = Ycol + (vbase + u) * a.Y_vstride;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int idx = t + k * T;
                if (idx < rows_out[u]) Yv[idx] = v[u * MVMAX + k];
            }
        }
    }
}

template <typename R, int M, int OUT>
__global__ void __launch_bounds__(row_threads_mixed<R>()) k_row_inv_c(StageCArgs a, const cpx<R>* __restrict__ twp) {
    using S = MSched<M>;
    constexpr int T = M / 8, PM = lpadded<cpx<R>>(M) + 1;
    constexpr int NV = 8;
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x;
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int tile = lid % gridDim.x;
    const int row0 = tile * a.RT;
    const int vec = lid / gridDim.x;
    const cpx<R>* Y = reinterpret_cast<const cpx<R>*>(a.Y) + vec * a.Y_vstride;
    const int rr = tid / T, t = tid % T;
    const int row = row0 + rr;
    if (a.active && !a.active[vec]) return;
    MaskView mask = a.mask;
    int rows_out = a.rows_out, cols_out = a.cols_out;
    if (a.tab) {
        const ProbDesc& d = a.tab[(a.vec0 + vec) / a.tab_vpp];
        mask = MaskView{d.bits, d.base, d.wpr};
        rows_out = d.n1;
        cols_out = d.n2;
        if constexpr (OUT == OUT_COMPACT) {
            const int64_t len = a.out_vstride - d.p;
            const int64_t per = (len + gridDim.x - 1) / gridDim.x;
            const int64_t b = d.p + tile * per, e = min(b + per, a.out_vstride);
            R* o = reinterpret_cast<R*>(a.out) + vec * a.out_vstride;
            for (int64_t i = b + tid; i < e; i += blockDim.x) o[i] = (R)0;
        }
        if (row0 >= rows_out) return;
    }
    auto pos = [&](int k) { return t + k * T; };  // the last inverse pass is radix 8
    int32_t oci[NV];
    uint64_t obits = 0u;
    row_output_cells<OUT, NV>(mask, row, rows_out, cols_out, oci, obits, pos);
    {
        const int nt = blockDim.x;  // = RT * T
        cpx<R> tv[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int o = tid + i * nt;
            const int r2 = o & (a.RT - 1);
            const int k = o >> a.log2RT;
            tv[i] = (row0 + r2 < rows_out) ? at32(Y, (uint32_t)(k * a.ldY + row0 + r2)) : cpx<R>{(R)0, (R)0};
        }
        // (the Nyquist value taken by a select, not assigned under a branch,
        // which kept it in scratch memory)
        const cpx<R> ny = (tid < a.RT && row0 + tid < rows_out) ? at32(Y, (uint32_t)(M * a.ldY + row0 + tid))
                                                                 : cpx<R>{(R)0, (R)0};
        if (tid < a.RT) lds[tid * PM + lpad<cpx<R>>(M)] = ny;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int o = tid + i * nt;
            lds[(o & (a.RT - 1)) * PM + lpad<cpx<R>>(o >> a.log2RT)] = tv[i];
        }
    }
    __syncthreads();
    // first inverse pass: inputs merged from the split half spectrum,
    // Z[k] = (X[k] + X*[M-k]) + i conj(W_{2M}^k) (X[k] - X*[M-k])
    cpx<R>* buf = lds + rr * PM;
    const cpx<R>* ws = twp + S::split_off;
    auto merged = [&](int k) {
        const cpx<R> xk = buf[lpad<cpx<R>>(k)];
        const cpx<R> xm = buf[lpad<cpx<R>>(M - k)];
        const cpx<R> s2 = cadd(xk, cconj(xm));
        const cpx<R> d = cmul(cconj(ws[k]), csub(xk, cconj(xm)));
        return cpx<R>{s2.x - d.y, s2.y + d.x};
    };
    constexpr int R0 = S::radix(true, 0), B0 = S::bpt(true, 0), Q0 = M / R0;
    cpx<R> v[MVMAX];
#pragma unroll
    for (int k = 0; k < MVMAX; ++k) v[k] = cpx<R>{(R)0, (R)0};
#pragma unroll
    for (int b = 0; b < B0; ++b) {
        const int j = t + b * T;
        if (j < Q0) {
#pragma unroll
            for (int r = 0; r < R0; ++r) v[b * R0 + r] = merged(j + r * Q0);
        }
    }
    __syncthreads();  // every read of X before the pass overwrites it
    mpass_compute_tw<R, M, true, 0>(v, MPassTw<R, M, true, 0>{});
    mpass_write<R, M, true, 0>(v, buf, t);
    __syncthreads();
    MLdsPasses<R, M, true, 1, S::npass - 1>::run(v, buf, 0, t, twp);
    {
        constexpr int PLAST = S::npass - 1;
        const auto w = mpass_twiddles<R, M, true, PLAST>(t, twp);
        mpass_read<R, M, true, PLAST>(v, buf, t);
        mpass_compute_tw<R, M, true, PLAST>(v, w);
    }
    if (row >= rows_out) return;
    row_outputs<R, OUT, NV>(a, row, cols_out, vec, oci, obits, v, pos);
}

// ---------------------------------------------------------------------------
// Mixed-radix stage kernels with run-time plans (the other embeddings
// 2^a 3^b 5^c 7^d that are not powers of two; fftm.hpp).  The data
// flow and layouts are those of the kernels above, with one value set per
// thread, complex exchanges, and every pass through LDS.  The last forward
// pass of a column leaves the spectrum in natural order in LDS, where the
// first inverse pass (radix RI, the plan's last forward radix, a template
// argument so that its per-thread layout is fixed) reads it multiplied by
// lam.
// ---------------------------------------------------------------------------
template <typename R, int IN>
__global__ void __launch_bounds__(row_threads_mixed<R>()) k_row_fwd_m(StageAArgs a, const cpx<R>* __restrict__ twp,
                                                    const MPlan* __restrict__ pl) {
    const int M = pl->L, T = pl->T, PM = lpadded<cpx<R>>(M) + 1;
    constexpr bool LOW = (IN == IN_COMPACT);
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x;
    const int rr = tid / T, t = tid % T;
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int row0 = (lid % gridDim.x) * a.RT;
    const int row = row0 + rr;
    const int vec = lid / gridDim.x;
    if (a.active && !a.active[vec]) return;
    MaskView mask = a.mask;
    int rows_in = a.rows_in, row_len = a.row_len;
    if (a.tab) {
        const ProbDesc& d = a.tab[(a.vec0 + vec) / a.tab_vpp];
        mask = MaskView{d.bits, d.base, d.wpr};
        rows_in = d.n1;
        row_len = d.n2;
        if (row0 >= rows_in) return;
    }
    cpx<R>* buf = lds + rr * PM;
    cpx<R> v[MVMAX];
#pragma unroll
    for (int k = 0; k < MVMAX; ++k) v[k] = cpx<R>{(R)0, (R)0};
    row_inputs<R, IN, 1, LOW>(a, mask, vec, row, rows_in, row_len, t, T, T, v);
    mr_butterflies<R, 8, false, LOW>(v);
    mr_write<R, 8>(v, buf, t, T, M, 1);
    __syncthreads();
    mr_lds_passes<R, false>(pl, 1, pl->npass, v, buf, 0, t, twp);
    // split Z into the real transform X[k] = (s - i w d) / 2, k = 0..M, with
    // w = W_{2M}^k from the plan table
    cpx<R>* Y = reinterpret_cast<cpx<R>*>(a.Y) + vec * a.Y_vstride;
    const cpx<R>* ws = twp + pl->split_off;
    auto split = [&](int r2, int k) {
        const cpx<R>* bp = lds + r2 * PM;
        const cpx<R> zk = bp[lpad<cpx<R>>(k == M ? 0 : k)];
        const cpx<R> zc = cconj(bp[lpad<cpx<R>>(k == 0 ? 0 : M - k)]);
        const cpx<R> s2 = cadd(zk, zc);
        const cpx<R> wd = cmul(ws[k], csub(zk, zc));
        at32(Y, (uint32_t)(k * a.ldY + row0 + r2)) = cpx<R>{(R)0.5 * (s2.x + wd.y), (R)0.5 * (s2.y - wd.x)};
    };
    const int nt = blockDim.x;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int o = tid + i * nt;
        split(o & (a.RT - 1), o >> a.log2RT);
    }
    if (tid < a.RT) split(tid, M);
}

// TMAX: the largest workgroup the launch may use (256, 512, 768 or 1024
// threads: one column of up to 2048, 4096, 6144 or 8192 points, or several
// shorter ones).
template <typename R, int MODE, int V, int RI, int TMAX>
__global__ void __launch_bounds__(TMAX) k_col_m(StageBArgs a, const cpx<R>* __restrict__ twp,
                                                const MPlan* __restrict__ pl) {
    const int L = pl->L, T = pl->T, PL = lpadded<cpx<R>>(L), npass = pl->npass;
    constexpr bool LOW = (MODE == B_LOW);
    constexpr int BI = mbpt<RI>();
    const int QI = L / RI;
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x;
    const int cl = T >= 256 ? 0 : tid / T, t = T >= 256 ? tid : tid % T;
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int col = (lid / gridDim.y) * a.CB + cl;
    const bool valid = col < a.ncols;
    const int vbase = (lid % gridDim.y) * V;
    cpx<R>* buf = lds + cl * V * PL;
    if (a.active) {
        bool any = false;
#pragma unroll
        for (int u = 0; u < V; ++u) any = any || (vbase + u < a.nvec && a.active[vbase + u]);
        if (!any) return;
    }
    int rows_in[V], rows_out[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
        rows_in[u] = a.rows_in;
        rows_out[u] = a.rows_out;
        if (a.tab) {
            const ProbDesc& d = a.tab[(a.vec0 + min(vbase + u, a.nvec - 1)) / a.tab_vpp];
            rows_in[u] = d.n1;
            rows_out[u] = d.n1;
        }
    }
    // spectrum values at the first inverse pass's input positions, fetched
    // up front (unused slots read position 0 of the last vector's spectrum)
    R lamv[MODE == B_SPEC ? 1 : V * BI * RI];
    if constexpr (MODE != B_SPEC) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int vl = min(vbase + u, a.nvec - 1);
            const R* lam;
            if (a.tab) {
                const ProbDesc& d = a.tab[(a.vec0 + vl) / a.tab_vpp];
                lam = reinterpret_cast<const R*>(sizeof(R) == 8 ? (const void*)d.lam64 : (const void*)d.lam32);
            } else {
                lam = reinterpret_cast<const R*>(a.lam) + (int64_t)((a.vec0 + vl) / a.vecs_per_theta) * a.lam_tstride;
            }
            lam += (int64_t)(valid ? col : 0) * L;
#pragma unroll
            for (int b = 0; b < BI; ++b) {
                const int j = t + b * T;
#pragma unroll
                for (int r = 0; r < RI; ++r) lamv[(u * BI + b) * RI + r] = lam[j < QI ? j + r * QI : 0];
            }
        }
    }
    cpx<R>* Ycol = reinterpret_cast<cpx<R>*>(a.Y) + (int64_t)(valid ? col : 0) * a.ldY;
    cpx<R> v[V * MVMAX];
#pragma unroll
    for (int u = 0; u < V; ++u) {
        const bool vu = valid && (vbase + u < a.nvec);
        const cpx<R>* Yv = Ycol + (vbase + u) * a.Y_vstride;
#pragma unroll
        for (int r = 0; r < MVMAX; ++r) {
            const int idx = t + r * T;
            v[u * MVMAX + r] = cpx<R>{(R)0, (R)0};
            if (r >= 8 || (LOW && r >= 4)) continue;
            if (vu && idx < rows_in[u]) v[u * MVMAX + r] = Yv[idx];
        }
    }
#pragma unroll
    for (int u = 0; u < V; ++u) {
        mr_butterflies<R, 8, false, LOW>(v + u * MVMAX);
        mr_write<R, 8>(v + u * MVMAX, buf + u * PL, t, T, L, 1);
    }
    __syncthreads();
    mr_lds_passes<R, false, V>(pl, 1, npass, v, buf, PL, t, twp);
    if constexpr (MODE == B_SPEC) {
        if (valid) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int pos = t + k * T;
                a.spec_out[(int64_t)col * L + pos] = (double)buf[lpad<cpx<R>>(pos)].x;
            }
        }
        return;
    } else {
        // first inverse pass: its inputs times lam
#pragma unroll
        for (int u = 0; u < V; ++u)
#pragma unroll
            for (int b = 0; b < BI; ++b) {
                const int j = t + b * T;
                if (j < QI) {
#pragma unroll
                    for (int r = 0; r < RI; ++r)
                        v[u * MVMAX + b * RI + r] =
                            cscale(buf[u * PL + lpad<cpx<R>>(j + r * QI)], lamv[(u * BI + b) * RI + r]);
                }
            }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < V; ++u) {
            mr_butterflies<R, RI, true>(v + u * MVMAX);
            mr_write<R, RI>(v + u * MVMAX, buf + u * PL, t, T, L, 1);
        }
        __syncthreads();
        mr_lds_passes<R, true, V>(pl, 1, npass - 1, v, buf, PL, t, twp);
        {
            // the last inverse pass is radix 8: outputs at t + k T
            const int PLAST = npass - 1;
            const auto w = mr_twiddles<R, 8>(t, T, L, pl->ns_i[PLAST], pl->magic_i[PLAST], twp + pl->tw_i[PLAST]);
#pragma unroll
            for (int u = 0; u < V; ++u) {
                mr_read<R, 8>(v + u * MVMAX, buf + u * PL, t, T, L);
                mr_compute<R, 8, true>(v + u * MVMAX, w);
            }
        }
#pragma unroll
        for (int u = 0; u < V; ++u) {
            if (!(valid && vbase + u < a.nvec)) continue;
            cpx<R>* Yv = Ycol + (vbase + u) * a.Y_vstride;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int idx = t + k * T;
                if (idx < rows_out[u]) Yv[idx] = v[u * MVMAX + k];
            }
        }
    }
}

// R0: radix of the first inverse pass (the plan's last forward radix).
template <typename R, int OUT, int R0>
__global__ void __launch_bounds__(row_threads_mixed<R>()) k_row_inv_m(StageCArgs a, const cpx<R>* __restrict__ twp,
                                                    const MPlan* __restrict__ pl) {
    const int M = pl->L, T = pl->T, PM = lpadded<cpx<R>>(M) + 1, npass = pl->npass;
    constexpr int NV = 8;
    extern __shared__ unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x;
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int tile = lid % gridDim.x;
    const int row0 = tile * a.RT;
    const int vec = lid / gridDim.x;
    const cpx<R>* Y = reinterpret_cast<const cpx<R>*>(a.Y) + vec * a.Y_vstride;
    const int rr = tid / T, t = tid % T;
    const int row = row0 + rr;
    if (a.active && !a.active[vec]) return;
    MaskView mask = a.mask;
    int rows_out = a.rows_out, cols_out = a.cols_out;
    if (a.tab) {
        const ProbDesc& d = a.tab[(a.vec0 + vec) / a.tab_vpp];
        mask = MaskView{d.bits, d.base, d.wpr};
        rows_out = d.n1;
        cols_out = d.n2;
        if constexpr (OUT == OUT_COMPACT) {
            const int64_t len = a.out_vstride - d.p;
            const int64_t per = (len + gridDim.x - 1) / gridDim.x;
            const int64_t b = d.p + tile * per, e = min(b + per, a.out_vstride);
            R* o = reinterpret_cast<R*>(a.out) + vec * a.out_vstride;
            for (int64_t i = b + tid; i < e; i += blockDim.x) o[i] = (R)0;
        }
        if (row0 >= rows_out) return;
    }
    auto pos = [&](int k) { return t + k * T; };  // the last inverse pass is radix 8
    int32_t oci[NV];
    uint64_t obits = 0u;
    row_output_cells<OUT, NV>(mask, row, rows_out, cols_out, oci, obits, pos);
    {
        const int nt = blockDim.x;  // = RT * T
        cpx<R> tv[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int o = tid + i * nt;
            const int r2 = o & (a.RT - 1);
            const int k = o >> a.log2RT;
            tv[i] = (row0 + r2 < rows_out) ? at32(Y, (uint32_t)(k * a.ldY + row0 + r2)) : cpx<R>{(R)0, (R)0};
        }
        // (the Nyquist value taken by a select, not assigned under a branch,
        // which kept it in scratch memory)
        const cpx<R> ny = (tid < a.RT && row0 + tid < rows_out) ? at32(Y, (uint32_t)(M * a.ldY + row0 + tid))
                                                                 : cpx<R>{(R)0, (R)0};
        if (tid < a.RT) lds[tid * PM + lpad<cpx<R>>(M)] = ny;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int o = tid + i * nt;
            lds[(o & (a.RT - 1)) * PM + lpad<cpx<R>>(o >> a.log2RT)] = tv[i];
        }
    }
    __syncthreads();
    // first inverse pass: inputs merged from the split half spectrum,
    // Z[k] = (X[k] + X*[M-k]) + i conj(W_{2M}^k) (X[k] - X*[M-k])
    cpx<R>* buf = lds + rr * PM;
    const cpx<R>* ws = twp + pl->split_off;
    auto merged = [&](int k) {
        const cpx<R> xk = buf[lpad<cpx<R>>(k)];
        const cpx<R> xm = buf[lpad<cpx<R>>(M - k)];
        const cpx<R> s2 = cadd(xk, cconj(xm));
        const cpx<R> d = cmul(cconj(ws[k]), csub(xk, cconj(xm)));
        return cpx<R>{s2.x - d.y, s2.y + d.x};
    };
    constexpr int B0 = mbpt<R0>();
    const int Q0 = M / R0;
    cpx<R> v[MVMAX];
#pragma unroll
    for (int k = 0; k < MVMAX; ++k) v[k] = cpx<R>{(R)0, (R)0};
#pragma unroll
    for (int b = 0; b < B0; ++b) {
        const int j = t + b * T;
        if (j < Q0) {
#pragma unroll
            for (int r = 0; r < R0; ++r) v[b * R0 + r] = merged(j + r * Q0);
        }
    }
    __syncthreads();  // every read of X before the pass overwrites it
    mr_butterflies<R, R0, true>(v);
    mr_write<R, R0>(v, buf, t, T, M, 1);
    __syncthreads();
    mr_lds_passes<R, true>(pl, 1, npass - 1, v, buf, 0, t, twp);
    {
        const int PLAST = npass - 1;
        const auto w = mr_twiddles<R, 8>(t, T, M, pl->ns_i[PLAST], pl->magic_i[PLAST], twp + pl->tw_i[PLAST]);
        mr_read<R, 8>(v, buf, t, T, M);
        mr_compute<R, 8, true>(v, w);
    }
    if (row >= rows_out) return;
    row_outputs<R, OUT, NV>(a, row, cols_out, vec, oci, obits, v, pos);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
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

// Per-length pass twiddle tables (fftk.hpp layout), built on first use.
template <typename Real, int LOG2L>
static void fill_plan(std::vector<std::array<long double, 2>>& out) {
    using S = Sched<LOG2L>;
    out.assign(S::tw_total > 0 ? S::tw_total : 1, {1.0L, 0.0L});
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int inv = 0; inv < 2; ++inv)
        for (int p = 1; p < S::npass; ++p) {
            const int R = 1 << S::lr(inv, p), NS = 1 << S::lns(inv, p);
            const int off = S::tw_off(inv, p);
            for (int jn = 0; jn < NS; ++jn)
                for (int r = 0; r < R; ++r) {
                    const long double ang = (inv ? 2.0L : -2.0L) * pi * (long double)(r * jn) / (long double)(NS * R);
                    out[off + tw_index<Real>(r, jn, NS)] = {cosl(ang), sinl(ang)};
                }
        }
}

template <typename R>
static const cpx<R>* plan_table(Ctx& c, int log2L) {
    static std::mutex mu;
    std::lock_guard<std::mutex> g(mu);
    void*& slot = (sizeof(R) == 8 ? c.plan64 : c.plan32)[log2L];
    if (slot) return static_cast<const cpx<R>*>(slot);
    std::vector<std::array<long double, 2>> tab;
    switch (log2L) {
        case 3: fill_plan<R, 3>(tab); break;
        case 4: fill_plan<R, 4>(tab); break;
        case 5: fill_plan<R, 5>(tab); break;
        case 6: fill_plan<R, 6>(tab); break;
        case 7: fill_plan<R, 7>(tab); break;
        case 8: fill_plan<R, 8>(tab); break;
        case 9: fill_plan<R, 9>(tab); break;
        case 10: fill_plan<R, 10>(tab); break;
        case 11: fill_plan<R, 11>(tab); break;
        case 12: fill_plan<R, 12>(tab); break;
        case 13: fill_plan<R, 13>(tab); break;
        default: throw Error(KRY_EINVAL, "transform length out of range");
    }
    std::vector<cpx<R>> h(tab.size());
    for (size_t i = 0; i < tab.size(); ++i) h[i] = cpx<R>{(R)tab[i][0], (R)tab[i][1]};
    slot = dev_alloc(c, h.size() * sizeof(cpx<R>));
    KRY_HIP(hipMemcpy(slot, h.data(), h.size() * sizeof(cpx<R>), hipMemcpyHostToDevice));
    return static_cast<const cpx<R>*>(slot);
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Lengths with compile-time mixed-radix kernels (3 2^a, 5 2^a, 7 2^a):
// row lengths M (half a torus side) and column lengths (torus sides).
#define KRY_CROWS(X) X(24) X(40) X(48) X(56) X(80) X(96) X(112) X(160) X(192) X(224) X(320) X(384) X(448) \
    X(640) X(768) X(896) X(1280) X(1536) X(1792) X(2560) X(3072) X(3584)
#define KRY_CCOLS(X) X(48) X(80) X(96) X(112) X(160) X(192) X(224) X(320) X(384) X(448) X(640) X(768) X(896) \
    X(1280) X(1536) X(1792) X(2560) X(3072) X(3584) X(5120) X(6144) X(7168)

static bool is_ct_row(int M) {
#define KRY_T(X) if (M == X) return true;
    KRY_CROWS(KRY_T)
#undef KRY_T
    return false;
}
static bool is_ct_col(int L) {
#define KRY_T(X) if (L == X) return true;
    KRY_CCOLS(KRY_T)
#undef KRY_T
    return false;
}

// Mixed-radix lengths (fftm.hpp): 2^a 3^b 5^c 7^d, a >= 3, not powers of two.
static bool mixed_len_ok(int L) {
    MPlan p;
    return !is_pow2(L) && mplan_make(L, &p);
}

static MPlan mixed_plan(int L) {
    MPlan p;
    if (!mplan_make(L, &p)) throw Error(KRY_EINVAL, "mixed-radix transform length not supported");
    return p;
}

bool torus_side_ok(int N) {
    if (N < 16 || N > 8192) return false;
    return is_pow2(N) || (N % 16 == 0 && mixed_len_ok(N) && mixed_len_ok(N / 2));
}

int spectral_qf_count(int N1, int N2) {
    return is_pow2(N1) ? (N2 / 2 + 1) * col_qf_waves(ilog2(N1)) : 0;
}

// Relative cost per point of a torus side: 1 for a power of two, 1.2 for a
// side with compile-time kernels (one factor 3, 5 or 7; measured 1.2-1.5
// times the power-of-two cost per point over both axes of a product), 1.75
// for the other sides (run-time plans: 2.2-3.5 times).
static double side_weight(int N) {
    if (is_pow2(N)) return 1.0;
    return is_ct_col(N) && is_ct_row(N / 2) ? 1.2 : 1.75;
}

int embedding_side(int m, int rule) {
    int best = 0;
    double best_cost = 0.0;
    for (int N = std::max(16, m); N <= 8192; ++N) {
        if (!torus_side_ok(N)) continue;
        if (rule == KRY_EMBED_SMALLEST) return N;
        const double cost = N * side_weight(N);
        if (!best || cost < best_cost) {
            best = N;
            best_cost = cost;
        }
        if (is_pow2(N)) break;  // every larger side costs more
    }
    return best;
}

// Pass twiddles of a mixed-radix length, [r][j mod Ns] per pass and
// direction, then W_{2L}^k for k = 0..L (the real-to-complex split).
static void fill_mplan(const MPlan& pl, std::vector<std::array<long double, 2>>& out) {
    out.assign(pl.tw_total, {1.0L, 0.0L});
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int inv = 0; inv < 2; ++inv)
        for (int p = 1; p < pl.npass; ++p) {
            const int R = pl.radix_at(inv, p), NS = inv ? pl.ns_i[p] : pl.ns_f[p];
            const int off = inv ? pl.tw_i[p] : pl.tw_f[p];
            for (int jn = 0; jn < NS; ++jn)
                for (int r = 0; r < R; ++r) {
                    const long double ang = (inv ? 2.0L : -2.0L) * pi * (long double)(r * jn) / (long double)(NS * R);
                    out[off + r * NS + jn] = {cosl(ang), sinl(ang)};
                }
        }
    for (int k = 0; k <= pl.L; ++k) {
        const long double ang = -2.0L * pi * (long double)k / (long double)(2 * pl.L);
        out[pl.split_off + k] = {cosl(ang), sinl(ang)};
    }
}

// A mixed-radix length's plan and twiddle table in one device allocation:
// the plan (read by the kernels pass by pass), then the twiddles.
template <typename R>
struct MTable {
    const MPlan* plan;
    const cpx<R>* tw;
};
constexpr size_t kPlanBytes = (sizeof(MPlan) + 255) & ~size_t(255);

// Built on first use (problems build theirs when they are created, so
// products allocate nothing).
template <typename R>
static MTable<R> mplan_table(Ctx& c, int L) {
    static std::mutex mu;
    std::lock_guard<std::mutex> g(mu);
    auto& m = sizeof(R) == 8 ? c.mplan64 : c.mplan32;
    auto it = m.find(L);
    if (it == m.end()) {
        const MPlan pl = mixed_plan(L);
        std::vector<std::array<long double, 2>> tab;
        fill_mplan(pl, tab);
        std::vector<unsigned char> h(kPlanBytes + tab.size() * sizeof(cpx<R>), 0);
        std::memcpy(h.data(), &pl, sizeof(MPlan));
        cpx<R>* hw = reinterpret_cast<cpx<R>*>(h.data() + kPlanBytes);
        for (size_t i = 0; i < tab.size(); ++i) hw[i] = cpx<R>{(R)tab[i][0], (R)tab[i][1]};
        void* slot = dev_alloc(c, h.size());
        KRY_HIP(hipMemcpy(slot, h.data(), h.size(), hipMemcpyHostToDevice));
        it = m.emplace(L, slot).first;
    }
    const unsigned char* base = static_cast<const unsigned char*>(it->second);
    return MTable<R>{reinterpret_cast<const MPlan*>(base), reinterpret_cast<const cpx<R>*>(base + kPlanBytes)};
}

void build_plan_tables(Ctx& c) {
    for (int lg = 3; lg <= 13; ++lg) {
        plan_table<double>(c, lg);
        plan_table<float>(c, lg);
    }
}

void build_embedding_tables(Ctx& c, int N1, int N2) {
    for (int L : {N1, N2 / 2})
        if (!is_pow2(L)) {
            mplan_table<double>(c, L);
            mplan_table<float>(c, L);
        }
}

struct RowTiling {
    int RT, T, threads;
    size_t lds;
};

// Rows per tile: transposed runs of RT * sizeof(cpx) = 64 * rt_scale bytes
// where the workgroup and LDS allow; more rows for short rows.  Each thread
// holds 8 vt values of its row.
template <typename R>
static RowTiling row_tiling(int M, int rt_scale = 1, int vt = 1, bool split = false) {
    const size_t cs = sizeof(cpx<R>);
    const int T = M / 8 / vt;  // threads per row
    const int tmax = is_pow2(M) ? row_threads_max<R>(vt) : row_threads_mixed<R>();
    const size_t PM = (size_t)M + M / 16 + 1;  // lpadded<cpx<R>>(M) + 1, as the kernels
    int RT = (int)(64 * rt_scale / cs);
    while (RT > 1 && RT * T > tmax) RT /= 2;
    while (RT > 1 && RT * PM * cs > 150 * 1024) RT /= 2;
    while (RT * T < 256 && RT < 64 && (size_t)(2 * RT) * PM * cs <= 64 * 1024) RT *= 2;
    RowTiling t;
    t.RT = RT;
    t.T = T;
    t.threads = RT * T;
    t.lds = RT * PM * (split ? sizeof(R) : cs);  // split exchanges: a buffer of reals
    return t;
}

// Row kernels with two virtual threads exist for rows of >= 1024 points.
template <int LG>
constexpr bool has_vt2() { return LG >= 10; }

template <typename R, int LG, int IN>
static void launch_row_fwd(const StageAArgs& a, dim3 grid, const RowTiling& t, int vt, bool split, Ctx& c,
                           hipStream_t st) {
    auto k = k_row_fwd<R, LG, IN, 1, false>;
    if constexpr (has_vt2<LG>()) {
        if (vt == 2) k = k_row_fwd<R, LG, IN, 2, false>;
        if (split) k = vt == 2 ? k_row_fwd<R, LG, IN, 2, true> : k_row_fwd<R, LG, IN, 1, true>;
    }
    set_lds(k, t.lds);
    hipLaunchKernelGGL(k, grid, dim3(t.threads), t.lds, st, a, plan_table<R>(c, LG), twiddles<R>(c));
    KRY_HIP(hipGetLastError());
}

template <typename R, int LG, int OUT>
static void launch_row_inv(const StageCArgs& a, dim3 grid, const RowTiling& t, int vt, bool split, Ctx& c,
                           hipStream_t st) {
    auto k = k_row_inv<R, LG, OUT, 1, false>;
    if constexpr (has_vt2<LG>()) {
        if (vt == 2) k = k_row_inv<R, LG, OUT, 2, false>;
        if (split) k = vt == 2 ? k_row_inv<R, LG, OUT, 2, true> : k_row_inv<R, LG, OUT, 1, true>;
    }
    set_lds(k, t.lds);
    hipLaunchKernelGGL(k, grid, dim3(t.threads), t.lds, st, a, plan_table<R>(c, LG), twiddles<R>(c));
    KRY_HIP(hipGetLastError());
}

template <typename R, int LG, int MODE, int V, bool SPLIT>
static void launch_col_v(const StageBArgs& b, int nvec, Ctx& c, hipStream_t st) {
    constexpr int L = 1 << LG, T = L / 8;
    const size_t lds = (size_t)b.CB * V * lpadded<cpx<R>>(L) * (SPLIT ? sizeof(R) : sizeof(cpx<R>));
    dim3 grid((b.ncols + b.CB - 1) / b.CB, (nvec + V - 1) / V);
    auto k = k_col<R, LG, MODE, V, SPLIT>;
    set_lds(k, lds);
    StageBArgs bb = b;
    bb.nvec = nvec;
    hipLaunchKernelGGL(k, grid, dim3(b.CB * T), lds, st, bb, plan_table<R>(c, LG));
    KRY_HIP(hipGetLastError());
}

// V vectors per workgroup share twiddle and spectrum loads; the spectrum
// transform takes one.  split: exchanges through a buffer of reals
// (transforms of 256 points or more, where LDS bounds the occupancy).
template <typename R, int LG, int MODE>
static void launch_col(const StageBArgs& b, int nvec, int V, bool split, Ctx& c, hipStream_t st) {
    if constexpr (MODE != B_SPEC && LG >= 8) {
        if (split) {
            if (V == 2) launch_col_v<R, LG, MODE, 2, true>(b, nvec, c, st);
            else launch_col_v<R, LG, MODE, 1, true>(b, nvec, c, st);
            return;
        }
    }
    if constexpr (MODE != B_SPEC) {
        if (V == 2) {
            launch_col_v<R, LG, MODE, 2, false>(b, nvec, c, st);
            return;
        }
    }
    launch_col_v<R, LG, MODE, 1, false>(b, nvec, c, st);
}

template <typename R, int M, int IN>
static void launch_row_fwd_c(const StageAArgs& a, dim3 grid, const RowTiling& t, Ctx& c, hipStream_t st) {
    auto k = k_row_fwd_c<R, M, IN>;
    set_lds(k, t.lds);
    hipLaunchKernelGGL(k, grid, dim3(t.threads), t.lds, st, a, mplan_table<R>(c, M).tw);
    KRY_HIP(hipGetLastError());
}

template <typename R, int M, int OUT>
static void launch_row_inv_c(const StageCArgs& a, dim3 grid, const RowTiling& t, Ctx& c, hipStream_t st) {
    auto k = k_row_inv_c<R, M, OUT>;
    set_lds(k, t.lds);
    hipLaunchKernelGGL(k, grid, dim3(t.threads), t.lds, st, a, mplan_table<R>(c, M).tw);
    KRY_HIP(hipGetLastError());
}

// Columns of a compile-time mixed-radix length: V = 2 vectors per workgroup
// where their LDS fits, else one.
template <typename R, int L, int MODE>
static void launch_col_c(const StageBArgs& b, int nvec, int V, Ctx& c, hipStream_t st) {
    constexpr int T = L / 8;
    const size_t per = (size_t)b.CB * lpadded<cpx<R>>(L) * sizeof(cpx<R>);
    if (MODE == B_SPEC || 2 * per > 160 * 1024) V = 1;
    const size_t lds = per * V;
    dim3 grid((b.ncols + b.CB - 1) / b.CB, (nvec + V - 1) / V);
    StageBArgs bb = b;
    bb.nvec = nvec;
    if (V == 2) {
        auto k = k_col_c<R, L, MODE, 2>;
        set_lds(k, lds);
        hipLaunchKernelGGL(k, grid, dim3(b.CB * T), lds, st, bb, mplan_table<R>(c, L).tw);
    } else {
        auto k = k_col_c<R, L, MODE, 1>;
        set_lds(k, lds);
        hipLaunchKernelGGL(k, grid, dim3(b.CB * T), lds, st, bb, mplan_table<R>(c, L).tw);
    }
    KRY_HIP(hipGetLastError());
}

template <typename R, int IN>
static void launch_row_fwd_m(const StageAArgs& a, dim3 grid, const RowTiling& t, const MPlan& pl, Ctx& c,
                             hipStream_t st) {
    auto k = k_row_fwd_m<R, IN>;
    set_lds(k, t.lds);
    const MTable<R> tb = mplan_table<R>(c, pl.L);
    hipLaunchKernelGGL(k, grid, dim3(t.threads), t.lds, st, a, tb.tw, tb.plan);
    KRY_HIP(hipGetLastError());
}

template <typename R, int OUT, int R0>
static void launch_row_inv_mr(const StageCArgs& a, dim3 grid, const RowTiling& t, const MPlan& pl, Ctx& c,
                              hipStream_t st) {
    auto k = k_row_inv_m<R, OUT, R0>;
    set_lds(k, t.lds);
    const MTable<R> tb = mplan_table<R>(c, pl.L);
    hipLaunchKernelGGL(k, grid, dim3(t.threads), t.lds, st, a, tb.tw, tb.plan);
    KRY_HIP(hipGetLastError());
}

// (the first inverse pass's radix is the plan's last forward radix: 2, 3, 4,
// 5 or 7 for a length that is not a power of two)
template <typename R, int OUT>
static void launch_row_inv_m(const StageCArgs& a, dim3 grid, const RowTiling& t, const MPlan& pl, Ctx& c,
                             hipStream_t st) {
    switch (pl.radix[pl.npass - 1]) {
        case 2: launch_row_inv_mr<R, OUT, 2>(a, grid, t, pl, c, st); break;
        case 3: launch_row_inv_mr<R, OUT, 3>(a, grid, t, pl, c, st); break;
        case 4: launch_row_inv_mr<R, OUT, 4>(a, grid, t, pl, c, st); break;
        case 5: launch_row_inv_mr<R, OUT, 5>(a, grid, t, pl, c, st); break;
        case 7: launch_row_inv_mr<R, OUT, 7>(a, grid, t, pl, c, st); break;
        default: throw Error(KRY_EINVAL, "mixed-radix plan without a non-8 last pass");
    }
}

template <typename R, int MODE, int V, int RI, int TMAX>
static void launch_col_mk(const StageBArgs& bb, dim3 grid, int threads, size_t lds, const MPlan& pl, Ctx& c,
                          hipStream_t st) {
    auto k = k_col_m<R, MODE, V, RI, TMAX>;
    set_lds(k, lds);
    const MTable<R> tb = mplan_table<R>(c, pl.L);
    hipLaunchKernelGGL(k, grid, dim3(threads), lds, st, bb, tb.tw, tb.plan);
    KRY_HIP(hipGetLastError());
}

template <typename R, int MODE, int V, int RI>
static void launch_col_mt(const StageBArgs& bb, dim3 grid, int threads, size_t lds, const MPlan& pl, Ctx& c,
                          hipStream_t st) {
    if (threads <= 256) launch_col_mk<R, MODE, V, RI, 256>(bb, grid, threads, lds, pl, c, st);
    else if constexpr (V == 1) {
        if (threads <= 512) launch_col_mk<R, MODE, 1, RI, 512>(bb, grid, threads, lds, pl, c, st);
        else if (threads <= 768) launch_col_mk<R, MODE, 1, RI, 768>(bb, grid, threads, lds, pl, c, st);
        else launch_col_mk<R, MODE, 1, RI, 1024>(bb, grid, threads, lds, pl, c, st);
    } else {
        throw Error(KRY_EINVAL, "two column vectors per workgroup take columns of at most 2048 points");
    }
}

template <typename R, int MODE, int V>
static void launch_col_mv(const StageBArgs& bb, dim3 grid, int threads, size_t lds, const MPlan& pl, Ctx& c,
                          hipStream_t st) {
    switch (pl.radix[pl.npass - 1]) {
        case 2: launch_col_mt<R, MODE, V, 2>(bb, grid, threads, lds, pl, c, st); break;
        case 3: launch_col_mt<R, MODE, V, 3>(bb, grid, threads, lds, pl, c, st); break;
        case 4: launch_col_mt<R, MODE, V, 4>(bb, grid, threads, lds, pl, c, st); break;
        case 5: launch_col_mt<R, MODE, V, 5>(bb, grid, threads, lds, pl, c, st); break;
        case 7: launch_col_mt<R, MODE, V, 7>(bb, grid, threads, lds, pl, c, st); break;
        default: throw Error(KRY_EINVAL, "mixed-radix plan without a non-8 last pass");
    }
}

// Columns of a mixed-radix length: V = 2 vectors per workgroup where their
// LDS fits and the column has at most 2048 points, else one.
template <typename R, int MODE>
static void launch_col_m(const StageBArgs& b, int nvec, int V, const MPlan& pl, Ctx& c, hipStream_t st) {
    const int threads = b.CB * pl.T;
    const size_t per = (size_t)b.CB * lpadded<cpx<R>>(pl.L) * sizeof(cpx<R>);
    if (MODE == B_SPEC || 2 * per > 160 * 1024 || threads > 256) V = 1;
    const size_t lds = per * V;
    dim3 grid((b.ncols + b.CB - 1) / b.CB, (nvec + V - 1) / V);
    StageBArgs bb = b;
    bb.nvec = nvec;
    if constexpr (MODE != B_SPEC) {
        if (V == 2) {
            launch_col_mv<R, MODE, 2>(bb, grid, threads, lds, pl, c, st);
            return;
        }
    }
    launch_col_mv<R, MODE, 1>(bb, grid, threads, lds, pl, c, st);
}

#define KRY_SIZES(X) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)

template <typename R>
static void run_stage_a(Problem& P, const ConvSpec& s, int vec0, int nvec, cpx<R>* Y, int ldY, int64_t Yvs,
                        const RowTiling& t, int vt, bool split, hipStream_t st) {
    const int M = s.N2 / 2;
    StageAArgs a;
    a.in = (const void*)((const R*)s.in + vec0 * s.in_vstride);
    if (s.in_mode == IN_NOISE) a.in = nullptr;
    a.in_vstride = s.in_vstride;
    a.in_rstride = s.in_rstride;
    a.mask = P.mask_view();
    a.rows_in = s.rows_in;
    a.row_len = s.row_len;
    a.RT = t.RT;
    a.log2RT = ilog2(t.RT);
    a.Y = Y;
    a.ldY = ldY;
    a.Y_vstride = Yvs;
    a.seed = s.seed;
    a.stream0 = s.stream0;
    a.vec0 = vec0;
    a.tab = s.tab;
    a.tab_vpp = s.tab_vpp;
    a.active = s.active ? s.active + vec0 : nullptr;
    KRY_REQUIRE(!s.upd_r || (s.in_mode == IN_COMPACT && sizeof(R) == 8 && s.upd_beta && !s.tab),
                "the direction update takes compact FP64 inputs of one problem");
    a.upd_r = s.upd_r ? (const void*)((const R*)s.upd_r + vec0 * s.in_vstride) : nullptr;
    a.upd_beta = s.upd_beta;
    dim3 grid((s.rows_in + t.RT - 1) / t.RT, nvec);
    const int lg = ilog2(M);
    Ctx& c = *P.ctx;
    if (is_ct_row(M)) {
        switch (M) {
#define KRY_AC(X)                                                                                   \
    case X:                                                                                         \
        if (s.in_mode == IN_COMPACT) launch_row_fwd_c<R, X, IN_COMPACT>(a, grid, t, c, st);           \
        else if (s.in_mode == IN_DENSE) launch_row_fwd_c<R, X, IN_DENSE>(a, grid, t, c, st);          \
        else launch_row_fwd_c<R, X, IN_NOISE>(a, grid, t, c, st);                                    \
        break;
            KRY_CROWS(KRY_AC)
#undef KRY_AC
        }
        return;
    }
    if (!is_pow2(M)) {
        const MPlan pl = mixed_plan(M);
        if (s.in_mode == IN_COMPACT) launch_row_fwd_m<R, IN_COMPACT>(a, grid, t, pl, c, st);
        else if (s.in_mode == IN_DENSE) launch_row_fwd_m<R, IN_DENSE>(a, grid, t, pl, c, st);
        else launch_row_fwd_m<R, IN_NOISE>(a, grid, t, pl, c, st);
        return;
    }
#define KRY_A(LG)                                                                             \
    case LG:                                                                                  \
        if (s.in_mode == IN_COMPACT) launch_row_fwd<R, LG, IN_COMPACT>(a, grid, t, vt, split, c, st);\
        else if (s.in_mode == IN_DENSE) launch_row_fwd<R, LG, IN_DENSE>(a, grid, t, vt, split, c, st);\
        else launch_row_fwd<R, LG, IN_NOISE>(a, grid, t, vt, split, c, st);                   \
        break;
    switch (lg) {
        KRY_SIZES(KRY_A)
        default: throw Error(KRY_EINVAL, "row transform length out of range");
    }
#undef KRY_A
}

template <typename R>
static void run_stage_b(Problem& P, int N1, int M, int vec0, int nvec, cpx<R>* Y, int ldY, int64_t Yvs, int rows_in,
                        int rows_out, const void* lam, int64_t lam_tstride, int vpt, double* spec_out,
                        hipStream_t st, const ProbDesc* tab = nullptr, int tab_vpp = 1,
                        const int* active = nullptr, int V = 1, bool split = false, bool lam_even = false,
                        double* pw_out = nullptr) {
    const int T = N1 / 8;
    StageBArgs b;
    b.Y = Y;
    b.ldY = ldY;
    b.Y_vstride = Yvs;
    b.ncols = M + 1;
    b.rows_in = rows_in;
    b.rows_out = rows_out;
    b.CB = T >= 256 ? 1 : 256 / T;
    b.lam = lam;
    b.lam_tstride = lam_tstride;
    b.vecs_per_theta = vpt;
    b.lam_even = lam_even && !tab && !spec_out ? 1 : 0;
    b.vec0 = vec0;
    b.spec_out = spec_out;
    b.pw_out = nullptr;
    if (pw_out) {
        KRY_REQUIRE(sizeof(R) == 8 && is_pow2(N1) && !tab && !spec_out,
                    "spectral quadratic forms need FP64 power-of-two columns");
        b.pw_out = pw_out;
    }
    b.tab = tab;
    b.tab_vpp = tab_vpp;
    b.active = active ? active + vec0 : nullptr;
    const int mode = spec_out ? B_SPEC : (2 * rows_in <= N1 ? B_LOW : B_FULL);
    const int lg = ilog2(N1);
    Ctx& c = *P.ctx;
    if (is_ct_col(N1)) {
        switch (N1) {
#define KRY_BC(X)                                                                 \
    case X:                                                                       \
        if (mode == B_LOW) launch_col_c<R, X, B_LOW>(b, nvec, V, c, st);          \
        else if (mode == B_FULL) launch_col_c<R, X, B_FULL>(b, nvec, V, c, st);   \
        else launch_col_c<R, X, B_SPEC>(b, nvec, 1, c, st);                       \
        break;
            KRY_CCOLS(KRY_BC)
#undef KRY_BC
        }
        return;
    }
    if (!is_pow2(N1)) {
        const MPlan pl = mixed_plan(N1);
        if (mode == B_LOW) launch_col_m<R, B_LOW>(b, nvec, V, pl, c, st);
        else if (mode == B_FULL) launch_col_m<R, B_FULL>(b, nvec, V, pl, c, st);
        else launch_col_m<R, B_SPEC>(b, nvec, 1, pl, c, st);
        return;
    }
#define KRY_B(LG)                                                                          \
    case LG + 1:                                                                           \
        if (mode == B_LOW) launch_col<R, LG + 1, B_LOW>(b, nvec, V, split, c, st);         \
        else if (mode == B_FULL) launch_col<R, LG + 1, B_FULL>(b, nvec, V, split, c, st);  \
        else launch_col<R, LG + 1, B_SPEC>(b, nvec, 1, false, c, st);                      \
        break;
    switch (lg) {
        KRY_SIZES(KRY_B)
        default: throw Error(KRY_EINVAL, "column transform length out of range");
    }
#undef KRY_B
}

template <typename R>
static void run_stage_c(Problem& P, const ConvSpec& s, int vec0, int nvec, cpx<R>* Y, int ldY, int64_t Yvs,
                        const RowTiling& t, int vt, bool split, hipStream_t st) {
    const int M = s.N2 / 2;
    StageCArgs c;
    c.Y = Y;
    c.ldY = ldY;
    c.Y_vstride = Yvs;
    c.rows_out = s.rows_out;
    c.cols_out = s.cols_out;
    c.RT = t.RT;
    c.log2RT = ilog2(t.RT);
    c.mask = P.mask_view();
    c.vin = s.vin ? (const void*)((const R*)s.vin + vec0 * s.vin_vstride) : nullptr;
    c.vin_vstride = s.vin_vstride;
    c.eta = s.eta;
    c.vecs_per_theta = s.vecs_per_theta;
    c.vec0 = vec0;
    c.out = (void*)((R*)s.out + vec0 * s.out_vstride);
    c.out_vstride = s.out_vstride;
    c.scale = s.scale;
    c.tab = s.tab;
    c.tab_vpp = s.tab_vpp;
    c.active = s.active ? s.active + vec0 : nullptr;
    dim3 grid((s.rows_out + t.RT - 1) / t.RT, nvec);
    const int lg = ilog2(M);
    Ctx& cx = *P.ctx;
    if (is_ct_row(M)) {
        switch (M) {
#define KRY_CC(X)                                                                              \
    case X:                                                                                    \
        if (s.out_mode == OUT_COMPACT) launch_row_inv_c<R, X, OUT_COMPACT>(c, grid, t, cx, st); \
        else launch_row_inv_c<R, X, OUT_GRID>(c, grid, t, cx, st);                             \
        break;
            KRY_CROWS(KRY_CC)
#undef KRY_CC
        }
        return;
    }
    if (!is_pow2(M)) {
        const MPlan pl = mixed_plan(M);
        if (s.out_mode == OUT_COMPACT) launch_row_inv_m<R, OUT_COMPACT>(c, grid, t, pl, cx, st);
        else launch_row_inv_m<R, OUT_GRID>(c, grid, t, pl, cx, st);
        return;
    }
#define KRY_C(LG)                                                                             \
    case LG:                                                                                  \
        if (s.out_mode == OUT_COMPACT) launch_row_inv<R, LG, OUT_COMPACT>(c, grid, t, vt, split, cx, st);\
        else launch_row_inv<R, LG, OUT_GRID>(c, grid, t, vt, split, cx, st);                  \
        break;
    switch (lg) {
        KRY_SIZES(KRY_C)
        default: throw Error(KRY_EINVAL, "row transform length out of range");
    }
#undef KRY_C
}

template <typename R>
void conv_apply(Problem& P, const ConvSpec& s, hipStream_t st) {
    KRY_REQUIRE(torus_side_ok(s.N1) && torus_side_ok(s.N2),
                "torus sides must be supported transform lengths (16..8192: powers of two or multiples of 16 of the form 2^a 3^b 5^c 7^d)");
    KRY_REQUIRE(s.rows_in <= s.N1 && s.row_len <= s.N2 && s.rows_out <= s.N1 && s.cols_out <= s.N2,
                "block larger than the torus");
    KRY_REQUIRE(s.in_mode != IN_COMPACT || 2 * s.row_len <= s.N2, "compact input wider than half the torus");
    KRY_REQUIRE(!s.tab || (s.in_mode == IN_COMPACT && s.tab_vpp >= 1), "problem tables take compact inputs");
    KRY_REQUIRE(!P.irregular || (s.in_mode != IN_COMPACT && s.out_mode != OUT_COMPACT),
                "irregular problems have no observation mask");
    if (s.nvec <= 0) return;
    const int M = s.N2 / 2;
    // launch configuration of this embedding and precision (bit-identical results)
    const Tuning tu = P.ctx->tuning_for(s.N1, s.N2, (int)sizeof(R), s.nvec);
    // (two value sets and split exchanges: power-of-two rows of >= 1024 points)
    const bool wide = M >= 1024 && is_pow2(M);
    const int vt = (wide && tu.row_vt == 2) ? 2 : 1;
    // (two vectors per column workgroup only when there are two to pair)
    const int V = s.nvec < 2 ? 1 : (tu.col_v ? tu.col_v : (sizeof(R) == 4 ? 2 : 1));
    const bool asplit = wide && (tu.row_split & 1) != 0;
    const bool csplit = wide && (tu.row_split & 2) != 0;
    const RowTiling ta = row_tiling<R>(M, tu.rt_scale, vt, asplit);
    const RowTiling tc = row_tiling<R>(M, tu.rt_scale, vt, csplit);  // same rows per tile
    const int rows_max = s.rows_in > s.rows_out ? s.rows_in : s.rows_out;
    const int ldY = ((rows_max + ta.RT - 1) / ta.RT) * ta.RT;
    const int64_t Yvs = (int64_t)(M + 1) * ldY;
    // vectors go through in chunks that keep the intermediate near 4 GB (or
    // within the caller's workspace)
    const int64_t per_vec = Yvs * (int64_t)sizeof(cpx<R>);
    int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(s.nvec, (int64_t)(4LL << 30) / per_vec));
    chunk = std::min(chunk, 65535);
    cpx<R>* Y;
    if (s.ws) {
        const int64_t fit = (int64_t)(s.ws_bytes / (size_t)per_vec);
        KRY_REQUIRE(fit >= 1, "workspace smaller than one vector's transform intermediate (" +
                                  std::to_string(per_vec) + " bytes)");
        chunk = (int)std::min<int64_t>(chunk, fit);
        Y = static_cast<cpx<R>*>(s.ws);
    } else {
        P.Y.ensure(*P.ctx, (size_t)Yvs * chunk * sizeof(cpx<R>));
        Y = P.Y.as<cpx<R>>();
    }
    StageProfile& pr = P.ctx->prof;
    const bool timing = pr.on && !s.ws;  // (recording events would create them)
    for (int v0 = 0; v0 < s.nvec; v0 += chunk) {
        const int nv = std::min(chunk, s.nvec - v0);
        std::array<int, 5> rec{};
        auto mark = [&](int slot) {
            if (!timing) return;
            if (pr.next == pr.pool.size()) {
                hipEvent_t e;
                KRY_HIP(hipEventCreate(&e));
                pr.pool.push_back(e);
            }
            rec[slot] = (int)pr.next;
            KRY_HIP(hipEventRecord(pr.pool[pr.next++], st));
        };
        mark(0);
        run_stage_a<R>(P, s, v0, nv, Y, ldY, Yvs, ta, vt, asplit, st);
        mark(1);
        run_stage_b<R>(P, s.N1, M, v0, nv, Y, ldY, Yvs, s.rows_in, s.rows_out, s.lam, s.lam_tstride,
                       s.vecs_per_theta, nullptr, st, s.tab, s.tab_vpp, s.active, V,
                       tu.col_split != 0 && is_pow2(s.N1), s.lam_even, s.pw_out);
        mark(2);
        run_stage_c<R>(P, s, v0, nv, Y, ldY, Yvs, tc, vt, csplit, st);
        mark(3);
        if (timing) {
            rec[4] = nv;
            pr.recs.push_back(rec);
        }
    }
}

template void conv_apply<double>(Problem&, const ConvSpec&, hipStream_t);
template void conv_apply<float>(Problem&, const ConvSpec&, hipStream_t);

template <typename R>
size_t conv_bytes_per_vec(int N1, int N2, int rows, Ctx& c, int nvec) {
    const int M = N2 / 2;
    const Tuning tu = c.tuning_for(N1, N2, (int)sizeof(R), nvec);
    const bool wide = M >= 1024 && is_pow2(M);
    const int vt = (wide && tu.row_vt == 2) ? 2 : 1;
    const bool asplit = wide && (tu.row_split & 1) != 0;
    const RowTiling ta = row_tiling<R>(M, tu.rt_scale, vt, asplit);
    const int ldY = ((rows + ta.RT - 1) / ta.RT) * ta.RT;
    return (size_t)(M + 1) * ldY * sizeof(cpx<R>);
}
template size_t conv_bytes_per_vec<double>(int, int, int, Ctx&, int);
template size_t conv_bytes_per_vec<float>(int, int, int, Ctx&, int);

// ---------------------------------------------------------------------------
// Lag grid and spectrum
// ---------------------------------------------------------------------------
void lag_grid_device(Ctx& c, int N1, int N2, double dx1, double dx2, const Matern& th, double* d_c,
                     hipStream_t st, bool drange) {
    (void)c;
    MaternDev m;
    m.drange = drange ? 1 : 0;
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

// lam[k2][k1] = lam[k2][N1 - k1] for N1 / 2 < k1 < N1 (N1 even): the
// spectrum of a covariance even in the row lag is even in k1; the transform
// leaves the two halves equal only to rounding, and the fold makes them equal
// bit for bit.
__global__ void k_fold_even(double* __restrict__ lam, int N1, int ncols) {
    const int h = N1 / 2 - 1;  // mirrored entries per column
    const int64_t n = (int64_t)ncols * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(i / h), k1 = N1 / 2 + 1 + (int)(i - (int64_t)col * h);
        lam[(int64_t)col * N1 + k1] = lam[(int64_t)col * N1 + (N1 - k1)];
    }
}

// The covariance is even in each lag separately (c(h1, h2) = c(-h1, h2)) when
// it is isotropic or its anisotropy axes are the grid's.
bool matern_even(const Matern& th) { return th.ratio == 1.0 || th.angle == 0.0; }

size_t spectrum_ws_bytes(int N1, int N2) {
    const int M = N2 / 2;
    const RowTiling ta = row_tiling<double>(M);
    const int ldY = ((N1 + ta.RT - 1) / ta.RT) * ta.RT;
    const size_t lag = ((size_t)N1 * N2 * sizeof(double) + 255) & ~size_t(255);
    return lag + (size_t)(M + 1) * ldY * sizeof(cpx<double>) + 1024 * 2 * sizeof(double);
}

void spectrum_device(Problem& P, int N1, int N2, const Matern& th, double* d_lam, double* lam_min,
                     double* lam_max, hipStream_t st, bool drange, void* ws) {
    Ctx& C = *P.ctx;
    const int M = N2 / 2;
    // stage A over every row of the lag grid, then the forward column pass
    const RowTiling ta = row_tiling<double>(M);
    const int ldY = ((N1 + ta.RT - 1) / ta.RT) * ta.RT;
    const int64_t Yvs = (int64_t)(M + 1) * ldY;
    double* lag;
    cpx<double>* Y;
    if (ws) {
        lag = static_cast<double*>(ws);
        Y = reinterpret_cast<cpx<double>*>(static_cast<char*>(ws) +
                                           (((size_t)N1 * N2 * sizeof(double) + 255) & ~size_t(255)));
    } else {
        P.lagtmp.ensure(C, (size_t)N1 * N2 * sizeof(double));
        P.spectmp.ensure(C, (size_t)Yvs * sizeof(cpx<double>) + 1024 * 2 * sizeof(double));
        lag = P.lagtmp.as<double>();
        Y = P.spectmp.as<cpx<double>>();
    }
    lag_grid_device(C, N1, N2, P.dx1, P.dx2, th, lag, st, drange);
    ConvSpec s;
    s.N1 = N1;
    s.N2 = N2;
    s.nvec = 1;
    s.in_mode = IN_DENSE;
    s.in = lag;
    s.in_vstride = 0;
    s.in_rstride = N2;
    s.rows_in = N1;
    s.row_len = N2;
    run_stage_a<double>(P, s, 0, 1, Y, ldY, Yvs, ta, 1, false, st);
    run_stage_b<double>(P, N1, M, 0, 1, Y, ldY, Yvs, N1, N1, nullptr, 0, 1, d_lam, st);
    if (matern_even(th)) {
        const int64_t n = (int64_t)(M + 1) * (N1 / 2 - 1);
        int64_t blocks = (n + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        if (n > 0) {
            hipLaunchKernelGGL(k_fold_even, dim3((unsigned)blocks), dim3(256), 0, st, d_lam, N1, M + 1);
            KRY_HIP(hipGetLastError());
        }
    }
    if (!lam_min) return;
    // min / max
    double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(Y) + (size_t)Yvs * sizeof(cpx<double>));
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
