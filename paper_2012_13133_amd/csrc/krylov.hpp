// Declarations of the batched Krylov building blocks (krylov.hip).
#pragma once
#include <functional>
#include <vector>

#include "internal.hpp"

namespace kry {

constexpr int KRY_MAX_LANCZOS = 1024;

// y_v = K x_v for nvec vectors of length n (contiguous, stride n).  With
// active (device, nvec flags) given, vectors whose flag is 0 may be skipped:
// their y is left unspecified.
template <typename R>
using MatvecFn = std::function<void(const R* x, R* y, int nvec, hipStream_t st, const int* active)>;

// Device buffers of one batched Lanczos run.  Coefficients are stored
// step-major: alpha[j * nvec + v].
template <typename R>
struct LanczosBuffers {
    R* Q;            // (reorth ? m + 1 : 3) slots of nvec x n
    R* W;            // nvec x n
    double* alpha;   // m x nvec
    double* beta;    // m x nvec
    double* znorm2;  // nvec
    double* scale;   // nvec
    int* active;     // nvec
    int* steps;      // nvec
    double* partial; // nvec x (m + 1) x nblk
    double* h;       // nvec x (m + 1)
};

template <typename R>
struct CgBuffers {
    R *r, *p, *w;
    double *rr, *bnorm2, *beta, *pw, *tmp, *partial;
    int *active, *iters;
    int* limit;  // per-vector iteration cap (device, nvec)
};

// Multi-shift CG: for shifts s, each tied to a group g whose base operator
// A_g supplies the shared Krylov space of the group's right-hand side
// b_g = D_{rhs(g)} (one of nd vectors D_0..D_{nd-1}),
//   Q[s * nd + j] = D_j^T (A_g + sigma_s I)^{-1} b_g    for j < nd,
// from scalar recurrences; the shifted solutions themselves are not formed.
// Group state lives at packed positions 0..G-1; a group whose shifts have all
// stopped is moved behind the active ones so products run on active groups
// only.  All FP64.
constexpr int KRY_MS_MAX_ND = 9;
struct MsCgBuffers {
    double *r, *p, *w;      // G x n, by position
    double *rr, *rc, *pw, *alpha, *alpha_old, *beta, *beta_old, *bnorm2;  // G (rc: (1 + nd) G), by position
    double *zeta, *zeta_old, *zeta_new, *alpha_s, *sigma, *relres;        // S
    double *d, *Q;                                                        // S x nd
    int *active, *iters, *limit, *pos, *list;                             // S
    double* gram;           // nd x nd
    int* rhs;               // G
    double* partial;        // (1 + nd) G x nblk (at least nd x nd x nblk)
    double* partial_pw;     // G x npw: p . w partials (npw: nblk, or what the fused product writes),
                            // read while the residual kernel writes `partial`
};
// Arguments of an iteration's scalar step (see ms_scalar_step).
struct MsScalarArgs {
    int Gact, nd, nblk, nlist, nS;  // nS: every shift, listed or not
    int npw;                         // p . w partials per position
    const double* partial_pw;
    double* partial;
    double *rr, *rc, *pw, *beta, *alpha, *alpha_old, *beta_old;
    const double* bnorm2;
    const int *list, *pos;
    const double* sigma;
    double *zeta, *zeta_old, *zeta_new, *alpha_s, *d, *Q, *relres;
    int *active, *iters;
    const int* limit;
    double rtol;
};
// The base product with the direction update folded into it: applies the
// operators of positions 0..k-1 to p after replacing p by r + beta p (per
// position), as the update would have done.  With pw non-null it also
// writes, per position, the partials of p . w (the count mscg_run is told),
// whose sum in order is the quadratic form of the updated p.
using MsFusedFn = std::function<void(const double* r, double* p, const double* beta, double* w, int k, double* pw,
                                     hipStream_t st)>;
// A(x, y, k, st) applies the base operators of positions 0..k-1;
// swap(a, b) exchanges whatever the caller keeps per position (spectra).
// D: nd (<= KRY_MS_MAX_ND) vectors of n, contiguous; rhs_of_group: index of
// each group's right-hand side in D.
// With `fused` (nullable) the products go through it and the direction
// update has no pass of its own; with fused_pw > 0 as well, the fused product
// writes fused_pw partials of p . w per position and the dot pass is skipped
// (B.partial_pw then holds G x max(nblk, fused_pw)).
void mscg_run(const MatvecFn<double>& A, const MsFusedFn* fused, int fused_pw,
              const std::function<void(int, int)>& swap,
              int64_t n, int G,
              const std::vector<int>& group_of_shift, const std::vector<double>& sigma, const double* D, int nd,
              const std::vector<int>& rhs_of_group, double rtol, int maxit, MsCgBuffers& B, std::vector<int>& iters,
              std::vector<double>& relres, std::vector<double>& Q, hipStream_t st);
// ---- irregularly spaced observations (irregular.hip) ----------------------------
// K x = A Sigma A^T x + eta x for compact vectors of an irregular problem:
// A^T by rows over the grid (FP64 sums), the circulant-embedding product on
// the grid, A by its four-slot rows (FP64 sums) plus the nugget term.
template <typename R>
MatvecFn<R> irregular_op(Problem& P, const void* lam, int64_t lam_tstride, int vpt, const double* d_eta);
// out (nvec grid vectors, stride n) = scale * A^T x (x: nvec compact, stride xs).
template <typename RI, typename RO>
void irr_scatter(const Problem& P, const RI* x, int64_t xs, int nvec, RO* out, double scale, const int* active,
                 hipStream_t st);
// out (nvec compact, stride p) = A grid (+ eta[v / vpt] xin when xin).
template <typename RI, typename RO>
void irr_gather(const Problem& P, const RI* grid, int nvec, RO* out, const RO* xin, const double* eta, int vpt,
                const int* active, hipStream_t st);
// out[v * p + j] = (A Sigma e_t)_j for target cell t = targets[v], from the
// embedding lag grid (row-major N1 x N2).
void irr_cross_corr(const Problem& P, const double* lag, const int64_t* targets, int nt, double* out,
                    hipStream_t st);
// dst[v][i] = src[v][obs_user[i]] (to the stored order; gather) or
// dst[v][obs_user[i]] = src[v][i] (back to the caller's order).
template <typename R>
void irr_permute(const Problem& P, const R* src, R* dst, int nvec, bool to_stored, hipStream_t st);
// y_b = A x_b + tau eps_b (eps from Philox stream b, domain NOISE, the
// caller's observation index).
void irr_boot_obs(const Problem& P, const double* fields, int B, double tau, uint64_t seed, double* yb,
                  hipStream_t st);

// Exchange vectors a and b (each n elements) of base + k * stride.
template <typename T>
void swap_vectors(T* base, int64_t stride, int a, int b, int64_t n, hipStream_t st);

// Adaptive stopping for lanczos_run: after every 5th step from step 10 on,
// the quadrature values of nout outputs (output v reads recurrence src[v]
// shifted by shift[v], or v itself when src is NULL) are compared with those
// 5 steps earlier; a point (per_point consecutive outputs) settles at the
// first check where all of its outputs moved by at most rtol times their
// size, and keeps those values (g_final) and that step (stop, 0 = not
// settled).  The run ends when every point has settled or at m steps.
struct LanczosAdaptive {
    double rtol;
    int nout, per_point;
    const int* src;
    const double* shift;
    double *g_prev, *g_cur, *g_final;  // nout each (device)
    int* stop;                         // nout / per_point (device)
    int* done;                         // 1 (device)
};

template <typename R>
void lanczos_run(const MatvecFn<R>& A, int64_t n, int nvec, int m, bool reorth, const R* Z, LanczosBuffers<R>& B,
                 hipStream_t st, const LanczosAdaptive* ad = nullptr);
// gamma for nvec outputs; output v uses recurrence src[v] shifted by
// shift[v] when those (device) arrays are given.
void quadrature(const double* alpha, const double* beta, const int* steps, const double* znorm2, int nvec,
                int64_t coef_stride, double* gamma, hipStream_t st, const int* src = nullptr,
                const double* shift = nullptr);
// CG on nvec systems; vector v stops at ||r|| <= rtol ||b|| or after
// limits[v] iterations (limits == nullptr: maxit for all).  graphs: replay
// a captured graph for each block of 16 iterations after the first (the
// operator must then launch the same kernels with the same arguments on
// every call and allocate nothing after its first call).
template <typename R>
void cg_run(const MatvecFn<R>& A, int64_t n, int nvec, const R* b, R* x, double rtol, int maxit, CgBuffers<R>& B,
            std::vector<int>& iters, std::vector<double>& relres, hipStream_t st,
            const std::vector<int>* limits = nullptr, bool graphs = false);
// Probe k of the problem at out + k * stride (stride 0: the problem's p).
template <typename R>
void make_probes(const Problem& P, int nprobe, uint64_t seed, int period, R* out, hipStream_t st,
                 int64_t stride = 0);
template <typename A, typename B>
void convert(const A* x, B* y, int64_t n, hipStream_t st);
template <typename R>
void axpby(const R* x, R* y, double a, double b, int64_t n, int nvec, hipStream_t st);
void add_f32(const float* d, double* x, int64_t n, hipStream_t st);

}  // namespace kry
