// Declarations of the batched Krylov building blocks (krylov.hip).
#pragma once
#include <functional>
#include <vector>

#include "internal.hpp"

namespace kry {

constexpr int KRY_MAX_LANCZOS = 512;

// y_v = K x_v for nvec vectors of length n (contiguous, stride n).
template <typename R>
using MatvecFn = std::function<void(const R* x, R* y, int nvec, hipStream_t st)>;

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

template <typename R>
void lanczos_run(const MatvecFn<R>& A, int64_t n, int nvec, int m, bool reorth, const R* Z, LanczosBuffers<R>& B,
                 hipStream_t st);
void quadrature(const double* alpha, const double* beta, const int* steps, const double* znorm2, int nvec,
                int64_t coef_stride, double* gamma, hipStream_t st);
// CG on nvec systems; vector v stops at ||r|| <= rtol ||b|| or after
// limits[v] iterations (limits == nullptr: maxit for all).
template <typename R>
void cg_run(const MatvecFn<R>& A, int64_t n, int nvec, const R* b, R* x, double rtol, int maxit, CgBuffers<R>& B,
            std::vector<int>& iters, std::vector<double>& relres, hipStream_t st,
            const std::vector<int>* limits = nullptr);
template <typename R>
void make_probes(const Problem& P, int nprobe, uint64_t seed, int period, R* out, hipStream_t st);
template <typename A, typename B>
void convert(const A* x, B* y, int64_t n, hipStream_t st);
template <typename R>
void axpby(const R* x, R* y, double a, double b, int64_t n, int nvec, hipStream_t st);
void add_f32(const float* d, double* x, int64_t n, hipStream_t st);

}  // namespace kry
