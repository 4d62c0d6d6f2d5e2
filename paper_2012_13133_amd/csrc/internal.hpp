// Host-side structures shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <functional>
#include <map>
#include <tuple>
#include <cstdint>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/kryging.h"
#include "common.hpp"

namespace kry {

// Error carried from the drivers to the ABI boundary, where it becomes a
// kry_status and a thread-local message.
struct Error : std::runtime_error {
    kry_status status;
    Error(kry_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define KRY_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::kry::Error(KRY_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define KRY_REQUIRE(cond, msg)                                        \
    do {                                                              \
        if (!(cond)) throw ::kry::Error(KRY_EINVAL, std::string(msg)); \
    } while (0)

// Per-stage timing of the masked product: events recorded around each
// stage launch while profiling is on, summed when read back.
struct StageProfile {
    bool on = false;
    std::vector<hipEvent_t> pool;          // reusable events
    std::vector<std::array<int, 5>> recs;  // event indices: A0, B0, C0, C1 per product, + nvec
    size_t next = 0;
};

// Launch configuration of the product's stage kernels (see kry_tuning).
struct Tuning {
    int col_v = 0;       // 0: default for the precision
    int rt_scale = 1;
    int row_vt = 1;
    int col_split = 0;   // column stage exchanges real and imaginary parts separately
    int row_split = 0;   // row stages likewise: bit 0 stage A, bit 1 stage C (rows of >= 1024 points)
    double ms = 0.0;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    StageProfile prof;
    uint64_t budget = 0;     // 0 = unlimited
    uint64_t allocated = 0;  // bytes currently held through dev_alloc
    uint64_t peak = 0;       // largest `allocated` since creation or the last reset
    cpx<double>* tw64 = nullptr;
    cpx<float>* tw32 = nullptr;
    void* plan64[14] = {};  // per-length pass twiddle tables (index log2 length)
    void* plan32[14] = {};
    std::map<int, void*> mplan64, mplan32;  // mixed-radix lengths' tables (by length)
    std::mutex alloc_mu;     // guards `allocated` (server slots allocate concurrently)
    bool graphs = true;  // replay captured graphs for CG iteration blocks
    // (N1, N2, bytes per real, batch class) -> configuration; class 0 holds
    // the setting for products of at most kSmallBatch vectors, class 1 the rest
    std::map<std::tuple<int, int, int, int>, Tuning> tuning;
    std::mutex tune_mu;
    static constexpr int kSmallBatch = 8;
    static int batch_class(int nvec) { return nvec <= kSmallBatch ? 0 : 1; }
    void* scratch = nullptr;  // device address of the no-allocation product's scratch array
    int embed_rule = KRY_EMBED_FAST;  // how new problems choose their embedding sides
    // The setting for products of nvec vectors: that batch class's, else the
    // other class's, else the built-in default.
    Tuning tuning_for(int N1, int N2, int real_bytes, int nvec = 1 << 30) {
        std::lock_guard<std::mutex> g(tune_mu);
        const int cls = batch_class(nvec);
        auto it = tuning.find(std::make_tuple(N1, N2, real_bytes, cls));
        if (it == tuning.end()) it = tuning.find(std::make_tuple(N1, N2, real_bytes, 1 - cls));
        return it == tuning.end() ? Tuning{} : it->second;
    }
};

void* dev_alloc(Ctx& c, size_t bytes);
void dev_free(Ctx& c, void* p, size_t bytes);
// Device address of the no-allocation product's scratch array on `device`
// (the current device), looked up once per device.
void* noalloc_scratch_init(int device);
// Runs f, turning an exception into a status and the thread's error message.
kry_status run_guarded(const std::function<void()>& f);

// A device buffer that only grows; freed with its owner.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    void ensure(Ctx& c, size_t need) {
        if (need <= bytes) return;
        if (ptr) dev_free(c, ptr, bytes);
        ptr = nullptr;
        bytes = 0;
        ptr = dev_alloc(c, need);
        bytes = need;
    }
    void release(Ctx& c) {
        if (ptr) dev_free(c, ptr, bytes);
        ptr = nullptr;
        bytes = 0;
    }
    template <typename T>
    T* as() const { return reinterpret_cast<T*>(ptr); }
};

struct Matern {
    double sigma2, tau2, range, nu, ratio, angle;
};

// Spectrum of one parameter point on the problem's embedding, scaled by
// 1 / (N1 N2) for the product, in both precisions; layout [k2][k1].
struct Spectrum {
    Matern theta{};
    bool valid = false;
    double lam_min = 0, lam_max = 0;
    DevBuf s64, s32;
};

// One problem of a product over several problems that share an embedding:
// its packed mask, grid block, observed count and spectra.  Compact vectors
// of such a product are stored with a common stride (the largest observed
// count); entries past a problem's own count are zero.
struct ProbDesc {
    const uint32_t* bits;
    const uint32_t* base;
    int wpr;
    int n1, n2;
    int64_t p;
    const double* lam64;
    const float* lam32;
};

// A problem: grid, packed mask, compact data (immutable after creation and
// shared with views) plus a mutable workspace.  A view shares the immutable
// part and owns a fresh workspace, so requests on one problem can run
// concurrently on different streams.
struct Problem {
    Ctx* ctx = nullptr;
    int n1 = 0, n2 = 0;
    double dx1 = 0, dx2 = 0;
    int N1 = 0, N2 = 0;          // embedding of the masked product
    int64_t p = 0;
    int words_per_row = 0;
    DevBuf bits, base;           // packed mask
    DevBuf cell;                 // compact index -> cell id (int32)
    DevBuf y64, y32;             // compact data
    // covariates of the mean X beta: q compact columns (FP64, q x p), the data
    // with its ordinary least-squares fit removed, yc = y - X beta_ols
    // (FP64, p), and on the host every cell's covariates (q x n1*n2),
    // beta_ols and log det X^T X over the observed cells
    int q = 0;
    DevBuf X64, yc64;
    std::shared_ptr<const std::vector<double>> h_X;
    std::vector<double> beta_ols;
    double logdet_xx = 0;
    // irregularly spaced observations: A as four (cell, weight) slots per
    // observation (cell -1 = unused) and A^T as rows over the grid cells
    // (offsets n + 1, observation ids, weights); cell / h_cell then hold
    // each observation's nearest cell (coloured probes)
    bool irregular = false;
    DevBuf a_cell, a_w, at_off, at_obs, at_w;
    // irregular problems store observations sorted by nearest grid cell (so
    // the mapping's gathers are coherent); compact vectors at the ABI keep
    // the caller's order: obs_user[i] = caller's index of stored observation i
    DevBuf obs_user;
    std::shared_ptr<const std::vector<int32_t>> h_obs_user;
    bool obs_permuted = false;  // false when the caller's order already is the stored order
    std::shared_ptr<const std::vector<int64_t>> h_cell;  // compact index -> cell id (host)
    std::shared_ptr<const std::vector<uint8_t>> h_mask;
    bool is_view = false;
    bool no_graphs = false;  // set on the server's request views (several threads)
    const ProbDesc* tab = nullptr;  // set on a group of problems sharing an embedding
    // workspace (per problem or per view)
    Spectrum spec;               // cache of the last parameter point
    DevBuf Y;                    // transform workspace
    DevBuf lagtmp, spectmp, spec_multi64, spec_multi32;
    DevBuf kws;                  // Krylov workspace
    DevBuf scal;                 // device scalars
    DevBuf tmp1, tmp2, tmp3, tmp4;  // per-call scratch of the drivers
    DevBuf irr;                  // grid vectors of the irregular product
    MaskView mask_view() const {
        return MaskView{bits.as<uint32_t>(), base.as<uint32_t>(), words_per_row};
    }
    Problem view() const {
        Problem v;
        v.ctx = ctx;
        v.n1 = n1;
        v.n2 = n2;
        v.dx1 = dx1;
        v.dx2 = dx2;
        v.N1 = N1;
        v.N2 = N2;
        v.p = p;
        v.words_per_row = words_per_row;
        v.bits = bits;
        v.base = base;
        v.cell = cell;
        v.y64 = y64;
        v.y32 = y32;
        v.irregular = irregular;
        v.a_cell = a_cell;
        v.a_w = a_w;
        v.at_off = at_off;
        v.at_obs = at_obs;
        v.at_w = at_w;
        v.obs_user = obs_user;
        v.h_obs_user = h_obs_user;
        v.obs_permuted = obs_permuted;
        v.q = q;
        v.X64 = X64;
        v.yc64 = yc64;
        v.h_X = h_X;
        v.beta_ols = beta_ols;
        v.logdet_xx = logdet_xx;
        v.h_cell = h_cell;
        v.h_mask = h_mask;
        v.is_view = true;
        return v;
    }
    // exchange workspaces with another problem or view (the immutable part
    // stays), so that one worker's buffers serve views of several problems
    void swap_work(Problem& o) {
        for (auto pr : {std::make_pair(&Y, &o.Y), std::make_pair(&lagtmp, &o.lagtmp),
                        std::make_pair(&spectmp, &o.spectmp), std::make_pair(&spec_multi64, &o.spec_multi64),
                        std::make_pair(&spec_multi32, &o.spec_multi32), std::make_pair(&kws, &o.kws),
                        std::make_pair(&scal, &o.scal), std::make_pair(&tmp1, &o.tmp1), std::make_pair(&tmp2, &o.tmp2),
                        std::make_pair(&tmp3, &o.tmp3), std::make_pair(&tmp4, &o.tmp4), std::make_pair(&irr, &o.irr)})
            std::swap(*pr.first, *pr.second);
        std::swap(spec.s64, o.spec.s64);
        std::swap(spec.s32, o.spec.s32);
        std::swap(spec.theta, o.spec.theta);
        std::swap(spec.valid, o.spec.valid);
        std::swap(spec.lam_min, o.spec.lam_min);
        std::swap(spec.lam_max, o.spec.lam_max);
    }
    void release_work() {
        for (DevBuf* b : {&Y, &lagtmp, &spectmp, &spec_multi64, &spec_multi32, &kws, &scal, &tmp1, &tmp2, &tmp3,
                          &tmp4, &irr, &spec.s64, &spec.s32})
            b->release(*ctx);
        spec.valid = false;
    }
};

// ---- transforms (conv.hip) -------------------------------------------------
enum InMode { IN_COMPACT = 0, IN_DENSE = 1, IN_NOISE = 2 };
enum OutMode { OUT_COMPACT = 0, OUT_GRID = 1 };

// One batched circulant-embedding product on an N1 x N2 torus:
//   rows_in x row_len input block (rows from the top-left corner) ->
//   FFT2 -> multiply by lam (per parameter point) -> inverse FFT2 ->
//   rows_out x cols_out output block.
struct ConvSpec {
    int N1 = 0, N2 = 0;
    int nvec = 0;
    int in_mode = IN_COMPACT;
    const void* in = nullptr;   // compact or dense rows (element type R)
    int64_t in_vstride = 0;
    int in_rstride = 0;         // dense / noise: row stride of the input
    int rows_in = 0, row_len = 0;
    uint64_t seed = 0;
    int stream0 = 0;
    int out_mode = OUT_COMPACT;
    void* out = nullptr;        // element type R
    int64_t out_vstride = 0;
    int rows_out = 0, cols_out = 0;
    const void* vin = nullptr;  // nugget term source (compact, element type R)
    int64_t vin_vstride = 0;
    const double* eta = nullptr;  // per parameter point (device)
    double scale = 1.0;
    const void* lam = nullptr;  // [theta][k2][k1], element type R, scaled
    int64_t lam_tstride = 0;
    int vecs_per_theta = 1;
    // every lam table is even in k1 bit for bit (lam[k2][k1] == lam[k2][N1 - k1],
    // as spectrum_device leaves it for an even covariance): the column stage
    // may then read the lower half only
    bool lam_even = false;
    // FP64, power-of-two N1, one table per vector or shared, no nugget term
    // (eta = 0): partials of the quadratic form x . (K x), formed in the
    // column stage from the spectrum of x, spectral_qf_count(N1, N2) per
    // vector, vector-major; summed in index order they give the form; nullable
    double* pw_out = nullptr;
    // several problems (device table): vector v belongs to tab[(v) / tab_vpp],
    // whose mask, block and spectrum replace the ones above; compact outputs
    // are zero from the problem's count up to out_vstride
    const ProbDesc* tab = nullptr;
    int tab_vpp = 1;
    // per-vector flags (device, nullable): vectors flagged 0 are skipped and
    // their outputs left as they were
    const int* active = nullptr;
    // compact FP64 input only: with upd_r set, the input vector is first
    // replaced, element by element, by upd_r + upd_beta[vector] * input (the
    // conjugate-gradient direction update p = r + beta p, written back to
    // the input; every element is read and written by exactly one thread)
    const void* upd_r = nullptr;
    const double* upd_beta = nullptr;
    // caller-provided workspace for the transform intermediate (nullable):
    // vectors then go through in chunks that fit it, and nothing is allocated
    void* ws = nullptr;
    size_t ws_bytes = 0;
};

// Bytes of the transform intermediate per vector (element type R) of a
// product on an N1 x N2 torus whose input and output blocks have at most
// `rows` rows, as conv_apply lays it out.
template <typename R>
size_t conv_bytes_per_vec(int N1, int N2, int rows, Ctx& c, int nvec);

template <typename R>
void conv_apply(Problem& P, const ConvSpec& s, hipStream_t st);

// Lag grid (N1 x N2 doubles, any sizes >= 1) of the embedding on device;
// with drange the range derivative of the correlation instead.
void lag_grid_device(Ctx& c, int N1, int N2, double dx1, double dx2, const Matern& th, double* d_c,
                     hipStream_t st, bool drange = false);
// Unscaled FP64 half spectrum [k2][k1] of the torus; returns min and max.
// With ws (spectrum_ws_bytes(N1, N2) bytes, device) the lag grid and the
// intermediate go there instead of the problem's workspace, and with
// lam_min == nullptr the min / max (and the wait for them) are skipped.
void spectrum_device(Problem& P, int N1, int N2, const Matern& th, double* d_lam, double* lam_min,
                     double* lam_max, hipStream_t st, bool drange = false, void* ws = nullptr);
size_t spectrum_ws_bytes(int N1, int N2);
// Every per-length twiddle table of the transforms, both precisions (so
// later products allocate none).
void build_plan_tables(Ctx& c);
// Torus sides the transforms support: 16..8192, powers of two or multiples
// of 16 of the form 2^a 3^b 5^c 7^d (mixed-radix plans); and the embedding
// side for a need of m by the rule (kry_ctx_set_embedding; 0 if none).
bool torus_side_ok(int N);
// Quadratic-form partials per vector that the column stage writes with
// ConvSpec::pw_out on an N1 x N2 torus (0: not available for this N1).
int spectral_qf_count(int N1, int N2);
// the covariance is even in each lag separately (its spectrum, as
// spectrum_device leaves it, even in k1 bit for bit)
bool matern_even(const Matern& th);
int embedding_side(int m, int rule = KRY_EMBED_SMALLEST);
// Twiddle tables of the mixed-radix lengths of an embedding N1 x N2 (column
// length N1, row length N2 / 2), built when a problem is created so that its
// products allocate nothing.
void build_embedding_tables(Ctx& c, int N1, int N2);
// Scale a half spectrum by s into FP64 and FP32 copies; optional sqrt of
// max(lam, 0) first (sampling).
void spectrum_scale(const double* lam, int64_t n, double s, bool sqrt_clip, double* out64,
                    float* out32, hipStream_t st);
// Cached, scaled spectrum of theta on the problem's embedding.
Spectrum& problem_spectrum(Problem& P, const Matern& th, hipStream_t st);

// ---- drivers (api.hip), used by the ABI and by the server ----------------------
void loglik_points(Problem& P, const kry_matern* thetas, int count, const kry_opts* o, kry_loglik_result* out,
                   hipStream_t st);
// One parameter point per problem for problems sharing an embedding (CG,
// no shift sharing); `work` is a view whose workspace the call uses.
void loglik_multi(Problem& work, const std::vector<Problem*>& probs, const kry_matern* th, const kry_opts* o,
                  kry_loglik_result* out, hipStream_t st);
// Kriging; sets *noconv when a CG solve stopped at cg_maxit.
void krige_impl(Problem& P, const kry_matern* theta, const kry_opts* opts, const std::vector<int64_t>& targets,
                double* mean_x, double* var_x, double* var_y, int bootstrap_B, bool* noconv, hipStream_t st);
void check_theta(const kry_matern* t);
void check_opts(const kry_opts* o);
int nprobes_of(const kry_opts* o);
// Lanczos steps the workspace must hold: lanczos_steps, or the adaptive cap.
int lanczos_cap(const kry_opts* o);
// One run of Algorithm 1 (k = o->gk_steps, reorthogonalisation per o) on
// the data (or on data64, compact FP64, when given).  V_k and Sigma V_k stay
// in the problem's Krylov workspace until its next use: k full-grid vectors
// each, of the precision's element type.
struct GkRun {
    std::vector<double> alpha, beta, z;  // B_k (alpha_1..k, beta_1..k+1), z_k
    double J = 0, beta1 = 0;
    const void* V = nullptr;
    const void* Sv = nullptr;
    int real_bytes = 8;
};
void gengk_run(Problem& P, const Matern& th, const kry_opts* o, GkRun& G, const double* data64, hipStream_t st);
// GLS estimate of beta at theta (the problem must have covariates); with d_w
// (compact, FP64) also K^{-1} (y - X beta_hat).
std::vector<double> gls_beta(Problem& P, const kry_matern* theta, const kry_opts* o, double* d_w, bool* noconv,
                             hipStream_t st);
Matern to_matern_abi(const kry_matern* t);
// The paper's objective and the low-rank posterior variance (plik.hip).
void plik_device(Problem& P, const kry_matern* theta, const double* beta, const kry_opts* o, kry_plik_result* r,
                 hipStream_t st);
void posterior_variance_device(Problem& P, const kry_matern* theta, const double* beta, const kry_opts* o,
                               double* var_x, double* var_y, double* mean_x, hipStream_t st);
void tridiag_eigen(std::vector<double>& d, std::vector<double> e, std::vector<double>& W);

// ---- Krylov building blocks (krylov.hip) --------------------------------------
int dot_blocks(int64_t n);
template <typename R>
void dot_batched(const R* a, int64_t sa, const R* b, int64_t sb, int64_t n, int nvec, double* partial,
                 double* out, hipStream_t st);

}  // namespace kry

// Opaque handles of the C ABI.
struct kry_ctx {
    kry::Ctx c;
};
struct kry_problem {
    kry::Problem P;
};
