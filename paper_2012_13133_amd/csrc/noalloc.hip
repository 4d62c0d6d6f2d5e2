// The masked product for callers that cannot allocate device memory (code
// under stream capture, tight serving loops): the lag grid, spectrum and
// transform intermediate live in one file-scope device array instead of the
// problem's workspace.
//
// The array's host-side name is not a device address: set-up (the context's
// creation) asks the runtime for its address on each device once, with that
// device current, and every use goes through that pointer.
#include <array>
#include <mutex>

#include "internal.hpp"

namespace kry {

namespace {

__device__ __align__(256) unsigned char scratch[KRY_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::array<void*, 64> g_addr{};  // per device

__global__ void k_store_scalar(double* __restrict__ dst, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = v;
}

__global__ void k_scale_half(const double* __restrict__ lam, int64_t n, double s, double* __restrict__ o64,
                             float* __restrict__ o32) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = lam[i] * s;
        if (o64) o64[i] = v;
        if (o32) o32[i] = (float)v;
    }
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

// Address of the scratch array on the current device (`device`), looked up
// once per device.
void* noalloc_scratch_init(int device) {
    KRY_REQUIRE(device >= 0 && device < (int)g_addr.size(), "device index out of range");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_addr[device]) {
        void* ptr = nullptr;
        KRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        KRY_REQUIRE(ptr != nullptr, "scratch array has no device address");
        g_addr[device] = ptr;
    }
    return g_addr[device];
}

// Scratch layout of one call: eta | scaled spectrum (the product's
// precision) | then either the spectrum phase (unscaled FP64 spectrum, lag
// grid, intermediate) or the product's intermediates, which reuse that space.
template <typename R>
static void matvec_noalloc(Problem& P, char* base, const Matern& th, int nvec, const R* in, R* out,
                           hipStream_t st) {
    const int N1 = P.N1, N2 = P.N2;
    const int64_t nspec = (int64_t)(N2 / 2 + 1) * N1;
    const size_t o_lam = 256;
    const size_t o_work = o_lam + align256((size_t)nspec * sizeof(R));
    const size_t spec_phase = (sizeof(R) == 4 ? align256((size_t)nspec * sizeof(double)) : 0) +
                              spectrum_ws_bytes(N1, N2);
    const size_t per_vec = conv_bytes_per_vec<R>(N1, N2, P.n1, *P.ctx, nvec);
    const size_t cap = KRY_NOALLOC_SCRATCH_BYTES;
    if (o_work + spec_phase > cap || o_work + per_vec > cap)
        throw Error(KRY_EINVAL, "a " + std::to_string(N1) + " x " + std::to_string(N2) + " embedding needs " +
                                    std::to_string(o_work + std::max(spec_phase, per_vec)) +
                                    " bytes of scratch, above the " + std::to_string(cap) +
                                    " of the no-allocation product");
    double* d_eta = reinterpret_cast<double*>(base);
    R* lam = reinterpret_cast<R*>(base + o_lam);
    char* work = base + o_work;
    // spectrum: FP64 into lam (FP64) or into the work area first (FP32)
    double* lam64 = sizeof(R) == 8 ? reinterpret_cast<double*>(lam) : reinterpret_cast<double*>(work);
    void* spec_ws = sizeof(R) == 8 ? (void*)work : (void*)(work + align256((size_t)nspec * sizeof(double)));
    spectrum_device(P, N1, N2, th, lam64, nullptr, nullptr, st, false, spec_ws);
    const double s = 1.0 / ((double)N1 * N2);
    int64_t blocks = (nspec + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_scale_half, dim3((unsigned)blocks), dim3(256), 0, st, lam64, nspec, s,
                       sizeof(R) == 8 ? reinterpret_cast<double*>(lam) : nullptr,
                       sizeof(R) == 4 ? reinterpret_cast<float*>(lam) : nullptr);
    KRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_store_scalar, dim3(1), dim3(64), 0, st, d_eta, th.tau2 / th.sigma2);
    KRY_HIP(hipGetLastError());
    ConvSpec c;
    c.N1 = N1;
    c.N2 = N2;
    c.nvec = nvec;
    c.in_mode = IN_COMPACT;
    c.in = in;
    c.in_vstride = P.p;
    c.rows_in = P.n1;
    c.row_len = P.n2;
    c.out_mode = OUT_COMPACT;
    c.out = out;
    c.out_vstride = P.p;
    c.rows_out = P.n1;
    c.cols_out = P.n2;
    c.vin = in;
    c.vin_vstride = P.p;
    c.eta = d_eta;
    c.lam = lam;
    c.lam_tstride = 0;
    c.vecs_per_theta = nvec;
    c.ws = work;
    c.ws_bytes = cap - o_work;
    conv_apply<R>(P, c, st);
}

}  // namespace kry

using namespace kry;

kry_status kry_matvec_device_noalloc(kry_problem* prob, const kry_matern* theta, int32_t precision, int32_t nvec,
                                     const void* d_v, void* d_out, void* hip_stream) {
    return run_guarded([&] {
        KRY_REQUIRE(prob && d_v && d_out, "NULL argument");
        check_theta(theta);
        KRY_REQUIRE(nvec >= 1, "nvec must be >= 1");
        KRY_REQUIRE(precision == KRY_FP64 || precision == KRY_FP32, "bad precision");
        Problem& P = prob->P;
        KRY_REQUIRE(!P.irregular, "the no-allocation product takes masked grid problems only");
        Ctx& C = *P.ctx;
        KRY_REQUIRE(C.scratch != nullptr, "scratch array not set up for this context");
        KRY_HIP(hipSetDevice(C.device));
        hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : C.stream;
        const Matern th{theta->sigma2, theta->tau2, theta->range, theta->nu, theta->aniso_ratio, theta->aniso_angle};
        char* base = static_cast<char*>(C.scratch);
        if (precision == KRY_FP64)
            matvec_noalloc<double>(P, base, th, nvec, static_cast<const double*>(d_v), static_cast<double*>(d_out), st);
        else
            matvec_noalloc<float>(P, base, th, nvec, static_cast<const float*>(d_v), static_cast<float*>(d_out), st);
    });
}
