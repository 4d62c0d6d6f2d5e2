// Workgroup-cooperative power-of-two FFTs in LDS (Stockham autosort form).
//
// A workgroup transforms `nfft` independent sequences of length L = 2^log2L
// held in LDS at buf + f * fstride.  Each pass of radix R splits every
// transform into L/R butterflies; with VPT values per thread the workgroup
// must have exactly nfft * L / VPT threads, and each thread owns VPT / R
// butterflies per pass.  Every pass first loads all of a thread's inputs into
// registers, synchronises, then writes the butterfly outputs to their
// autosorted positions, so one LDS buffer suffices (no ping-pong copy).
//
// Pass with current span Ns (product of earlier radices), butterfly j:
//   inputs   x[j + r * L/R],                  r = 0..R-1
//   twiddle  x_r *= W_{Ns R}^{r (j mod Ns)}   (W_n = exp(-2 pi i / n); conj for inverse)
//   outputs  y[(j div Ns) Ns R + (j mod Ns) + r Ns] = DFT_R(x)_r
// Radix-8 passes are used while at least three factors of two remain, then
// one radix-4 or radix-2 pass.  Forward transforms are unnormalised and
// inverse transforms use the conjugate twiddles (also unnormalised).
#pragma once
#include "common.hpp"

namespace kry {

// W_{2^log2n}^e from the table tw[e'] = exp(-2 pi i e' / TW_N).
template <typename R, bool INV>
__device__ __forceinline__ cpx<R> twiddle(const cpx<R>* __restrict__ tw, int e, int log2n) {
    cpx<R> w = tw[(e << (TW_LOG2 - log2n)) & (TW_N - 1)];
    if (INV) w.y = -w.y;
    return w;
}

// multiply by -i (forward) or +i (inverse)
template <typename R, bool INV>
__device__ __forceinline__ cpx<R> rot90(cpx<R> a) {
    return INV ? cpx<R>{-a.y, a.x} : cpx<R>{a.y, -a.x};
}

template <typename R>
__device__ __forceinline__ void bfly2(cpx<R>& a, cpx<R>& b) {
    const cpx<R> t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft2(cpx<R>* v) {
    bfly2(v[0], v[1]);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cpx<R>* v) {
    bfly2(v[0], v[2]);
    bfly2(v[1], v[3]);
    v[3] = rot90<R, INV>(v[3]);
    bfly2(v[0], v[1]);
    bfly2(v[2], v[3]);
    const cpx<R> t = v[1];  // natural order: X0=v0, X1=v2, X2=v1, X3=v3
    v[1] = v[2];
    v[2] = t;
}

template <typename R, bool INV>
__device__ __forceinline__ void dft8(cpx<R>* v) {
    // radix-2 split into even / odd length-4 DFTs
    cpx<R> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<R> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<R, INV>(e);
    dft4<R, INV>(o);
    const R h = (R)0.70710678118654752440084436210484903928;
    // W8^1, W8^2, W8^3 applied to o[1..3]
    const cpx<R> w1 = INV ? cpx<R>{h, h} : cpx<R>{h, -h};
    const cpx<R> w3 = INV ? cpx<R>{-h, h} : cpx<R>{-h, -h};
    o[1] = cmul(o[1], w1);
    o[2] = rot90<R, INV>(o[2]);
    o[3] = cmul(o[3], w3);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = cadd(e[k], o[k]);
        v[k + 4] = csub(e[k], o[k]);
    }
}

template <typename R, int RADIX, bool INV>
__device__ __forceinline__ void dft(cpx<R>* v) {
    if constexpr (RADIX == 8) dft8<R, INV>(v);
    else if constexpr (RADIX == 4) dft4<R, INV>(v);
    else dft2<R, INV>(v);
}

template <int RADIX>
constexpr int ilog2c() { return RADIX == 8 ? 3 : (RADIX == 4 ? 2 : 1); }

template <typename R, int RADIX, bool INV, int VPT>
__device__ __forceinline__ void stockham_pass(cpx<R>* buf, int log2L, int log2Ns, int fstride,
                                              int tid, int nthreads, const cpx<R>* __restrict__ tw) {
    constexpr int BPT = VPT / RADIX;
    constexpr int LR = ilog2c<RADIX>();
    const int log2nb = log2L - LR;  // butterflies per transform = L / RADIX
    const int nbmask = (1 << log2nb) - 1;
    const int nsmask = (1 << log2Ns) - 1;
    cpx<R> v[BPT][RADIX];
    int dst[BPT];
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int g = tid + b * nthreads;
        const int f = g >> log2nb;
        const int j = g & nbmask;
        const int base = f * fstride;
#pragma unroll
        for (int r = 0; r < RADIX; ++r) v[b][r] = buf[base + j + (r << log2nb)];
        const int jn = j & nsmask;
        if (log2Ns > 0) {
#pragma unroll
            for (int r = 1; r < RADIX; ++r) v[b][r] = cmul(v[b][r], twiddle<R, INV>(tw, r * jn, log2Ns + LR));
        }
        dst[b] = base + ((j >> log2Ns) << (log2Ns + LR)) + jn;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        dft<R, RADIX, INV>(v[b]);
#pragma unroll
        for (int r = 0; r < RADIX; ++r) buf[dst[b] + (r << log2Ns)] = v[b][r];
    }
    __syncthreads();
}

// In-place FFT of nfft sequences of length 2^log2L in LDS.  Requires
// blockDim == nfft * 2^log2L / VPT and log2L >= 3.  Caller synchronises
// before (data written) and the function synchronises after the last pass.
template <typename R, bool INV, int VPT>
__device__ void fft_lds(cpx<R>* buf, int log2L, int fstride, int tid, int nthreads,
                        const cpx<R>* __restrict__ tw) {
    int s = 0;
    int rem = log2L;
    while (rem >= 3) {
        stockham_pass<R, 8, INV, VPT>(buf, log2L, s, fstride, tid, nthreads, tw);
        s += 3;
        rem -= 3;
    }
    if (rem == 2) stockham_pass<R, 4, INV, VPT>(buf, log2L, s, fstride, tid, nthreads, tw);
    else if (rem == 1) stockham_pass<R, 2, INV, VPT>(buf, log2L, s, fstride, tid, nthreads, tw);
}

}  // namespace kry
