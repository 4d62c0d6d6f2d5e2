// FFT primitives: twiddle-table access, multiplication by -i / +i and the
// radix-2, -4 and -8 butterflies (unnormalised forward DFTs; the inverse
// ones use conjugate twiddles).  The passes that use them are in fftk.hpp.
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

}  // namespace kry
