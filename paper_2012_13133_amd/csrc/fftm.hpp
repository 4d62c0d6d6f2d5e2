// Register-resident mixed-radix FFT passes (lengths L = 2^a 3^b 5^c, a >= 3)
// with compile-time plans, for embeddings that are not powers of two.
//
// A transform of length L is done by T = L/8 threads.  The forward plan is
// radix 8 (all of them first; the first pass is always radix 8, so the
// zero-padded half of an input and the natural positions t + k T of the
// first pass's inputs and the last inverse pass's outputs are those of the
// power-of-two plans), then the radix-3 and radix-5 passes, then the
// remaining radix 2 or 4; the inverse plan is the forward plan reversed.
// Pass p of radix R and span Ns (product of the earlier radices) is the
// Stockham autosort step of fftk.hpp:
//   inputs   x[j + r L/R]                      r = 0..R-1
//   twiddle  x_r *= W_{Ns R}^{r (j mod Ns)}
//   outputs  y[(j div Ns) Ns R + (j mod Ns) + r Ns]
// for butterflies j = t + b T, b < ceil(8/R); a thread's butterfly b takes
// part only when j < L/R (radix 3: three butterflies for two thirds of the
// threads, two for the rest; radix 5: two for three fifths of them), so
// every pass goes through LDS.  Twiddles come from a per-length table laid
// out [r][j mod Ns] per pass and direction (the inverse direction holds its
// own, conjugate, entries), followed by W_{2L}^k, k = 0..L, for the
// real-to-complex split of a row transform.
#pragma once
#include "fftk.hpp"

namespace kry {

template <int L>
struct MSched {
    static constexpr int count(int p) {
        int c = 0, x = L;
        while (x % p == 0) {
            x /= p;
            ++c;
        }
        return c;
    }
    static constexpr int A = count(2), N3 = count(3), N5 = count(5);
    static constexpr int E8 = A / 3, REM = A % 3;
    static constexpr int npass = E8 + N3 + N5 + (REM ? 1 : 0);
    static constexpr int T = L / 8;
    static constexpr int fwd_radix(int q) {
        return q < E8 ? 8 : q < E8 + N3 ? 3 : q < E8 + N3 + N5 ? 5 : (1 << REM);
    }
    static constexpr int radix(bool inv, int p) { return fwd_radix(inv ? npass - 1 - p : p); }
    static constexpr int ns(bool inv, int p) {
        int s = 1;
        for (int i = 0; i < p; ++i) s *= radix(inv, i);
        return s;
    }
    static constexpr int bpt(bool inv, int p) { return (8 + radix(inv, p) - 1) / radix(inv, p); }
    static constexpr int tw_size(bool inv, int p) { return p == 0 ? 0 : ns(inv, p) * radix(inv, p); }
    static constexpr int dir_total(bool inv) {
        int o = 0;
        for (int i = 0; i < npass; ++i) o += tw_size(inv, i);
        return o;
    }
    static constexpr int tw_off(bool inv, int p) {
        int o = inv ? dir_total(false) : 0;
        for (int i = 0; i < p; ++i) o += tw_size(inv, i);
        return o;
    }
    static constexpr int split_off = dir_total(false) + dir_total(true);
    static constexpr int tw_total = split_off + L + 1;
    static constexpr bool valid() {
        int x = L;
        while (x % 2 == 0) x /= 2;
        while (x % 3 == 0) x /= 3;
        while (x % 5 == 0) x /= 5;
        return x == 1 && A >= 3;
    }
    static_assert(valid(), "mixed-radix lengths are 2^a 3^b 5^c with a >= 3");
};

// values a thread holds in one pass: ceil(8 / R) R for R in {2, 3, 4, 5, 8}
constexpr int MVMAX = 10;

template <typename R, bool INV>
__device__ __forceinline__ void dft3(cpx<R>* v) {
    const R h = (R)0.5, k = (R)0.86602540378443864676372317075293618347;  // sin(pi / 3)
    const cpx<R> a = v[0], s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const cpx<R> m{a.x - h * s.x, a.y - h * s.y};
    const cpx<R> q = rot90<R, INV>(cpx<R>{k * d.x, k * d.y});  // -i k d forward, +i k d inverse
    v[0] = cadd(a, s);
    v[1] = cadd(m, q);
    v[2] = csub(m, q);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft5(cpx<R>* v) {
    const R c1 = (R)0.30901699437494742410229341718281905886;   // cos(2 pi / 5)
    const R c2 = (R)-0.80901699437494742410229341718281905886;  // cos(4 pi / 5)
    const R s1 = (R)0.95105651629515357211643933337938214340;   // sin(2 pi / 5)
    const R s2 = (R)0.58778525229247312916870595463907276860;   // sin(4 pi / 5)
    const cpx<R> x0 = v[0];
    const cpx<R> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const cpx<R> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const cpx<R> a1{x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y};
    const cpx<R> a2{x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y};
    const cpx<R> b1 = rot90<R, INV>(cpx<R>{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
    const cpx<R> b2 = rot90<R, INV>(cpx<R>{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
    v[0] = cadd(x0, cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
}

template <typename R, int RADIX, bool INV>
__device__ __forceinline__ void dftm(cpx<R>* v) {
    if constexpr (RADIX == 3) dft3<R, INV>(v);
    else if constexpr (RADIX == 5) dft5<R, INV>(v);
    else dft<R, RADIX, INV>(v);
}

template <typename R, int L, bool INV, int P>
struct MPassTw {
    using S = MSched<L>;
    static constexpr int RADIX = S::radix(INV, P);
    static constexpr int BPT = S::bpt(INV, P);
    cpx<R> w[P > 0 ? BPT * RADIX : 1];
};

// Twiddles of pass P for thread t (loaded ahead of the pass's exchange);
// butterflies that take no part read entry 0.
template <typename R, int L, bool INV, int P>
__device__ __forceinline__ MPassTw<R, L, INV, P> mpass_twiddles(int t, const cpx<R>* __restrict__ tw) {
    using S = MSched<L>;
    using PT = MPassTw<R, L, INV, P>;
    constexpr int RADIX = PT::RADIX, NS = S::ns(INV, P), T = S::T, Q = L / RADIX;
    PT out;
    if constexpr (P > 0) {
#pragma unroll
        for (int b = 0; b < PT::BPT; ++b) {
            const int j = t + b * T;
            const int jn = j < Q ? j % NS : 0;
            const cpx<R>* wp = tw + S::tw_off(INV, P) + jn;
#pragma unroll
            for (int r = 1; r < RADIX; ++r) out.w[b * RADIX + r] = wp[r * NS];
        }
    }
    return out;
}

// Twiddle and butterfly of pass P (every butterfly slot is computed; those
// that take no part are never stored).  LOWHALF: a radix-8 first pass whose
// inputs 4..7 are zero.
template <typename R, int L, bool INV, int P, bool LOWHALF = false>
__device__ __forceinline__ void mpass_compute_tw(cpx<R>* v, const MPassTw<R, L, INV, P>& tw) {
    using PT = MPassTw<R, L, INV, P>;
    constexpr int RADIX = PT::RADIX;
#pragma unroll
    for (int b = 0; b < PT::BPT; ++b) {
        if constexpr (P > 0) {
#pragma unroll
            for (int r = 1; r < RADIX; ++r) v[b * RADIX + r] = cmul(v[b * RADIX + r], tw.w[b * RADIX + r]);
        }
        if constexpr (LOWHALF && RADIX == 8) dft8_low<R, INV>(v + b * RADIX);
        else dftm<R, RADIX, INV>(v + b * RADIX);
    }
}

template <typename R, int L, bool INV, int P>
__device__ __forceinline__ void mpass_read(cpx<R>* v, const cpx<R>* buf, int t) {
    using S = MSched<L>;
    constexpr int RADIX = S::radix(INV, P), T = S::T, Q = L / RADIX;
    using E = cpx<R>;
#pragma unroll
    for (int b = 0; b < S::bpt(INV, P); ++b) {
        const int j = t + b * T;
        if (j < Q) {
#pragma unroll
            for (int r = 0; r < RADIX; ++r) v[b * RADIX + r] = buf[lpad<E>(j + r * Q)];
        }
    }
}

template <typename R, int L, bool INV, int P>
__device__ __forceinline__ void mpass_write(const cpx<R>* v, cpx<R>* buf, int t) {
    using S = MSched<L>;
    constexpr int RADIX = S::radix(INV, P), NS = S::ns(INV, P), T = S::T, Q = L / RADIX;
    using E = cpx<R>;
#pragma unroll
    for (int b = 0; b < S::bpt(INV, P); ++b) {
        const int j = t + b * T;
        if (j < Q) {
            const int dst = (j / NS) * NS * RADIX + j % NS;
#pragma unroll
            for (int r = 0; r < RADIX; ++r) buf[lpad<E>(dst + r * NS)] = v[b * RADIX + r];
        }
    }
}

// Passes P..PE-1 entirely through LDS (read, barrier, compute, write,
// barrier) for V transforms at buf + u * stride (values v[u * MVMAX + k]).
template <typename R, int L, bool INV, int P, int PE, int V = 1>
struct MLdsPasses {
    __device__ __forceinline__ static void run(cpx<R>* v, cpx<R>* buf, int stride, int t,
                                               const cpx<R>* __restrict__ tw) {
        if constexpr (P < PE) {
            const auto w = mpass_twiddles<R, L, INV, P>(t, tw);
#pragma unroll
            for (int u = 0; u < V; ++u) mpass_read<R, L, INV, P>(v + u * MVMAX, buf + u * stride, t);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < V; ++u) {
                mpass_compute_tw<R, L, INV, P>(v + u * MVMAX, w);
                mpass_write<R, L, INV, P>(v + u * MVMAX, buf + u * stride, t);
            }
            __syncthreads();
            MLdsPasses<R, L, INV, P + 1, PE, V>::run(v, buf, stride, t, tw);
        }
    }
};

}  // namespace kry
