// Register-resident mixed-radix FFT passes for the embeddings that are not
// powers of two: lengths L = 2^a 3^b 5^c 7^d with a >= 3, L / 8 threads per
// transform.  Two forms share the plan and the twiddle tables: compile-time
// plans (MSched, the mpass_* steps) for the lengths with one odd factor,
// 3 2^a, 5 2^a and 7 2^a, whose kernels are instantiated per length; and
// run-time plans (MPlan, the mr_* steps) for every other such length.
//
// A transform of length L is done by T = L/8 threads.  The forward plan is
// radix 8 (all of them first; the first pass is always radix 8, so the
// zero-padded half of an input and the natural positions t + k T of the
// first pass's inputs and the last inverse pass's outputs are those of the
// power-of-two plans), then the radix-3, radix-5 and radix-7 passes, then the
// remaining radix 2 or 4; the inverse plan is the forward plan reversed.
// Pass p of radix R and span Ns (product of the earlier radices) is the
// Stockham autosort step of fftk.hpp:
//   inputs   x[j + r L/R]                      r = 0..R-1
//   twiddle  x_r *= W_{Ns R}^{r (j mod Ns)}
//   outputs  y[(j div Ns) Ns R + (j mod Ns) + r Ns]
// for butterflies j = t + b T, b < ceil(8/R); a thread's butterfly b takes
// part only when j < L/R (radix 3: three butterflies for two thirds of the
// threads, two for the rest; radix 5 and 7: two for three fifths and one
// seventh of them), so every pass goes through LDS.  A run-time plan
// (radices, spans, twiddle offsets) sits in device memory ahead of the
// length's twiddle table; a pass's radix selects one of six compiled pass
// bodies, whose register layout is fixed at compile time.
// Twiddles come from a per-length table laid out [r][j mod Ns] per pass and
// direction (the inverse direction holds its own, conjugate, entries),
// followed by W_{2L}^k, k = 0..L, for the real-to-complex split of a row
// transform.
#pragma once
#include "fftk.hpp"

namespace kry {

// values a thread holds in one pass: ceil(8 / R) R for R in {2, 3, 4, 5, 7, 8}
constexpr int MVMAX = 14;
// passes of a plan (8 * 3^6 = 5832 takes seven)
constexpr int MPMAX = 12;

struct MPlan {
    int L = 0, T = 0, npass = 0;
    int radix[MPMAX] = {};           // forward order
    int ns_f[MPMAX] = {}, ns_i[MPMAX] = {};  // spans, forward and inverse order
    int tw_f[MPMAX] = {}, tw_i[MPMAX] = {};  // twiddle table offsets of the passes
    // ceil(2^32 / span) (0 for span 1): j div span = umulhi(j, magic) for
    // j, span < 2^13, since j (magic span - 2^32) < 2^26 < 2^32
    unsigned magic_f[MPMAX] = {}, magic_i[MPMAX] = {};
    int split_off = 0, tw_total = 0;
    __host__ __device__ int radix_at(bool inv, int p) const { return radix[inv ? npass - 1 - p : p]; }
};

// The plan of length L, or false when L is not 2^a 3^b 5^c 7^d with a >= 3
// (or needs more than MPMAX passes).
inline bool mplan_make(int L, MPlan* out) {
    if (L < 8) return false;
    int x = L, a = 0, n3 = 0, n5 = 0, n7 = 0;
    while (x % 2 == 0) x /= 2, ++a;
    while (x % 3 == 0) x /= 3, ++n3;
    while (x % 5 == 0) x /= 5, ++n5;
    while (x % 7 == 0) x /= 7, ++n7;
    if (x != 1 || a < 3) return false;
    MPlan p;
    p.L = L;
    p.T = L / 8;
    const int e8 = a / 3, rem = a % 3;
    auto push = [&](int r, int k) {
        for (int i = 0; i < k; ++i) p.radix[p.npass++] = r;
    };
    if (e8 + n3 + n5 + n7 + (rem ? 1 : 0) > MPMAX) return false;
    push(8, e8);
    push(3, n3);
    push(5, n5);
    push(7, n7);
    if (rem) push(1 << rem, 1);
    int off = 0;
    for (int inv = 0; inv < 2; ++inv) {
        int ns = 1;
        for (int q = 0; q < p.npass; ++q) {
            const int r = p.radix_at(inv, q);
            (inv ? p.ns_i : p.ns_f)[q] = ns;
            (inv ? p.magic_i : p.magic_f)[q] =
                ns > 1 ? (unsigned)(((1ull << 32) + (unsigned long long)ns - 1) / (unsigned long long)ns) : 0u;
            (inv ? p.tw_i : p.tw_f)[q] = off;
            if (q > 0) off += ns * r;  // the first pass of each direction has no twiddles
            ns *= r;
        }
    }
    p.split_off = off;
    p.tw_total = off + L + 1;
    *out = p;
    return true;
}

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

// DFT-7 by its symmetric pairs: with t_m = x_m + x_{7-m}, u_m = x_m - x_{7-m}
// (m = 1, 2, 3), c_m = cos(2 pi m / 7), s_m = sin(2 pi m / 7):
//   X_k = x_0 + sum_m cos(2 pi k m / 7) t_m  -/+  i sum_m sin(2 pi k m / 7) u_m,
//   X_{7-k} the same with the sign of the sine part flipped (k = 1, 2, 3).
template <typename R, bool INV>
__device__ __forceinline__ void dft7(cpx<R>* v) {
    const R c1 = (R)0.6234898018587335305250048840042398106322;
    const R c2 = (R)-0.222520933956314404288902564496794759466;
    const R c3 = (R)-0.900968867902419126236102319507445051165;
    const R s1 = (R)0.7818314824680298087084445266740577502323;
    const R s2 = (R)0.9749279121818236070181316829939312172327;
    const R s3 = (R)0.4338837391175581204757683328483587546099;
    const cpx<R> x0 = v[0];
    const cpx<R> t1 = cadd(v[1], v[6]), t2 = cadd(v[2], v[5]), t3 = cadd(v[3], v[4]);
    const cpx<R> u1 = csub(v[1], v[6]), u2 = csub(v[2], v[5]), u3 = csub(v[3], v[4]);
    const cpx<R> a1{x0.x + c1 * t1.x + c2 * t2.x + c3 * t3.x, x0.y + c1 * t1.y + c2 * t2.y + c3 * t3.y};
    const cpx<R> a2{x0.x + c2 * t1.x + c3 * t2.x + c1 * t3.x, x0.y + c2 * t1.y + c3 * t2.y + c1 * t3.y};
    const cpx<R> a3{x0.x + c3 * t1.x + c1 * t2.x + c2 * t3.x, x0.y + c3 * t1.y + c1 * t2.y + c2 * t3.y};
    const cpx<R> b1 = rot90<R, INV>(
        cpx<R>{s1 * u1.x + s2 * u2.x + s3 * u3.x, s1 * u1.y + s2 * u2.y + s3 * u3.y});
    const cpx<R> b2 = rot90<R, INV>(
        cpx<R>{s2 * u1.x - s3 * u2.x - s1 * u3.x, s2 * u1.y - s3 * u2.y - s1 * u3.y});
    const cpx<R> b3 = rot90<R, INV>(
        cpx<R>{s3 * u1.x - s1 * u2.x + s2 * u3.x, s3 * u1.y - s1 * u2.y + s2 * u3.y});
    v[0] = cadd(x0, cadd(t1, cadd(t2, t3)));
    v[1] = cadd(a1, b1);
    v[6] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[5] = csub(a2, b2);
    v[3] = cadd(a3, b3);
    v[4] = csub(a3, b3);
}

template <typename R, int RADIX, bool INV>
__device__ __forceinline__ void dftm(cpx<R>* v) {
    if constexpr (RADIX == 3) dft3<R, INV>(v);
    else if constexpr (RADIX == 5) dft5<R, INV>(v);
    else if constexpr (RADIX == 7) dft7<R, INV>(v);
    else dft<R, RADIX, INV>(v);
}

// ---- compile-time plans ------------------------------------------------
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
    static constexpr int A = count(2), N3 = count(3), N5 = count(5), N7 = count(7);
    static constexpr int E8 = A / 3, REM = A % 3;
    static constexpr int npass = E8 + N3 + N5 + N7 + (REM ? 1 : 0);
    static constexpr int T = L / 8;
    static constexpr int fwd_radix(int q) {
        return q < E8                  ? 8
               : q < E8 + N3           ? 3
               : q < E8 + N3 + N5      ? 5
               : q < E8 + N3 + N5 + N7 ? 7
                                       : (1 << REM);
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
        while (x % 7 == 0) x /= 7;
        return x == 1 && A >= 3;
    }
    static_assert(valid(), "mixed-radix lengths are 2^a 3^b 5^c 7^d with a >= 3");
};

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

// ---- run-time plans -----------------------------------------------------
template <int RADIX>
constexpr int mbpt() { return (8 + RADIX - 1) / RADIX; }

template <typename R, int RADIX>
struct MTw {
    cpx<R> w[mbpt<RADIX>() * RADIX];
};

// Twiddles of a pass of span NS > 1 for thread t, from the pass's table
// `tw` (loaded ahead of the pass's exchange); butterflies that take no part
// read entry 0.
__device__ __forceinline__ int mr_div(int j, unsigned magic) { return (int)__umulhi((unsigned)j, magic); }

template <typename R, int RADIX>
__device__ __forceinline__ MTw<R, RADIX> mr_twiddles(int t, int T, int L, int NS, unsigned magic,
                                                     const cpx<R>* __restrict__ tw) {
    MTw<R, RADIX> out;
    const int Q = L / RADIX;
#pragma unroll
    for (int b = 0; b < mbpt<RADIX>(); ++b) {
        const int j = t + b * T;
        const int jn = j < Q ? j - mr_div(j, magic) * NS : 0;
        const cpx<R>* wp = tw + jn;
#pragma unroll
        for (int r = 1; r < RADIX; ++r) out.w[b * RADIX + r] = wp[r * NS];
    }
    return out;
}

// Butterflies of every slot of a pass (slots that take no part are never
// stored).  LOWHALF: a radix-8 first pass whose inputs 4..7 are zero.
template <typename R, int RADIX, bool INV, bool LOWHALF = false>
__device__ __forceinline__ void mr_butterflies(cpx<R>* v) {
#pragma unroll
    for (int b = 0; b < mbpt<RADIX>(); ++b) {
        if constexpr (LOWHALF && RADIX == 8) dft8_low<R, INV>(v + b * RADIX);
        else dftm<R, RADIX, INV>(v + b * RADIX);
    }
}

// Twiddles, then butterflies (every pass but the first of a direction).
template <typename R, int RADIX, bool INV>
__device__ __forceinline__ void mr_compute(cpx<R>* v, const MTw<R, RADIX>& tw) {
#pragma unroll
    for (int b = 0; b < mbpt<RADIX>(); ++b)
#pragma unroll
        for (int r = 1; r < RADIX; ++r) v[b * RADIX + r] = cmul(v[b * RADIX + r], tw.w[b * RADIX + r]);
    mr_butterflies<R, RADIX, INV>(v);
}

template <typename R, int RADIX>
__device__ __forceinline__ void mr_read(cpx<R>* v, const cpx<R>* buf, int t, int T, int L) {
    using E = cpx<R>;
    const int Q = L / RADIX;
#pragma unroll
    for (int b = 0; b < mbpt<RADIX>(); ++b) {
        const int j = t + b * T;
        if (j < Q) {
#pragma unroll
            for (int r = 0; r < RADIX; ++r) v[b * RADIX + r] = buf[lpad<E>(j + r * Q)];
        }
    }
}

// (NS = 1: the first pass of a direction, magic unused)
template <typename R, int RADIX>
__device__ __forceinline__ void mr_write(const cpx<R>* v, cpx<R>* buf, int t, int T, int L, int NS,
                                         unsigned magic = 0u) {
    using E = cpx<R>;
    const int Q = L / RADIX;
#pragma unroll
    for (int b = 0; b < mbpt<RADIX>(); ++b) {
        const int j = t + b * T;
        if (j < Q) {
            const int jq = NS == 1 ? j : mr_div(j, magic);
            const int dst = jq * NS * RADIX + (j - jq * NS);
#pragma unroll
            for (int r = 0; r < RADIX; ++r) buf[lpad<E>(dst + r * NS)] = v[b * RADIX + r];
        }
    }
}

// One pass (not the first of its direction: NS > 1) of radix RADIX entirely
// through LDS (read, barrier, compute, write, barrier) for V transforms at
// buf + u * stride (values v[u * MVMAX + k]).
template <typename R, int RADIX, bool INV, int V>
__device__ __forceinline__ void mr_lds_pass(cpx<R>* v, cpx<R>* buf, int stride, int t, int T, int L, int NS,
                                            unsigned magic, const cpx<R>* __restrict__ tw) {
    const MTw<R, RADIX> w = mr_twiddles<R, RADIX>(t, T, L, NS, magic, tw);
#pragma unroll
    for (int u = 0; u < V; ++u) mr_read<R, RADIX>(v + u * MVMAX, buf + u * stride, t, T, L);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < V; ++u) {
        mr_compute<R, RADIX, INV>(v + u * MVMAX, w);
        mr_write<R, RADIX>(v + u * MVMAX, buf + u * stride, t, T, L, NS, magic);
    }
    __syncthreads();
}

// Passes P0..PE-1 (P0 >= 1) of the plan through LDS, each by the body of its
// radix (the radix is the same for every thread of the workgroup).  The plan
// is read from device memory: indexed by the pass, a plan passed by value
// would be copied to private memory.
template <typename R, bool INV, int V = 1>
__device__ __forceinline__ void mr_lds_passes(const MPlan* __restrict__ pl, int P0, int PE, cpx<R>* v,
                                              cpx<R>* buf, int stride, int t, const cpx<R>* __restrict__ twp) {
    for (int p = P0; p < PE; ++p) {
        // T and L pass through an empty asm statement each iteration, so the
        // compiler does not hoist the six bodies' address arithmetic (which
        // depends only on t, T and L) out of the loop and keep it all live
        int T = pl->T, L = pl->L;
        asm volatile("" : "+s"(T), "+s"(L));
        const int NS = INV ? pl->ns_i[p] : pl->ns_f[p];
        const unsigned mg = INV ? pl->magic_i[p] : pl->magic_f[p];
        const cpx<R>* tw = twp + (INV ? pl->tw_i[p] : pl->tw_f[p]);
        switch (pl->radix_at(INV, p)) {
            case 8: mr_lds_pass<R, 8, INV, V>(v, buf, stride, t, T, L, NS, mg, tw); break;
            case 7: mr_lds_pass<R, 7, INV, V>(v, buf, stride, t, T, L, NS, mg, tw); break;
            case 5: mr_lds_pass<R, 5, INV, V>(v, buf, stride, t, T, L, NS, mg, tw); break;
            case 4: mr_lds_pass<R, 4, INV, V>(v, buf, stride, t, T, L, NS, mg, tw); break;
            case 3: mr_lds_pass<R, 3, INV, V>(v, buf, stride, t, T, L, NS, mg, tw); break;
            default: mr_lds_pass<R, 2, INV, V>(v, buf, stride, t, T, L, NS, mg, tw); break;
        }
    }
}

}  // namespace kry
