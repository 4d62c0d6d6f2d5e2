// Register-resident power-of-two FFT passes with compile-time plans.
//
// A transform of length L = 2^LOG2L is done by T = L/8 threads, each holding
// 8 values between passes.  The forward plan uses radix-8 passes first and
// one radix-4 or radix-2 pass last; the inverse plan is the forward plan
// reversed.  Pass p of radix R and span Ns (product of the earlier radices)
// is the Stockham autosort step
//   inputs   x[j + r L/R]                      r = 0..R-1
//   twiddle  x_r *= W_{Ns R}^{r (j mod Ns)}     (table, conjugate for inverse)
//   outputs  y[(j div Ns) Ns R + (j mod Ns) + r Ns]
// for butterflies j = t + b T, b = 0..8/R-1.  Twiddles come from a per-length
// table holding R entries for every j mod Ns of each pass with Ns > 1, laid
// out so that the lanes of a wavefront, which have consecutive j, read
// consecutive 16-byte pieces: FP64 tables hold entry r of every j mod Ns
// contiguously (index r Ns + j mod Ns); FP32 tables hold the entries in pairs
// (r = 2p, 2p + 1) of every j mod Ns contiguously (index 2 (p Ns + j mod Ns)
// + r mod 2), one 16-byte load per pair.
//
// Because the last forward pass (radix R, Ns = L/R) leaves thread t holding
// positions j + r L/R and the first inverse pass (radix R, Ns = 1) reads the
// same positions, a pointwise multiply between them needs no exchange.
//
// Values exchanged through LDS use a padded index, one unused slot after
// every G elements: G = 16 for complex elements and 8-byte reals, 32 for
// 4-byte reals.  With LDS banks of 4 bytes served 128 bytes per cycle, these
// make the passes' strided writes and contiguous reads conflict-free for
// transforms of 256 points and more (one slot per 8 elements left the
// contiguous 8-byte reads two-way conflicted).
#pragma once
#include "fft.hpp"

namespace kry {

template <typename E>
constexpr int pad_log2() { return sizeof(E) == 4 ? 5 : 4; }
template <typename E>
__device__ __forceinline__ int lpad(int i) { return i + (i >> pad_log2<E>()); }
// lpad(base + d) = lpad(base) + lpad_off(d) when d is a multiple of the group
// or (base mod G) + (d mod G) < G
template <typename E>
constexpr int lpad_off(int d) { return d + (d >> pad_log2<E>()); }
template <typename E>
constexpr int lpadded(int L) { return L + (L >> pad_log2<E>()); }
template <typename E>
constexpr int pad_group() { return 1 << pad_log2<E>(); }

template <int LOG2L>
struct Sched {
    static constexpr int L = 1 << LOG2L;
    static constexpr int n8 = LOG2L / 3;
    static constexpr int rem = LOG2L % 3;
    static constexpr int npass = n8 + (rem ? 1 : 0);
    static constexpr int lr(bool inv, int p) {
        const int q = inv ? npass - 1 - p : p;
        return q < n8 ? 3 : rem;
    }
    static constexpr int lns(bool inv, int p) {
        int s = 0;
        for (int i = 0; i < p; ++i) s += lr(inv, i);
        return s;
    }
    static constexpr int tw_size(bool inv, int p) { return p == 0 ? 0 : (1 << lns(inv, p)) << lr(inv, p); }
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
    static constexpr int tw_total = dir_total(false) + dir_total(true);
};

// DFT-8 whose inputs 4..7 are zero (the zero-padded half of a transform).
template <typename R, bool INV>
__device__ __forceinline__ void dft8_low(cpx<R>* v) {
    const cpx<R> x0 = v[0], x1 = v[1], x2 = v[2], x3 = v[3];
    const cpx<R> e0 = cadd(x0, x2), e2 = csub(x0, x2);
    const cpx<R> e1 = cadd(x0, rot90<R, INV>(x2)), e3 = csub(x0, rot90<R, INV>(x2));
    cpx<R> o0 = cadd(x1, x3), o2 = csub(x1, x3);
    cpx<R> o1 = cadd(x1, rot90<R, INV>(x3)), o3 = csub(x1, rot90<R, INV>(x3));
    const R h = (R)0.70710678118654752440084436210484903928;
    const cpx<R> w1 = INV ? cpx<R>{h, h} : cpx<R>{h, -h};
    const cpx<R> w3 = INV ? cpx<R>{-h, h} : cpx<R>{-h, -h};
    o1 = cmul(o1, w1);
    o2 = rot90<R, INV>(o2);
    o3 = cmul(o3, w3);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

// Twiddles of pass P for thread t (R - 1 per butterfly), loaded ahead of the
// pass so their latency overlaps the LDS exchange and barrier before it.
// Index of entry r of j mod Ns in a pass's twiddle table (see above).
template <typename R>
constexpr int tw_index(int r, int jn, int NS) {
    return sizeof(R) == 8 ? r * NS + jn : 2 * ((r >> 1) * NS + jn) + (r & 1);
}

template <typename R, int LOG2L, bool INV, int P>
struct PassTw {
    static constexpr int RADIX = 1 << Sched<LOG2L>::lr(INV, P);
    static constexpr int BPT = 8 / RADIX;
    cpx<R> w[P > 0 ? BPT * RADIX : 1];
};

template <typename R, int LOG2L, bool INV, int P>
__device__ __forceinline__ PassTw<R, LOG2L, INV, P> pass_twiddles(int t, const cpx<R>* __restrict__ tw) {
    using S = Sched<LOG2L>;
    using PT = PassTw<R, LOG2L, INV, P>;
    constexpr int RADIX = PT::RADIX;
    constexpr int NS = 1 << S::lns(INV, P);
    constexpr int T = S::L / 8;
    PT out;
    if constexpr (P > 0) {
#pragma unroll
        for (int b = 0; b < PT::BPT; ++b) {
            const int jn = (t + b * T) & (NS - 1);
            if constexpr (sizeof(R) == 8) {
                const cpx<R>* wp = tw + S::tw_off(INV, P) + jn;
#pragma unroll
                for (int r = 1; r < RADIX; ++r) out.w[b * RADIX + r] = wp[r * NS];
            } else {
                // pairs as float4 (the pass offsets are even, the table 16-byte aligned)
                const float4* wp = reinterpret_cast<const float4*>(tw + S::tw_off(INV, P)) + jn;
#pragma unroll
                for (int q = 0; q < RADIX / 2; ++q) {
                    const float4 e = wp[q * NS];
                    if (q > 0) out.w[b * RADIX + 2 * q] = cpx<R>{e.x, e.y};
                    out.w[b * RADIX + 2 * q + 1] = cpx<R>{e.z, e.w};
                }
            }
        }
    }
    return out;
}

// Twiddle and butterfly of pass P on V independent sets of 8 register values
// (v[u * 8 + k]) with twiddles already loaded, applied to every set.
template <typename R, int LOG2L, bool INV, int P, bool LOWHALF = false, int V = 1>
__device__ __forceinline__ void pass_compute_tw(cpx<R>* v, const PassTw<R, LOG2L, INV, P>& tw) {
    using PT = PassTw<R, LOG2L, INV, P>;
    constexpr int RADIX = PT::RADIX;
#pragma unroll
    for (int b = 0; b < PT::BPT; ++b) {
        if constexpr (P > 0) {
#pragma unroll
            for (int u = 0; u < V; ++u)
#pragma unroll
                for (int r = 1; r < RADIX; ++r)
                    v[u * 8 + b * RADIX + r] = cmul(v[u * 8 + b * RADIX + r], tw.w[b * RADIX + r]);
        }
#pragma unroll
        for (int u = 0; u < V; ++u) {
            if constexpr (LOWHALF && RADIX == 8) dft8_low<R, INV>(v + u * 8);
            else dft<R, RADIX, INV>(v + u * 8 + b * RADIX);
        }
    }
}

template <typename R, int LOG2L, bool INV, int P, bool LOWHALF = false, int V = 1>
__device__ __forceinline__ void pass_compute(cpx<R>* v, int t, const cpx<R>* __restrict__ tw) {
    pass_compute_tw<R, LOG2L, INV, P, LOWHALF, V>(v, pass_twiddles<R, LOG2L, INV, P>(t, tw));
}


// Inputs of pass P from LDS (transform base `buf`).
template <typename R, int LOG2L, bool INV, int P>
__device__ __forceinline__ void pass_read(cpx<R>* v, const cpx<R>* buf, int t) {
    using S = Sched<LOG2L>;
    constexpr int RADIX = 1 << S::lr(INV, P);
    constexpr int T = S::L / 8;
    constexpr int Q = S::L / RADIX;
    using E = cpx<R>;
#pragma unroll
    for (int b = 0; b < 8 / RADIX; ++b) {
        const int j = t + b * T;
        if constexpr (Q % pad_group<E>() == 0) {
            const cpx<R>* p = buf + lpad<E>(j);
#pragma unroll
            for (int r = 0; r < RADIX; ++r) v[b * RADIX + r] = p[lpad_off<E>(r * Q)];
        } else {
#pragma unroll
            for (int r = 0; r < RADIX; ++r) v[b * RADIX + r] = buf[lpad<E>(j + r * Q)];
        }
    }
}

// Outputs of pass P to their autosorted LDS positions.
template <typename R, int LOG2L, bool INV, int P>
__device__ __forceinline__ void pass_write(const cpx<R>* v, cpx<R>* buf, int t) {
    using S = Sched<LOG2L>;
    constexpr int LR = S::lr(INV, P);
    constexpr int RADIX = 1 << LR;
    constexpr int LNS = S::lns(INV, P);
    constexpr int NS = 1 << LNS;
    constexpr int T = S::L / 8;
    using E = cpx<R>;
    constexpr int G = pad_group<E>();
    // dst mod G = j mod NS when NS divides G and NS * RADIX is a multiple of G
    constexpr bool FAST = (NS % G == 0) || (G % NS == 0 && (NS * RADIX) % G == 0);
#pragma unroll
    for (int b = 0; b < 8 / RADIX; ++b) {
        const int j = t + b * T;
        const int dst = ((j >> LNS) << (LNS + LR)) + (j & (NS - 1));
        if constexpr (FAST) {
            cpx<R>* p = buf + lpad<E>(dst);
#pragma unroll
            for (int r = 0; r < RADIX; ++r) p[lpad_off<E>(r * NS)] = v[b * RADIX + r];
        } else {
#pragma unroll
            for (int r = 0; r < RADIX; ++r) buf[lpad<E>(dst + r * NS)] = v[b * RADIX + r];
        }
    }
}

// ---- split exchange: real parts, then imaginary parts, through a buffer of
// reals (lpadded<R>(L) per transform at least).  A workgroup then needs half the LDS of a
// complex exchange, so more workgroups fit a CU, at four barriers per
// exchange instead of two.  Index logic as in pass_read / pass_write.
template <typename R, int C>
__device__ __forceinline__ R& part(cpx<R>& z) {
    if constexpr (C == 0) return z.x;
    else return z.y;
}

template <typename R, int LOG2L, bool INV, int P, int C>
__device__ __forceinline__ void pass_read_part(cpx<R>* v, const R* buf, int t) {
    using S = Sched<LOG2L>;
    constexpr int RADIX = 1 << S::lr(INV, P);
    constexpr int T = S::L / 8;
    constexpr int Q = S::L / RADIX;
#pragma unroll
    for (int b = 0; b < 8 / RADIX; ++b) {
        const int j = t + b * T;
        if constexpr (Q % pad_group<R>() == 0) {
            const R* p = buf + lpad<R>(j);
#pragma unroll
            for (int r = 0; r < RADIX; ++r) part<R, C>(v[b * RADIX + r]) = p[lpad_off<R>(r * Q)];
        } else {
#pragma unroll
            for (int r = 0; r < RADIX; ++r) part<R, C>(v[b * RADIX + r]) = buf[lpad<R>(j + r * Q)];
        }
    }
}

template <typename R, int LOG2L, bool INV, int P, int C>
__device__ __forceinline__ void pass_write_part(cpx<R>* v, R* buf, int t) {
    using S = Sched<LOG2L>;
    constexpr int LR = S::lr(INV, P);
    constexpr int RADIX = 1 << LR;
    constexpr int LNS = S::lns(INV, P);
    constexpr int NS = 1 << LNS;
    constexpr int T = S::L / 8;
    constexpr int G = pad_group<R>();
    constexpr bool FAST = (NS % G == 0) || (G % NS == 0 && (NS * RADIX) % G == 0);
#pragma unroll
    for (int b = 0; b < 8 / RADIX; ++b) {
        const int j = t + b * T;
        const int dst = ((j >> LNS) << (LNS + LR)) + (j & (NS - 1));
        if constexpr (FAST) {
            R* p = buf + lpad<R>(dst);
#pragma unroll
            for (int r = 0; r < RADIX; ++r) p[lpad_off<R>(r * NS)] = part<R, C>(v[b * RADIX + r]);
        } else {
#pragma unroll
            for (int r = 0; r < RADIX; ++r) buf[lpad<R>(dst + r * NS)] = part<R, C>(v[b * RADIX + r]);
        }
    }
}

// Exchange from the outputs of pass PW to the inputs of pass PW + 1 for V
// transforms at buf + u * stride (reals).  Starts with a barrier, so the
// previous exchange's readers are done before the buffer is overwritten.
template <typename R, int LOG2L, bool INV, int PW, int V>
__device__ __forceinline__ void exchange_split(cpx<R>* v, R* buf, int stride, int t) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < V; ++u) pass_write_part<R, LOG2L, INV, PW, 0>(v + u * 8, buf + u * stride, t);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < V; ++u) pass_read_part<R, LOG2L, INV, PW + 1, 0>(v + u * 8, buf + u * stride, t);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < V; ++u) pass_write_part<R, LOG2L, INV, PW, 1>(v + u * 8, buf + u * stride, t);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < V; ++u) pass_read_part<R, LOG2L, INV, PW + 1, 1>(v + u * 8, buf + u * stride, t);
}

// Passes P..PE of a plan after pass P - 1 was computed in registers: for
// each, its twiddles are fetched, the values exchanged (split) and the pass
// computed.
template <typename R, int LOG2L, bool INV, int P, int PE, int V>
struct SplitPasses {
    __device__ __forceinline__ static void run(cpx<R>* v, R* buf, int stride, int t, const cpx<R>* __restrict__ tw) {
        if constexpr (P <= PE) {
            const auto w = pass_twiddles<R, LOG2L, INV, P>(t, tw);
            exchange_split<R, LOG2L, INV, P - 1, V>(v, buf, stride, t);
            pass_compute_tw<R, LOG2L, INV, P, false, V>(v, w);
            SplitPasses<R, LOG2L, INV, P + 1, PE, V>::run(v, buf, stride, t, tw);
        }
    }
};

// Natural-order position of register value k after the last pass (or before
// the first pass) of a plan whose boundary radix is 2^LR.
template <int LOG2L, int LR>
__device__ __forceinline__ int edge_pos(int t, int k) {
    constexpr int RADIX = 1 << LR;
    constexpr int T = (1 << LOG2L) / 8;
    constexpr int Q = (1 << LOG2L) / RADIX;
    return t + (k / RADIX) * T + (k % RADIX) * Q;
}

// Passes P..PE-1 entirely through LDS (read, sync, compute, write, sync) for V
// transforms at buf + u * stride.
template <typename R, int LOG2L, bool INV, int P, int PE, int V = 1>
struct LdsPasses {
    __device__ __forceinline__ static void run(cpx<R>* v, cpx<R>* buf, int stride, int t,
                                               const cpx<R>* __restrict__ tw) {
        if constexpr (P < PE) {
            const auto w = pass_twiddles<R, LOG2L, INV, P>(t, tw);
#pragma unroll
            for (int u = 0; u < V; ++u) pass_read<R, LOG2L, INV, P>(v + u * 8, buf + u * stride, t);
            __syncthreads();
            pass_compute_tw<R, LOG2L, INV, P, false, V>(v, w);
#pragma unroll
            for (int u = 0; u < V; ++u) pass_write<R, LOG2L, INV, P>(v + u * 8, buf + u * stride, t);
            __syncthreads();
            LdsPasses<R, LOG2L, INV, P + 1, PE, V>::run(v, buf, stride, t, tw);
        }
    }
};

// Ordering point for LDS exchanges among the lanes of one wavefront: a
// wavefront's LDS instructions are performed in program order, so fences that
// stop the compiler (and the memory model) from moving accesses across this
// point are enough; no workgroup barrier is needed.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
    if constexpr (WAVE) wave_sync();
    else __syncthreads();
}

// Passes P..PE-1 through LDS for one transform at buf handled by TR = T / VT
// threads, thread t acting for the virtual threads t + u TR, u < VT (values
// v[u * 8 + k]).  WAVE: the transform's threads lie in one wavefront, so the
// exchanges need wave_sync only.
template <typename R, int LOG2L, bool INV, int P, int PE, int VT, bool WAVE>
struct LdsPassesVT {
    __device__ __forceinline__ static void run(cpx<R>* v, cpx<R>* buf, int t, const cpx<R>* __restrict__ tw) {
        if constexpr (P < PE) {
            constexpr int TR = (1 << LOG2L) / 8 / VT;
            PassTw<R, LOG2L, INV, P> w[VT];
#pragma unroll
            for (int u = 0; u < VT; ++u) w[u] = pass_twiddles<R, LOG2L, INV, P>(t + u * TR, tw);
#pragma unroll
            for (int u = 0; u < VT; ++u) pass_read<R, LOG2L, INV, P>(v + u * 8, buf, t + u * TR);
            lds_sync<WAVE>();
#pragma unroll
            for (int u = 0; u < VT; ++u) pass_compute_tw<R, LOG2L, INV, P>(v + u * 8, w[u]);
#pragma unroll
            for (int u = 0; u < VT; ++u) pass_write<R, LOG2L, INV, P>(v + u * 8, buf, t + u * TR);
            lds_sync<WAVE>();
            LdsPassesVT<R, LOG2L, INV, P + 1, PE, VT, WAVE>::run(v, buf, t, tw);
        }
    }
};

// Split exchange for one transform handled by TR = T / VT threads (thread t
// acting for the virtual threads t + u TR), as LdsPassesVT: real parts, then
// imaginary parts, through a buffer of reals (padded L).
template <typename R, int LOG2L, bool INV, int PW, int VT, bool WAVE>
__device__ __forceinline__ void exchange_split_vt(cpx<R>* v, R* buf, int t) {
    constexpr int TR = (1 << LOG2L) / 8 / VT;
    lds_sync<WAVE>();
#pragma unroll
    for (int u = 0; u < VT; ++u) pass_write_part<R, LOG2L, INV, PW, 0>(v + u * 8, buf, t + u * TR);
    lds_sync<WAVE>();
#pragma unroll
    for (int u = 0; u < VT; ++u) pass_read_part<R, LOG2L, INV, PW + 1, 0>(v + u * 8, buf, t + u * TR);
    lds_sync<WAVE>();
#pragma unroll
    for (int u = 0; u < VT; ++u) pass_write_part<R, LOG2L, INV, PW, 1>(v + u * 8, buf, t + u * TR);
    lds_sync<WAVE>();
#pragma unroll
    for (int u = 0; u < VT; ++u) pass_read_part<R, LOG2L, INV, PW + 1, 1>(v + u * 8, buf, t + u * TR);
}

// Passes P..PE after pass P - 1 was computed in registers, with split
// exchanges between them (one transform, VT virtual threads per thread).
template <typename R, int LOG2L, bool INV, int P, int PE, int VT, bool WAVE>
struct SplitPassesVT {
    __device__ __forceinline__ static void run(cpx<R>* v, R* buf, int t, const cpx<R>* __restrict__ tw) {
        if constexpr (P <= PE) {
            constexpr int TR = (1 << LOG2L) / 8 / VT;
            PassTw<R, LOG2L, INV, P> w[VT];
#pragma unroll
            for (int u = 0; u < VT; ++u) w[u] = pass_twiddles<R, LOG2L, INV, P>(t + u * TR, tw);
            exchange_split_vt<R, LOG2L, INV, P - 1, VT, WAVE>(v, buf, t);
#pragma unroll
            for (int u = 0; u < VT; ++u) pass_compute_tw<R, LOG2L, INV, P>(v + u * 8, w[u]);
            SplitPassesVT<R, LOG2L, INV, P + 1, PE, VT, WAVE>::run(v, buf, t, tw);
        }
    }
};

}  // namespace kry
