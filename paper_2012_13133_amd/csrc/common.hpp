// Shared device-side definitions: complex arithmetic, the packed observation
// mask and the Philox4x32-10 generator.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace kry {

constexpr int TW_LOG2 = 13;  // twiddle table exp(-2 pi i e / 8192) covers lengths up to 8192
constexpr int TW_N = 1 << TW_LOG2;

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
// Complex product with explicit fused multiply-adds.  The library is built
// with implicit contraction off, so every vector sees the same rounding
// whichever unrolled copy or batch slot computes it.
__device__ __forceinline__ float fma_rn(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_rn(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Element i of an array addressed by a 32-bit byte offset from its base, so
// that a base shared by the workgroup stays in scalar registers and each lane
// adds only its offset.  Callers guarantee i * sizeof(T) < 2^32.
template <typename T>
__device__ __forceinline__ T& at32(T* base, uint32_t i) {
    using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return *reinterpret_cast<T*>(reinterpret_cast<C*>(base) + i * (uint32_t)sizeof(T));
}
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {fma_rn(a.x, b.x, -(a.y * b.y)), fma_rn(a.x, b.y, a.y * b.x)};
}
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }

// Packed observation mask of an n1 x n2 grid.  Row i occupies words_per_row
// 32-bit words; bit b of word w is cell (i, 32 w + b).  base[w] is the number
// of observed cells in all earlier words (row-major), so the compact index of
// an observed cell is base[w] + popcount of the lower bits of its word.
struct MaskView {
    const uint32_t* bits;
    const uint32_t* base;
    int words_per_row;
};

__device__ __forceinline__ bool mask_lookup(const MaskView& m, int i, int j, int64_t& cidx) {
    const int w = i * m.words_per_row + (j >> 5);
    const uint32_t word = m.bits[w];
    const uint32_t bit = 1u << (j & 31);
    cidx = (int64_t)m.base[w] + __popc(word & (bit - 1u));
    return (word & bit) != 0u;
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) -------------------
struct u32x4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 ctr, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = M0 * ctr.a, hi0 = __umulhi(M0, ctr.a);
        const uint32_t lo1 = M1 * ctr.c, hi1 = __umulhi(M1, ctr.c);
        ctr = {hi1 ^ ctr.b ^ k0, lo1, hi0 ^ ctr.d ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return ctr;
}

enum : uint32_t { DOMAIN_PROBE = 1, DOMAIN_FIELD = 2, DOMAIN_NOISE = 3, DOMAIN_TARGET = 4 };

// Rademacher sign for (index, probe): bit 0 of the first output word.
__device__ __forceinline__ double rademacher(uint32_t index, uint32_t probe, uint64_t seed) {
    u32x4 o = philox4x32_10({index, probe, DOMAIN_PROBE, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
    return (o.a & 1u) ? -1.0 : 1.0;
}

// Standard normal for (index, stream, domain) by Box-Muller on two 53-bit
// uniforms built from the four output words.
__device__ __forceinline__ double philox_normal(uint32_t index, uint32_t stream, uint32_t domain,
                                                uint64_t seed) {
    u32x4 o = philox4x32_10({index, stream, domain, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double two26 = 67108864.0, inv53 = 1.0 / 9007199254740992.0;
    const double u1 = ((double)(o.a >> 5) * two26 + (double)(o.b >> 6) + 0.5) * inv53;
    const double u2 = ((double)(o.c >> 5) * two26 + (double)(o.d >> 6)) * inv53;
    return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// Workgroups go to the chip's 8 XCDs round-robin by linear id.  This maps a
// workgroup's linear id to a logical id such that each XCD receives one
// contiguous range of logical ids, so neighbouring tiles (which share cache
// lines or read the same spectrum) meet in the same L2.  A bijection on
// [0, nblocks).
__device__ __forceinline__ int xcd_remap(int lid, int nblocks) {
    constexpr int NX = 8;
    const int xcd = lid % NX, slot = lid / NX;
    const int q = nblocks / NX, r = nblocks % NX;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

}  // namespace kry
