// Device-side single-precision operation sequence for sampling and rollouts.
//
// The rollout contract is bit-exactness for a given counter-based seed, so
// sin/cos/log/tan are not taken from the device math library (whose last-bit
// behaviour is its own) but spelled out here from their textbook
// definitions: Cody-Waite reduction by pi/2 with a three-float split, Taylor
// polynomials on [-pi/4, pi/4], and log via 2 atanh((m-1)/(m+1)).  Every
// +, -, * and / is one IEEE binary32 operation (the library is built with
// -ffp-contract=off and correctly rounded division); every fma is written
// out with __builtin_fmaf; the square root is seq_sqrt below, because the
// compiler lowers the f32 square root to the hardware's 1-ulp instruction.
//
// Philox4x64-10 follows Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3" (SC'11): ten rounds of the 4x64 S-box with the
// published multipliers and Weyl key increments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emppi {

// pi/2 = PIO2_HI + PIO2_MID + PIO2_LO (each the float nearest to what is left)
__device__ constexpr float PIO2_HI = 0x1.921fb6p+0f;
__device__ constexpr float PIO2_MID = -0x1.777a5cp-25f;
__device__ constexpr float PIO2_LO = -0x1.ee59dap-50f;
__device__ constexpr float INV_PIO2 = 0x1.45f306p-1f;  // float nearest 2/pi
__device__ constexpr float TWO_PI = 0x1.921fb6p+2f;    // float nearest 2 pi
// 1/3!, 1/5!, 1/7!, 1/9! with alternating signs (sine) and 1/2! .. 1/10! (cosine)
__device__ constexpr float SIN3 = -0x1.555556p-3f, SIN5 = 0x1.111112p-7f,
                           SIN7 = -0x1.a01a02p-13f, SIN9 = 0x1.71de3ap-19f;
__device__ constexpr float COS2 = -0x1.0p-1f, COS4 = 0x1.555556p-5f, COS6 = -0x1.6c16c2p-10f,
                           COS8 = 0x1.a01a02p-16f, COS10 = -0x1.27e4fcp-22f;
// ln 2 split (16 significant bits + remainder), 1/(2k+1), sqrt 2
__device__ constexpr float LN2_HI = 0x1.62e4p-1f, LN2_LO = 0x1.7f7d1cp-20f;
__device__ constexpr float ATANH3 = 0x1.555556p-2f, ATANH5 = 0x1.99999ap-3f,
                           ATANH7 = 0x1.24924ap-3f, ATANH9 = 0x1.c71c72p-4f;
__device__ constexpr float SQRT2F = 0x1.6a09e6p+0f;

// sin and cos of x: k = rint(x 2/pi), r = x - k pi/2 (three fused steps),
// Horner polynomials in r^2, quadrant rotation by k mod 4.
__device__ __forceinline__ void seq_sincos(float x, float& s_out, float& c_out) {
    const float k = __builtin_rintf(x * INV_PIO2);
    float r = __builtin_fmaf(-k, PIO2_HI, x);
    r = __builtin_fmaf(-k, PIO2_MID, r);
    r = __builtin_fmaf(-k, PIO2_LO, r);
    const float r2 = r * r;
    float ps = __builtin_fmaf(r2, SIN9, SIN7);
    ps = __builtin_fmaf(r2, ps, SIN5);
    ps = __builtin_fmaf(r2, ps, SIN3);
    const float sn = __builtin_fmaf(r * r2, ps, r);
    float pc = __builtin_fmaf(r2, COS10, COS8);
    pc = __builtin_fmaf(r2, pc, COS6);
    pc = __builtin_fmaf(r2, pc, COS4);
    pc = __builtin_fmaf(r2, pc, COS2);
    const float cs = __builtin_fmaf(r2, pc, 1.0f);
    const int q = static_cast<int>(k) & 3;
    const float a = (q & 1) ? cs : sn;     // |sin| or |cos| by quadrant parity
    const float b = (q & 1) ? sn : cs;
    s_out = (q & 2) ? -a : a;
    c_out = ((q + 1) & 2) ? -b : b;
}

// Natural log of a positive normal float: x = m 2^e, m in [sqrt(2)/2, sqrt(2)),
// log x = e ln 2 + 2 atanh(s), s = (m - 1)/(m + 1), series to s^9.
__device__ __forceinline__ float seq_log(float x) {
    const uint32_t bits = __float_as_uint(x);
    int e = static_cast<int>((bits >> 23) & 0xffu) - 127;
    float m = __uint_as_float((bits & 0x7fffffu) | 0x3f800000u);
    if (m > SQRT2F) {
        m = m * 0.5f;
        e += 1;
    }
    const float f = m - 1.0f;
    const float s = f / (m + 1.0f);
    const float z = s * s;
    float p = __builtin_fmaf(z, ATANH9, ATANH7);
    p = __builtin_fmaf(z, p, ATANH5);
    p = __builtin_fmaf(z, p, ATANH3);
    const float a = __builtin_fmaf(s * z, p, s);
    const float lnm = a + a;
    const float fe = static_cast<float>(e);
    return __builtin_fmaf(fe, LN2_HI, __builtin_fmaf(fe, LN2_LO, lnm));
}

// Correctly rounded square root.  v_sqrt_f32 is accurate to 1 ulp, so the
// IEEE result is s or one of its float neighbours s-, s+.  With exact fused
// residuals: x <= s * s-  means sqrt(x) is below the rounding boundary
// between s- and s (the geometric mean of s- and s lies below their midpoint,
// and no float x falls between s * s- and the squared midpoint), so the
// result is s-; x > s * s+ likewise means s+.  Tiny inputs are scaled by 2^32
// (result by 2^-16) so that the hardware instruction never sees a denormal.
__device__ __forceinline__ float seq_sqrt(float x) {
    const bool tiny = x < 0x1.0p-96f;
    const float xs = tiny ? x * 0x1.0p+32f : x;
    const float s = __builtin_amdgcn_sqrtf(xs);
    const float sd = __uint_as_float(__float_as_uint(s) - 1u);
    const float su = __uint_as_float(__float_as_uint(s) + 1u);
    float r = s;
    if (__builtin_fmaf(-sd, s, xs) <= 0.0f) r = sd;
    if (__builtin_fmaf(-su, s, xs) > 0.0f) r = su;
    return tiny ? r * 0x1.0p-16f : r;
}

__device__ __forceinline__ float seq_tan(float x) {
    float s, c;
    seq_sincos(x, s, c);
    return s / c;
}

// ---------------------------------------------------------------- Philox4x64-10
struct U64x4 {
    uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    U64x4 out;
    out.v[0] = c0;
    out.v[1] = c1;
    out.v[2] = c2;
    out.v[3] = c3;
    return out;
}

// Uniform in (0,1): (2 j + 1) 2^-24 from the top 23 bits j of a word (exact).
__device__ __forceinline__ float word_uniform(uint64_t w) {
    const uint32_t j = static_cast<uint32_t>(w >> 41);
    return static_cast<float>(2u * j + 1u) * 0x1.0p-24f;
}

// Four standard normals of (seed, step, rollout r, horizon h, stream): Philox
// counter (h, r, step, stream), key (seed, 0); Box-Muller on word pairs
// (w0, w1) and (w2, w3): sqrt(-2 log u1) * (cos, sin)(2 pi u2).
__device__ __forceinline__ void normals4(uint64_t seed, uint64_t step, uint32_t r, uint32_t h,
                                         uint64_t stream, float z[4]) {
    const U64x4 w = philox4x64_10(h, r, step, stream, seed, 0);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float u1 = word_uniform(w.v[2 * p]);
        const float u2 = word_uniform(w.v[2 * p + 1]);
        const float rad = seq_sqrt(-2.0f * seq_log(u1));
        float s, c;
        seq_sincos(TWO_PI * u2, s, c);
        z[2 * p] = rad * c;
        z[2 * p + 1] = rad * s;
    }
}

}  // namespace emppi
