// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11) and Box-Muller normals, device side.
//
// One round maps counter (x0, x1, x2, x3) under key (k0, k1) to
//   (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0))
// and the key is bumped by the Weyl constants between rounds.  The noise of
// the step uses counter (site, step, block | tag << 16, replica) and key
// (seed mod 2^32, seed >> 32); the key and all counter words but the site are
// uniform across a launch.  Each Box-Muller pair takes a full 32-bit word for
// its radius and 16 bits for its angle, so a D3Q19 site (15 normals) needs
// three Philox blocks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sincos_table.h"

namespace flb {

struct Philox4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply (v_mad_u64_u32) gives both halves of a product
        const uint64_t p0 = (uint64_t)M0 * c0;
        const uint64_t p1 = (uint64_t)M1 * c2;
        // three-input XOR in one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += W0;
        k1 += W1;
    }
    return Philox4{c0, c1, c2, c3};
}

// Uniforms u = (r + 1) 2^-32 in (0, 1].  FP32 evaluates it as
// fma(float(r), 2^-32, 2^-32): exact for r < 2^24, so the small-u tail that sets
// the large Box-Muller radii keeps full 32-bit resolution; larger r round to 24
// significant bits (r = 2^32 - 1 gives exactly 1).  FP64 works from the exact
// r + 1 (neg2_log_u32).
__device__ __forceinline__ float u01f(uint32_t r) {
    return __builtin_fmaf((float)r, 0x1.0p-32f, 0x1.0p-32f);
}

// Box-Muller with a 32-bit radius word r and a 16-bit angle h:
// R = sqrt(-2 ln u), u = (r + 1) 2^-32;  theta = 2 pi v, v = (h + 1) 2^-16;
// (z0, z1) = R (cos theta, sin theta).
// FP32 uses the hardware transcendentals directly: v_log_f32 (log2),
// v_sqrt_f32, and v_sin_f32 / v_cos_f32, which take their argument in
// revolutions (sin(2 pi x)), so v needs no range reduction.
__device__ __forceinline__ void box_muller(uint32_t r, uint32_t h, float& z0, float& z1) {
    const float u = u01f(r);
    const float v = (float)(h + 1u) * 0x1.0p-16f;
    constexpr float MINUS_2_LN2 = -1.3862943611198906f;   // -2 ln 2
    const float rad = __builtin_amdgcn_sqrtf(MINUS_2_LN2 * __builtin_amdgcn_logf(u));
    z0 = rad * __builtin_amdgcn_cosf(v);
    z1 = rad * __builtin_amdgcn_sinf(v);
}
// sin and cos of 2 pi k / 65536 for an integer k in [1, 65536], from the
// angle-sum identity: k = 256 j + l (j taken mod 256), A = 2 pi j / 256,
// B = 2 pi l / 65536, and tab holds the correctly rounded (sin, cos) of A
// (entries 0..255) and of B (entries 256..511); sin(A + B) = sA cB + cA sB,
// cos(A + B) = cA cB - sA sB, each one product and one fused multiply-add
// (within about one unit in the last place).  tab is SINCOS_TABLE or a copy
// of it in LDS; every kernel gets the same bits either way.
__device__ __forceinline__ void sincos_turn16(uint32_t k, const double2* tab, double& s,
                                              double& c) {
    const double2 a = tab[(k >> 8) & 255u];
    const double2 b = tab[256u + (k & 255u)];
    s = fma(a.x, b.y, a.y * b.x);
    c = fma(a.y, b.y, -(a.x * b.x));
}

// -2 ln u for u = (r + 1) 2^-32.  With d = r + 1 = 2^e m (exact; the mantissa
// is moved to m in [sqrt(1/2), sqrt(2))), ln u = (e - 32) ln 2 + ln m and
// ln m = 2 artanh(s), s = (m - 1) / (m + 1), |s| < 0.172, from the series
// 2 (s + s^3/3 + ... + s^21/21) (first omitted term below 1e-18 relative).
// ln 2 is split into a 24-bit head, whose products with e - 32 are exact,
// and the remainder.
__device__ __forceinline__ double neg2_log_u32(uint32_t r) {
    const double d = (double)r + 1.0;
    const long long bits = __double_as_longlong(d);
    int e = (int)(bits >> 52) - 1023;
    double m = __longlong_as_double((bits & 0x000fffffffffffffLL) | 0x3ff0000000000000LL);
    if (m > 1.4142135623730951) {
        m *= 0.5;
        e += 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double two_s = 2.0 * s;
    const double ln_m = fma(two_s * s2, p, two_s);
    constexpr double LN2 = 0.6931471805599453;
    constexpr double LN2_HEAD = (double)(float)LN2;
    constexpr double LN2_TAIL = LN2 - LN2_HEAD;
    const double k = (double)(e - 32);
    return -2.0 * fma(k, LN2_HEAD, fma(k, LN2_TAIL, ln_m));
}

__device__ __forceinline__ void box_muller(uint32_t r, uint32_t h, const double2* tab,
                                           double& z0, double& z1) {
    const double rad = sqrt(neg2_log_u32(r));
    double s, c;
    sincos_turn16(h + 1u, tab, s, c);   // theta = 2 pi (h + 1) 2^-16
    z0 = rad * c;
    z1 = rad * s;
}
__device__ __forceinline__ void box_muller(uint32_t r, uint32_t h, const double2*, float& z0,
                                           float& z1) {
    box_muller(r, h, z0, z1);
}

// The 2 NPAIR normals of one site-step.  Words w[0 ..) are the Philox outputs
// of blocks 0, 1, ... (counter word 2 = block | tag << 16) in order x, y, z, w.
// Pair p takes its radius from word w[p] and its angle from word
// w[NPAIR + p/2] (high 16 bits for even p, low 16 bits for odd p);
// z[2p], z[2p+1] = R (cos, sin).  D3Q19: 8 pairs from 12 words (3 blocks);
// D2Q9: 3 pairs from 5 words (2 blocks).
template <int NPAIR>
struct NoiseLayout {
    static constexpr int NWORD = NPAIR + (NPAIR + 1) / 2;
    static constexpr int NBLK = (NWORD + 3) / 4;
};

// tab: the FP64 angle table (SINCOS_TABLE, or a copy in LDS); FP32 ignores it.
template <int NPAIR, typename Real>
__device__ __forceinline__ void site_normals(uint32_t site, uint32_t step, uint32_t tag,
                                             uint32_t replica, uint32_t k0, uint32_t k1,
                                             Real (&z)[2 * NPAIR],
                                             const double2* tab = SINCOS_TABLE) {
    constexpr int NBLK = NoiseLayout<NPAIR>::NBLK;
    uint32_t w[4 * NBLK];
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
        const Philox4 r = philox4x32_10(site, step, (uint32_t)b | (tag << 16), replica, k0, k1);
        w[4 * b + 0] = r.x;
        w[4 * b + 1] = r.y;
        w[4 * b + 2] = r.z;
        w[4 * b + 3] = r.w;
    }
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) {
        const uint32_t a = w[NPAIR + p / 2];
        const uint32_t h = (p % 2 == 0) ? (a >> 16) : (a & 0xffffu);
        box_muller(w[p], h, tab, z[2 * p], z[2 * p + 1]);
    }
}

}  // namespace flb
