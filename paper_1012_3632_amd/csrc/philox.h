// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11) and Box-Muller normals, device side.
//
// One round maps counter (x0, x1, x2, x3) under key (k0, k1) to
//   (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0))
// and the key is bumped by the Weyl constants between rounds.  The noise of
// the step uses counter (site, step, block | tag << 16, replica) and key
// (seed mod 2^32, seed >> 32); the key and all counter words but the site are
// uniform across a launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
// significant bits (r = 2^32 - 1 gives exactly 1).
__device__ __forceinline__ float u01f(uint32_t r) {
    return __builtin_fmaf((float)r, 0x1.0p-32f, 0x1.0p-32f);
}
__device__ __forceinline__ double u01d(uint32_t r) {
    return ((double)r + 1.0) * 0x1.0p-32;
}

// Box-Muller on two words: (sqrt(-2 ln u0) cos 2 pi u1, sqrt(-2 ln u0) sin 2 pi u1).
// FP32 uses the hardware transcendentals directly: v_log_f32 (log2),
// v_sqrt_f32, and v_sin_f32 / v_cos_f32, which take their argument in
// revolutions (sin(2 pi x)), so u1 needs no range reduction.
__device__ __forceinline__ void box_muller(uint32_t r0, uint32_t r1, float& z0, float& z1) {
    const float u0 = u01f(r0), u1 = u01f(r1);
    constexpr float MINUS_2_LN2 = -1.3862943611198906f;   // -2 ln 2
    const float rad = __builtin_amdgcn_sqrtf(MINUS_2_LN2 * __builtin_amdgcn_logf(u0));
    z0 = rad * __builtin_amdgcn_cosf(u1);
    z1 = rad * __builtin_amdgcn_sinf(u1);
}
__device__ __forceinline__ void box_muller(uint32_t r0, uint32_t r1, double& z0, double& z1) {
    const double u0 = u01d(r0), u1 = u01d(r1);
    const double rad = sqrt(-2.0 * log(u0));
    double s, c;
    sincos(2.0 * 3.141592653589793 * u1, &s, &c);
    z0 = rad * c;
    z1 = rad * s;
}

// The NBLK * 4 normals of one site-step: z[4 b + k] from block b, word pair k/2.
template <int NBLK, typename Real>
__device__ __forceinline__ void site_normals(uint32_t site, uint32_t step, uint32_t tag,
                                             uint32_t replica, uint32_t k0, uint32_t k1,
                                             Real (&z)[4 * NBLK]) {
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
        const Philox4 r = philox4x32_10(site, step, (uint32_t)b | (tag << 16), replica, k0, k1);
        box_muller(r.x, r.y, z[4 * b + 0], z[4 * b + 1]);
        box_muller(r.z, r.w, z[4 * b + 2], z[4 * b + 3]);
    }
}

}  // namespace flb
