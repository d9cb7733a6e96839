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
        const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
        const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return Philox4{c0, c1, c2, c3};
}

// Uniforms in (0, 1]: FP32 from the top 24 bits, FP64 from all 32 bits.
__device__ __forceinline__ float u01f(uint32_t r) {
    return (float)((r >> 8) + 1u) * 0x1.0p-24f;
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
