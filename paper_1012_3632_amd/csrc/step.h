// Forward kernels of the fluctuating LB step: initial state, density after
// streaming, the fused pull + collide (+ force) step with optional FP64
// statistics, hydrodynamic fields, raw noise words and the statistics
// finalization.  Shared declarations for the host side live in internal.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "collide.h"

namespace flb {

// Box and launch geometry, uniform over a launch.
struct Geom {
    int32_t nx, ny, nz;
    int32_t nbx, nby, nbz;   // tiles per direction
    uint32_t nblocks;        // nbx * nby * nbz
    uint32_t V;              // sites
    int32_t zc;              // z-marching launches: planes per block (else 0)
};

// Non-ideal force parameters (Landau psi and square-gradient kappa).
template <typename Real>
struct ForceParams {
    Real a, b, shift;   // shift = rho0 - rho_c, so rho - rho_c = delta rho + shift
    Real kappa;
    Real eta;
};

// Step index: read from device memory when captured in a graph.
struct StepIndex {
    const unsigned long long* dev;   // nullable
    unsigned long long host;
    __device__ __forceinline__ uint32_t get() const {
        return (uint32_t)((dev ? *dev : 0ull) + host);
    }
};

// XCD-aware block order: the hardware deals consecutive workgroups round-robin
// over the 8 XCDs; renumber so that each XCD walks a contiguous slab of tiles
// and neighbouring tiles share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nblocks) {
    constexpr uint32_t NX = 8;
    const uint32_t per = nblocks / NX;
    const uint32_t full = per * NX;
    if (b >= full) return b;
    return (b % NX) * per + b / NX;
}

}  // namespace flb
