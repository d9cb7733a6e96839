// Device helpers shared by the forward and adjoint kernels: periodic pull,
// wavefront and block reductions, tile placement and the LDS-staged
// square-gradient force of a tile.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "collide.h"
#include "step.h"

namespace flb {

// ------------------------------------------------------------------ helpers

// The FP64 noise angle table for a block of NT threads: a copy of
// SINCOS_TABLE in LDS (8 KB, filled here, one barrier), or, for FP32 (which
// does not use it), the global table untouched.  All threads of the block
// must call it.
template <typename Real, int NT>
__device__ __forceinline__ const double2* noise_table() {
    if constexpr (sizeof(Real) == 8) {
        __shared__ double2 lds_tab[512];
        for (int t = threadIdx.x; t < 512; t += NT) lds_tab[t] = SINCOS_TABLE[t];
        __syncthreads();
        return lds_tab;
    } else {
        return SINCOS_TABLE;
    }
}

template <int LAT>
__device__ __forceinline__ uint32_t site_index(int x, int y, int z, const Geom& g) {
    return (uint32_t)((z * g.ny + y) * g.nx + x);
}

// Element idx of a population plane: 32-bit byte offset from the plane base
// (the plane base is uniform, so the access uses the SGPR-base + 32-bit
// VGPR-offset global addressing; a plane is below 4 GiB by construction).
template <typename Real>
__device__ __forceinline__ Real plane_ld(const Real* __restrict__ base, uint32_t idx) {
    return *(const Real*)((const char*)base + idx * (uint32_t)sizeof(Real));
}
template <typename Real>
__device__ __forceinline__ void plane_st(Real* __restrict__ base, uint32_t idx, Real v) {
    *(Real*)((char*)base + idx * (uint32_t)sizeof(Real)) = v;
}
// Same with a non-temporal hint (the next read of this value is a step away).
template <typename Real>
__device__ __forceinline__ void plane_st_nt(Real* __restrict__ base, uint32_t idx, Real v) {
    __builtin_nontemporal_store(v, (Real*)((char*)base + idx * (uint32_t)sizeof(Real)));
}

// f_i(x) = S_i(x - c_i), periodic.
template <int LAT, typename Real>
__device__ __forceinline__ void pull(const Real* __restrict__ fin, int x, int y, int z,
                                     const Geom& g, Real (&f)[Lattice<LAT>::Q]) {
    using L = Lattice<LAT>;
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int sx = L::cx[i] == 0 ? x : (L::cx[i] > 0 ? xm : xp);
        const int sy = L::cy[i] == 0 ? y : (L::cy[i] > 0 ? ym : yp);
        const int sz = L::cz[i] == 0 ? z : (L::cz[i] > 0 ? zm : zp);
        f[i] = plane_ld(fin + (size_t)i * g.V, (uint32_t)((sz * g.ny + sy) * g.nx + sx));
    }
}

// Pull for a wavefront whose lanes share one (y, z) row (y, z uniform, e.g.
// from readfirstlane): the row offset goes into the uniform plane base
// (scalar arithmetic) and each lane only adds its x, x - 1 or x + 1.
template <int LAT, typename Real>
__device__ __forceinline__ void pull_rows(const Real* __restrict__ fin, int x, int y, int z,
                                          const Geom& g, Real (&f)[Lattice<LAT>::Q]) {
    using L = Lattice<LAT>;
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int sx = L::cx[i] == 0 ? x : (L::cx[i] > 0 ? xm : xp);
        const int sy = L::cy[i] == 0 ? y : (L::cy[i] > 0 ? ym : yp);
        const int sz = L::cz[i] == 0 ? z : (L::cz[i] > 0 ? zm : zp);
        const Real* row = fin + ((size_t)i * g.V + (size_t)(uint32_t)((sz * g.ny + sy) * g.nx));
        f[i] = plane_ld(row, (uint32_t)sx);
    }
}

// In-place step pairs (one population buffer).  The first step of a pair
// pulls S_i(x - c_i) from plane i and stores its result S*_i(x) in plane
// opp(i) at x + c_i; the second reads plane opp(i) at x (which then holds
// S*_i(x - c_i), i.e. the streamed population) and stores S**_i(x) in plane i
// at x, the ordinary layout again.  Each location a thread writes is one it
// has itself read, and no other thread touches it, so the update is in place.
template <int LAT, typename Real>
__device__ __forceinline__ void push_rows_opp(Real* f, int x, int y, int z, const Geom& g,
                                              const Real (&v)[Lattice<LAT>::Q]) {
    using L = Lattice<LAT>;
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int dx = L::cx[i] == 0 ? x : (L::cx[i] > 0 ? xp : xm);
        const int dy = L::cy[i] == 0 ? y : (L::cy[i] > 0 ? yp : ym);
        const int dz = L::cz[i] == 0 ? z : (L::cz[i] > 0 ? zp : zm);
        Real* row = f + ((size_t)L::opp[i] * g.V + (size_t)(uint32_t)((dz * g.ny + dy) * g.nx));
        plane_st(row, (uint32_t)dx, v[i]);
    }
}
template <int LAT, typename Real>
__device__ __forceinline__ void load_rows_opp(const Real* f, int x, int y, int z, const Geom& g,
                                              Real (&v)[Lattice<LAT>::Q]) {
    using L = Lattice<LAT>;
    const size_t row = (size_t)(uint32_t)((z * g.ny + y) * g.nx);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) v[i] = plane_ld(f + ((size_t)L::opp[i] * g.V + row), (uint32_t)x);
}
template <int LAT, typename Real>
__device__ __forceinline__ void store_rows(Real* f, int x, int y, int z, const Geom& g,
                                           const Real (&v)[Lattice<LAT>::Q]) {
    using L = Lattice<LAT>;
    const size_t row = (size_t)(uint32_t)((z * g.ny + y) * g.nx);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) plane_st(f + ((size_t)i * g.V + row), (uint32_t)x, v[i]);
}

// A DPP lane move within 16-lane rows (pattern CTRL; a source outside the
// row would read 0, the old operand).
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
}

// One butterfly stage of a 16-lane row reduction of N values per lane: the
// lane pairs given by the DPP pattern CTRL (partners differ in lane bit
// `hi`'s position and hold the same value indices) swap halves of their
// lists, so each lane keeps H = ceil(N/2) partial sums: of its lower half
// (hi = 0) or of its upper half (hi = 1, padded with a zero when N is odd).
// base and len track the original index of the lane's first entry and how
// many of its entries are real.
template <int CTRL, int N, int H, typename Acc>
__device__ __forceinline__ void row_fold(const Acc (&v)[N], Acc (&o)[H], int hi, int& base,
                                         int& len) {
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const Acc lo_v = v[k];
        const Acc hi_v = (k + H < N) ? v[k + H] : Acc(0);
        const Acc keep = hi ? hi_v : lo_v;
        const Acc send = hi ? lo_v : hi_v;
        o[k] = keep + dpp_shift<CTRL>(send);
    }
    if (hi) {
        base += H;
        len = len > H ? len - H : 0;
    } else {
        len = len < H ? len : H;
    }
}

// Block reductions in two phases, in a fixed order.  Phase 1 (rows_to_lds):
// 16-lane row sums of NV values by four DPP butterfly stages (row_ror:8,
// row_half_mirror, quad_perm [2,3,0,1], quad_perm [1,0,3,2]); partners swap
// halves of their lists, so the row's 16 lanes end holding its NV sums
// between them, and every lane stores its sums in FP64 to its row's LDS
// slots; no barrier.  Phase 2 (lds_rows_finish): a barrier, then thread
// k < NV sums the rows and adds (ADD) or stores its value at out[k * stride].
// lds holds 4 * NW * NV doubles (NW wavefronts).  All lanes must be active in
// phase 1 (the DPP reads neighbouring lanes).
template <int NV, typename Acc>
__device__ __forceinline__ void rows_to_lds(Acc (&v)[NV], double* lds) {
    const int lane = threadIdx.x & 63;
    const int row = threadIdx.x >> 4;
    constexpr int H1 = (NV + 1) / 2, H2 = (H1 + 1) / 2, H3 = (H2 + 1) / 2, H4 = (H3 + 1) / 2;
    Acc a1[H1], a2[H2], a3[H3], a4[H4];
    int base = 0, len = NV;
    row_fold<0x128, NV, H1, Acc>(v, a1, (lane >> 3) & 1, base, len);    // row_ror:8
    row_fold<0x141, H1, H2, Acc>(a1, a2, (lane >> 2) & 1, base, len);   // row_half_mirror
    row_fold<0x4E, H2, H3, Acc>(a2, a3, (lane >> 1) & 1, base, len);    // quad_perm 2,3,0,1
    row_fold<0xB1, H3, H4, Acc>(a3, a4, lane & 1, base, len);           // quad_perm 1,0,3,2
#pragma unroll
    for (int p = 0; p < H4; ++p)
        if (p < len) lds[row * NV + base + p] = (double)a4[p];
}
template <int NV, int NT, bool ADD>
__device__ __forceinline__ void lds_rows_finish(const double* lds, double* __restrict__ out,
                                                uint32_t stride) {
    constexpr int NR = 4 * ((NT + 63) / 64);   // 16-lane rows in the block
    __syncthreads();
    if (threadIdx.x < NV) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) acc += lds[r * NV + threadIdx.x];
        if constexpr (ADD) out[(size_t)threadIdx.x * stride] += acc;
        else out[(size_t)threadIdx.x * stride] = acc;
    }
}
// Reduce NV values over the block and add them, in FP64, to slot[0..NV):
// the 16-lane row sums are formed in Acc, the sums over rows, wavefronts and
// steps in FP64.
template <int NV, int NT, typename Acc>
__device__ __forceinline__ void block_accumulate(Acc (&v)[NV], double* __restrict__ slot,
                                                 double* lds) {
    rows_to_lds<NV, Acc>(v, lds);
    lds_rows_finish<NV, NT, true>(lds, slot, 1);
}

template <int LAT, int TX, int TY, int TZ>
__device__ __forceinline__ void tile_origin(const Geom& g, int& x0, int& y0, int& z0) {
    const uint32_t b = xcd_remap(blockIdx.x, g.nblocks);
    const uint32_t bx = b % (uint32_t)g.nbx;
    const uint32_t r = b / (uint32_t)g.nbx;
    const uint32_t by = r % (uint32_t)g.nby;
    const uint32_t bz = r / (uint32_t)g.nby;
    x0 = (int)bx * TX;
    y0 = (int)by * TY;
    z0 = (int)bz * TZ;
}

__device__ __forceinline__ int wrap_any(int v, int n) {
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// ------------------------------------------------------------------ force tile

// Chemical potential mu = psi'(rho) - kappa lap_h rho on the tile plus a
// one-site halo, from the density on the tile plus a two-site halo, both in
// LDS; then F = -rho grad_h mu + eta grad_h(cs2 rho) at a site of the tile.
template <int LAT, typename Real, int TX, int TY, int TZ>
struct ForceTile {
    using L = Lattice<LAT>;
    static constexpr int D = L::D;
    static constexpr int HZ = (LAT == 0) ? 0 : 1;
    static constexpr int RX = TX + 4, RY = TY + 4, RZ = TZ + 4 * HZ;
    static constexpr int MX = TX + 2, MY = TY + 2, MZ = TZ + 2 * HZ;
    static constexpr int NR = RX * RY * RZ, NM = MX * MY * MZ;
    static constexpr int NT = TX * TY * TZ;

    // nthreads: the block's thread count (NT unless a wider tile is staged by
    // a smaller block)
    static __device__ __forceinline__ void stage(const Real* __restrict__ drho, const Geom& g,
                                                 const ForceParams<Real>& fp, int x0, int y0,
                                                 int z0, Real* rs, Real* ms, int nthreads = NT) {
        load_rho(drho, g, x0, y0, z0, rs, nthreads);
        __syncthreads();
        mu_from_rho(fp, rs, ms, nthreads);
    }

    // The density loads of stage alone (no barrier).
    static __device__ __forceinline__ void load_rho(const Real* __restrict__ drho, const Geom& g,
                                                    int x0, int y0, int z0, Real* rs,
                                                    int nthreads) {
        for (int l = threadIdx.x; l < NR; l += nthreads) {
            const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
            const int gx = wrap_any(x0 + lx - 2, g.nx);
            const int gy = wrap_any(y0 + ly - 2, g.ny);
            const int gz = wrap_any(z0 + lz - 2 * HZ, g.nz);
            rs[l] = drho[(uint32_t)((gz * g.ny + gy) * g.nx + gx)];
        }
    }

    // The same, with the density of every staged site formed here from the
    // populations of fin (pulled and summed in the order of k_density, so the
    // staged values are the same bits): no separate density pass.  2-D tiles
    // only.  own: the populations the calling thread pulled for its own site
    // (tx, ty) of the tile, or for that site's periodic image when it lies
    // past a ragged edge; the tile's own sites take their density from them,
    // and only the two-site ring around the tile is pulled here.
    static __device__ __forceinline__ void stage_pop(const Real* __restrict__ fin, const Geom& g,
                                                     const ForceParams<Real>& fp, int x0, int y0,
                                                     int tx, int ty, const Real (&own)[L::Q],
                                                     Real* rs, Real* ms) {
        static_assert(LAT == 0 && TZ == 1, "the ring staging is written for 2-D tiles");
        constexpr int NRING = 4 * RX + 4 * TY;   // rows 0, 1, RY-2, RY-1 and columns 0, 1, RX-2, RX-1
        const int tid = threadIdx.x;
        {
            Real acc = Real(0);
#pragma unroll
            for (int i = 0; i < L::Q; ++i) acc += own[i];
            rs[(ty + 2) * RX + tx + 2] = acc;
        }
        for (int r = tid; r < NRING; r += NT) {
            int lx, ly;
            if (r < 4 * RX) {
                const int k = r / RX;   // 0, 1, 2, 3 -> rows 0, 1, RY - 2, RY - 1
                lx = r - k * RX;
                ly = k < 2 ? k : RY - 4 + k;
            } else {
                const int c = r - 4 * RX;   // 0 .. 4 TY - 1
                const int k = c / TY;       // 0, 1, 2, 3 -> columns 0, 1, RX - 2, RX - 1
                lx = k < 2 ? k : RX - 4 + k;
                ly = 2 + (c - k * TY);
            }
            Real f[L::Q];
            pull<LAT, Real>(fin, wrap_any(x0 + lx - 2, g.nx), wrap_any(y0 + ly - 2, g.ny), 0, g, f);
            Real acc = Real(0);
#pragma unroll
            for (int i = 0; i < L::Q; ++i) acc += f[i];
            rs[ly * RX + lx] = acc;
        }
        __syncthreads();
        mu_from_rho(fp, rs, ms, NT);
    }

    static __device__ __forceinline__ void mu_from_rho(const ForceParams<Real>& fp, const Real* rs,
                                                       Real* ms, int nthreads) {
        mu_rows(fp, rs, ms, nthreads);
        __syncthreads();
    }

    // The chemical potential of mu_from_rho alone (no barrier).
    static __device__ __forceinline__ void mu_rows(const ForceParams<Real>& fp, const Real* rs,
                                                   Real* ms, int nthreads) {
        const int tid = threadIdx.x;
        for (int l = tid; l < NM; l += nthreads) {
            const int mx = l % MX, my = (l / MX) % MY, mz = l / (MX * MY);
            const int c = ((mz + HZ) * RY + (my + 1)) * RX + (mx + 1);
            const Real rc = rs[c];
            Real lap = Real(0);
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const int n = c + (L::cz[i] * RY + L::cy[i]) * RX + L::cx[i];
                lap += Real(L::w[i]) * (rs[n] - rc);
            }
            lap *= Real(6);   // 2 / cs2
            const Real d = rc + fp.shift;
            ms[l] = Real(2) * fp.a * d + Real(4) * fp.b * d * d * d - fp.kappa * lap;
        }
    }

    // Force at tile-local site (lx, ly, lz); also returns delta rho there.
    static __device__ __forceinline__ void force(const Real* rs, const Real* ms,
                                                 const ForceParams<Real>& fp, Real rho0, int lx,
                                                 int ly, int lz, Real (&F)[D]) {
        const int cm = ((lz + HZ) * MY + (ly + 1)) * MX + (lx + 1);
        const int cr = ((lz + 2 * HZ) * RY + (ly + 2)) * RX + (lx + 2);
        Real gm[D], gr[D];
#pragma unroll
        for (int a = 0; a < D; ++a) gm[a] = gr[a] = Real(0);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const Real mu = ms[cm + (L::cz[i] * MY + L::cy[i]) * MX + L::cx[i]];
            const Real rn = rs[cr + (L::cz[i] * RY + L::cy[i]) * RX + L::cx[i]];
            const int c3[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
            for (int a = 0; a < D; ++a) {
                if (c3[a] == 0) continue;
                const Real wc = Real(L::w[i] * c3[a]);
                gm[a] += wc * mu;
                gr[a] += wc * rn;
            }
        }
        const Real rho = rho0 + rs[cr];
#pragma unroll
        for (int a = 0; a < D; ++a) F[a] = -rho * Real(3) * gm[a] + fp.eta * gr[a];
    }
};

// ------------------------------------------------------------------ force march

// The same density -> chemical potential -> force chain for a D3Q19 block
// that sweeps a column of TX x TY sites through a run of z planes.  LDS holds
// a ring of five density planes (TX + 4) x (TY + 4) and three chemical
// potential planes (TX + 2) x (TY + 2): every step in z stages one new density
// plane and evaluates one new mu plane, so the halo is only in x and y.
// Ring slots are numbered relative to the first plane zb of the run.
//
// With a barrier after the density plane is written and one after the mu
// plane, five density slots and three mu slots are enough: at plane z the
// density of z + 2 overwrites that of z - 3, last read by the force at
// z - 2, and mu(z + 1) overwrites mu(z - 2), last read by the force at z - 1;
// both reads precede a barrier that every thread has passed.
template <typename Real, int TX, int TY>
struct ForceMarch {
    using L = Lattice<1>;
    static constexpr int RX = TX + 4, RY = TY + 4, MX = TX + 2, MY = TY + 2;
    static constexpr int NRP = RX * RY, NMP = MX * MY, NT = TX * TY;
    static constexpr int NLD = (NRP + NT - 1) / NT;   // density values staged per thread
    static constexpr int LDS = 5 * NRP + 3 * NMP;

    static __device__ __forceinline__ int rslot(int z, int zb) { return (z - zb + 5) % 5; }
    static __device__ __forceinline__ int mslot(int z, int zb) { return (z - zb + 3) % 3; }

    // in-plane offsets (gy nx + gx) of this thread's staged density values
    static __device__ __forceinline__ void plane_offsets(const Geom& g, int x0, int y0,
                                                         uint32_t (&off)[NLD]) {
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int l = (int)threadIdx.x + k * NT;
            const int lx = l % RX, ly = l / RX;
            const int gx = wrap_any(x0 + lx - 2, g.nx);
            const int gy = wrap_any(y0 + ly - 2, g.ny);
            off[k] = (uint32_t)(gy * g.nx + gx);
        }
    }
    static __device__ __forceinline__ void load_plane(const Real* __restrict__ drho, const Geom& g,
                                                      const uint32_t (&off)[NLD], int z,
                                                      Real (&r)[NLD]) {
        const uint32_t base = (uint32_t)(wrap_any(z, g.nz) * g.ny) * (uint32_t)g.nx;
#pragma unroll
        for (int k = 0; k < NLD; ++k)
            if ((int)threadIdx.x + k * NT < NRP) r[k] = drho[base + off[k]];
    }
    static __device__ __forceinline__ void store_plane(const Real (&r)[NLD], Real* rs) {
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int l = (int)threadIdx.x + k * NT;
            if (l < NRP) rs[l] = r[k];
        }
    }
    // mu on plane z (tile plus a one-site halo in x and y) from density planes z-1, z, z+1
    static __device__ __forceinline__ void mu_plane(const Real* lds_r, Real* lds_m, int z, int zb,
                                                    const ForceParams<Real>& fp) {
        const Real* rp[3] = {lds_r + rslot(z - 1, zb) * NRP, lds_r + rslot(z, zb) * NRP,
                             lds_r + rslot(z + 1, zb) * NRP};
        Real* mo = lds_m + mslot(z, zb) * NMP;
        for (int l = threadIdx.x; l < NMP; l += NT) {
            const int mx = l % MX, my = l / MX;
            const int c = (my + 1) * RX + (mx + 1);
            const Real rc = rp[1][c];
            // (2 / cs2) sum_i w_i (rho(x + c_i) - rho(x)) with the D3Q19
            // weights 1/18 (6 faces) and 1/36 (12 edges):
            // faces / 3 + edges / 6 - 4 rho(x)
            Real faces = Real(0), edges = Real(0);
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const Real r = rp[1 + L::cz[i]][c + L::cy[i] * RX + L::cx[i]];
                if (i <= 6) faces += r;
                else edges += r;
            }
            const Real lap = faces * Real(1.0 / 3) + edges * Real(1.0 / 6) - Real(4) * rc;
            const Real d = rc + fp.shift;
            mo[l] = Real(2) * fp.a * d + Real(4) * fp.b * d * d * d - fp.kappa * lap;
        }
    }
    // force at the tile site (tx, ty) of plane z
    static __device__ __forceinline__ void force(const Real* lds_r, const Real* lds_m, int z, int zb,
                                                 const ForceParams<Real>& fp, Real rho0, int tx,
                                                 int ty, Real (&F)[3]) {
        const Real* rp[3] = {lds_r + rslot(z - 1, zb) * NRP, lds_r + rslot(z, zb) * NRP,
                             lds_r + rslot(z + 1, zb) * NRP};
        const Real* mp[3] = {lds_m + mslot(z - 1, zb) * NMP, lds_m + mslot(z, zb) * NMP,
                             lds_m + mslot(z + 1, zb) * NMP};
        const int cm = (ty + 1) * MX + (tx + 1);
        const int cr = (ty + 2) * RX + (tx + 2);
        Real gm[3] = {Real(0), Real(0), Real(0)};
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const Real mu = mp[1 + L::cz[i]][cm + L::cy[i] * MX + L::cx[i]];
            const int c3[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (c3[a] == 0) continue;
                gm[a] += Real(L::w[i] * c3[a]) * mu;
            }
        }
        const Real rho = rho0 + rp[1][cr];
#pragma unroll
        for (int a = 0; a < 3; ++a) F[a] = -rho * Real(3) * gm[a];
        // eta = 1 adds the density gradient (eta is uniform: a scalar branch)
        if (fp.eta != Real(0)) {
            Real gr[3] = {Real(0), Real(0), Real(0)};
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const Real rn = rp[1 + L::cz[i]][cr + L::cy[i] * RX + L::cx[i]];
                const int c3[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (c3[a] == 0) continue;
                    gr[a] += Real(L::w[i] * c3[a]) * rn;
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) F[a] += fp.eta * gr[a];
        }
    }
};

}  // namespace flb
