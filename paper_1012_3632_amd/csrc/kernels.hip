// Forward kernels of the fluctuating LB step for gfx950 and their launchers.
//
// Layout: shifted populations delta f in structure-of-arrays order
// f[i * V + site], site = x + nx (y + ny z).  A launch covers the box with
// tiles of TX x TY x TZ sites, one site per thread, so that a wavefront reads
// 64 (or more) consecutive x-sites of every population plane: every load and
// store of the pull step is a coalesced row segment (the +-x neighbours are
// the same segment shifted by one element).  The order of tiles is remapped so
// that each XCD walks a contiguous slab of the box (shared L2 for the y/z
// neighbour rows).
//
// Force model: the density after streaming is produced by k_density; the
// step kernel stages a tile of it with a two-site halo in LDS, evaluates the
// chemical potential on the tile plus a one-site halo in LDS, and forms the
// force at each site from those (no extra HBM pass for mu).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "internal.h"

namespace flb {

// ------------------------------------------------------------------ kernels

template <int LAT, typename Real>
__global__ void k_init(Real* __restrict__ f, const double* __restrict__ drho, uint32_t V) {
    using L = Lattice<LAT>;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const double d = drho ? drho[s] : 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) f[(size_t)i * V + s] = (Real)(L::w[i] * d);
}

// delta rho(x) = sum_i delta S_i(x - c_i)
template <int LAT, typename Real>
__global__ void k_density(const Real* __restrict__ fin, Real* __restrict__ out, Geom g) {
    using L = Lattice<LAT>;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const int x = (int)(s % (uint32_t)g.nx);
    const uint32_t r = s / (uint32_t)g.nx;
    const int y = (int)(r % (uint32_t)g.ny), z = (int)(r / (uint32_t)g.ny);
    Real f[L::Q];
    pull<LAT, Real>(fin, x, y, z, g, f);
    Real acc = Real(0);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) acc += f[i];
    out[s] = acc;
}

// The collision and store of one site of k_step from its pulled populations
// f; FIRST: the first site this thread adds to its statistics, which then
// take its moments directly (no zeroed accumulators).
template <int LAT, typename Real, bool FORCE, bool STATS, bool ROWS, bool NTS, bool FIRST>
__device__ __forceinline__ void step_site(Real (&f)[Lattice<LAT>::Q], Real* __restrict__ fout,
                                          int x, int y, int z, const Geom& g,
                                          const CollideParams<Real>& P,
                                          const Real (&F)[Lattice<LAT>::D], uint32_t step,
                                          const double2* tab, Real* v) {
    using L = Lattice<LAT>;
    using M = Moments<LAT, Real>;
    constexpr int Q = L::Q;
    Real m[Q];
    M::forward(f, m);
    if constexpr (STATS) {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            if constexpr (FIRST) {
                v[a] = m[a];
                v[Q + a] = m[a] * m[a];
            } else {
                v[a] += m[a];
                v[Q + a] += m[a] * m[a];
            }
        }
    }
    const uint32_t site = site_index<LAT>(x, y, z, g);
    Real zn[2 * L::NPAIR];
    if (P.noise_on)
        site_normals<L::NPAIR, Real>(site, step, 0u, P.replica, P.key0, P.key1, zn, tab);
    collide_moments<LAT, Real, FORCE>(m, F, zn, P);
    M::inverse(m, f);
    if constexpr (ROWS) {
        const size_t row = (size_t)(uint32_t)((z * g.ny + y) * g.nx);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if constexpr (NTS) plane_st_nt(fout + ((size_t)i * g.V + row), (uint32_t)x, f[i]);
            else plane_st(fout + ((size_t)i * g.V + row), (uint32_t)x, f[i]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) plane_st(fout + (size_t)i * g.V, site, f[i]);
    }
}

template <int LAT, typename Real, bool FORCE, bool STATS, int TX, int TY, int TZ, int SPT,
          bool NTS, bool FUSED = false>
__global__ __launch_bounds__(TX* TY* TZ) void k_step(
    const Real* __restrict__ fin, Real* __restrict__ fout, const Real* __restrict__ drho, Geom g,
    CollideParams<Real> P, ForceParams<Real> fp, StepIndex st, double* __restrict__ partial,
    Real* __restrict__ rho_out) {
    using L = Lattice<LAT>;
    using M = Moments<LAT, Real>;
    using FT = ForceTile<LAT, Real, TX, TY, TZ>;
    constexpr int Q = L::Q, D = L::D, NT = TX * TY * TZ;
    constexpr int LDS_F = FORCE ? (FT::NR + FT::NM) : 1;
    constexpr int LDS_S = STATS ? 4 * ((NT + 63) / 64) * 2 * Q : 1;
    __shared__ Real lds_force[LDS_F];
    __shared__ double lds_stats[LDS_S];

    static_assert(!FORCE || SPT == 1, "the force tile covers one site per thread");
    const double2* tab = SINCOS_TABLE;
    if constexpr (!FORCE) tab = noise_table<Real, NT>();
    // with TX a multiple of 64 every wavefront lies in one (y, z) row
    constexpr bool ROWS = (TX % 64) == 0;
    int x0, y0, z0;
    tile_origin<LAT, TX, TY * SPT, TZ>(g, x0, y0, z0);
    const int tx = threadIdx.x % TX;
    int ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    if constexpr (ROWS) {
        ty = __builtin_amdgcn_readfirstlane(ty);
        tz = __builtin_amdgcn_readfirstlane(tz);
    }
    const int x = x0 + tx, z = z0 + tz;

    Real F[D], fpre[FORCE ? Q : 1];
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] = Real(0);
    if constexpr (FORCE) {
        // the populations are pulled before the density tile is staged, so
        // that the two sets of loads are in flight together
        const bool in0 = x < g.nx && y0 + ty < g.ny && z < g.nz;
        if constexpr (FUSED) {
            // every thread pulls its site (a periodic image past a ragged
            // edge): the staged density of the tile's own sites comes from it
            if (in0 && ROWS) pull_rows<LAT, Real>(fin, x, y0 + ty, z, g, fpre);
            else pull<LAT, Real>(fin, wrap_any(x, g.nx), wrap_any(y0 + ty, g.ny), z, g, fpre);
            FT::stage_pop(fin, g, fp, x0, y0, tx, ty, fpre, lds_force, lds_force + FT::NR);
            // the density of fin at this site, as the density pass would
            // write it (the same sum in the same order), when asked for
            if (rho_out && in0) {
                Real acc = Real(0);
#pragma unroll
                for (int i = 0; i < Q; ++i) acc += fpre[i];
                rho_out[site_index<LAT>(x, y0 + ty, z, g)] = acc;
            }
        } else {
            if (in0) {
                if constexpr (ROWS) pull_rows<LAT, Real>(fin, x, y0 + ty, z, g, fpre);
                else pull<LAT, Real>(fin, x, y0 + ty, z, g, fpre);
            }
            FT::stage(drho, g, fp, x0, y0, z0, lds_force, lds_force + FT::NR);
        }
        if (in0) FT::force(lds_force, lds_force + FT::NR, fp, P.rho0, tx, ty, tz, F);
    }

    // pulled populations of one site (the force path has them already)
    auto pull_site = [&](int y, Real (&f)[Q]) {
        if constexpr (FORCE) {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = fpre[i];
        } else if constexpr (ROWS) {
            pull_rows<LAT, Real>(fin, x, y, z, g, f);
        } else {
            pull<LAT, Real>(fin, x, y, z, g, f);
        }
    };
    const uint32_t step = st.get();
    Real v[2 * Q];
    if (x0 + TX <= g.nx && y0 + TY * SPT <= g.ny && z0 + TZ <= g.nz) {
        // the tile lies inside the lattice (uniform): no per-lane checks
        {
            Real f[Q];
            pull_site(y0 + ty, f);
            step_site<LAT, Real, FORCE, STATS, ROWS, NTS, true>(f, fout, x, y0 + ty, z, g, P, F,
                                                                step, tab, v);
        }
#pragma unroll
        for (int sp = 1; sp < SPT; ++sp) {
            Real f[Q];
            pull_site(y0 + ty + sp * TY, f);
            step_site<LAT, Real, FORCE, STATS, ROWS, NTS, false>(f, fout, x, y0 + ty + sp * TY, z,
                                                                 g, P, F, step, tab, v);
        }
    } else {
        if constexpr (STATS) {
#pragma unroll
            for (int k = 0; k < 2 * Q; ++k) v[k] = Real(0);
        }
#pragma unroll
        for (int sp = 0; sp < SPT; ++sp) {
            const int y = y0 + ty + sp * TY;
            if (x < g.nx && y < g.ny && z < g.nz) {
                Real f[Q];
                pull_site(y, f);
                step_site<LAT, Real, FORCE, STATS, ROWS, NTS, false>(f, fout, x, y, z, g, P, F,
                                                                     step, tab, v);
            }
        }
    }
    if constexpr (STATS) {
        const uint32_t b = xcd_remap(blockIdx.x, g.nblocks);
        block_accumulate<2 * Q, NT>(v, partial + (size_t)b * 2 * Q, lds_stats);
    }
}

// One step of an in-place pair (ideal gas), phase PH = 0 (pull, push to the
// opposite plane at x + c_i) or 1 (local read of the opposite plane, store in
// the ordinary layout); see push_rows_opp.  Tiles of TX x (TY SPT) sites, TX a
// multiple of 64, SPT sites per thread stacked in y as in k_step; the
// collision, noise counters and statistics are those of k_step, so a pair
// gives bit-identical populations to two ordinary steps.  With one buffer
// instead of two the working set of a lattice is halved, which lets a 128^3
// FP32 D3Q19 state stay in the 256 MB last-level cache.
// The update of one site of an in-place pair; FIRST: the site is the first
// this thread adds to its statistics, which take its moments directly (no
// zeroed accumulators to merge with lanes that skip a site).
template <int LAT, typename Real, bool STATS, int PH, bool FIRST>
__device__ __forceinline__ void ip_site(Real* f, int x, int y, int z, const Geom& g,
                                        const CollideParams<Real>& P, uint32_t step,
                                        const double2* tab, Real* v) {
    using L = Lattice<LAT>;
    using M = Moments<LAT, Real>;
    constexpr int Q = L::Q, D = L::D;
    Real fl[Q], m[Q];
    if constexpr (PH == 0) pull_rows<LAT, Real>(f, x, y, z, g, fl);
    else load_rows_opp<LAT, Real>(f, x, y, z, g, fl);
    M::forward(fl, m);
    if constexpr (STATS) {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            if constexpr (FIRST) {
                v[a] = m[a];
                v[Q + a] = m[a] * m[a];
            } else {
                v[a] += m[a];
                v[Q + a] += m[a] * m[a];
            }
        }
    }
    const uint32_t site = site_index<LAT>(x, y, z, g);
    Real zn[2 * L::NPAIR];
    if (P.noise_on) site_normals<L::NPAIR, Real>(site, step, 0u, P.replica, P.key0, P.key1, zn, tab);
    const Real F[D] = {};
    collide_moments<LAT, Real, false>(m, F, zn, P);
    M::inverse(m, fl);
    // x is re-read here so that the store addresses are formed late
    // (not held in registers through the collision)
    int xs = x;
    asm volatile("" : "+v"(xs));
    if constexpr (PH == 0) push_rows_opp<LAT, Real>(f, xs, y, z, g, fl);
    else store_rows<LAT, Real>(f, xs, y, z, g, fl);
}

// One step of an in-place pair (ideal gas), phase PH = 0 (pull, push to the
// opposite plane at x + c_i) or 1 (local read of the opposite plane, store in
// the ordinary layout); see push_rows_opp.  Tiles of TX x (TY SPT) sites, TX a
// multiple of 64, SPT sites per thread stacked in y as in k_step; the
// collision, noise counters and statistics are those of k_step, so a pair
// gives bit-identical populations to two ordinary steps.  With one buffer
// instead of two the working set of a lattice is halved, which lets a 128^3
// FP32 D3Q19 state stay in the 256 MB last-level cache.  A tile inside the
// lattice (the test is uniform over the block) takes a path with no per-lane
// range checks.
template <int LAT, typename Real, bool STATS, int PH, int TX, int TY, int SPT = 1>
__global__ __launch_bounds__(TX* TY) void k_step_ip(Real* f, Geom g, CollideParams<Real> P,
                                                     StepIndex st, double* __restrict__ partial) {
    using L = Lattice<LAT>;
    constexpr int Q = L::Q, NT = TX * TY;
    static_assert(TX % 64 == 0, "one (y, z) row per wavefront");
    constexpr int LDS_S = STATS ? 4 * (NT / 64) * 2 * Q : 1;
    __shared__ double lds_stats[LDS_S];
    const double2* tab = noise_table<Real, NT>();
    int x0, y0, z0;
    tile_origin<LAT, TX, TY * SPT, 1>(g, x0, y0, z0);
    const int tx = threadIdx.x % TX;
    const int ty = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / TX));
    const int x = x0 + tx, z = z0;
    const uint32_t step = st.get();
    Real v[STATS ? 2 * Q : 1];
    if (x0 + TX <= g.nx && y0 + TY * SPT <= g.ny && z < g.nz) {
        ip_site<LAT, Real, STATS, PH, true>(f, x, y0 + ty, z, g, P, step, tab, v);
#pragma unroll
        for (int sp = 1; sp < SPT; ++sp)
            ip_site<LAT, Real, STATS, PH, false>(f, x, y0 + ty + sp * TY, z, g, P, step, tab, v);
    } else {
        if constexpr (STATS) {
#pragma unroll
            for (int k = 0; k < 2 * Q; ++k) v[k] = Real(0);
        }
#pragma unroll
        for (int sp = 0; sp < SPT; ++sp) {
            const int y = y0 + ty + sp * TY;
            if (x < g.nx && y < g.ny && z < g.nz)
                ip_site<LAT, Real, STATS, PH, false>(f, x, y, z, g, P, step, tab, v);
        }
    }
    if constexpr (STATS) {
        const uint32_t b = xcd_remap(blockIdx.x, g.nblocks);
        block_accumulate<2 * Q, NT>(v, partial + (size_t)b * 2 * Q, lds_stats);
    }
}

// The next step's density formed inside the z-march.  After streaming, the
// density at x is sum_i S*_i(x - c_i) over the post-collision populations S*
// that the march has just computed.  Each thread keeps running sums for the
// planes of its column that can still receive.  The rest population and the
// two along z stay in the thread; the six that move along x only reach the
// neighbouring lane through a wavefront shift (DPP); the ten with c_y != 0
// go through LDS (NYS slots of one value per thread), written only by rows
// whose receiver row is in the tile.  A source counts when it lies in the
// same 64-wide x segment (one wavefront row), in the block's rows
// [y0, min(y0 + TY, ny)) and planes [zb, ze), and in the box.  The tile's
// first and last rows also sum, for each receiver of the row just outside
// the tile, the movers that cross into it (ghost rows, by the same shifts
// and running sums; the same segment and plane-run rules).  k_density_fix
// adds the ghost rows and every other source after the launch.  TX is a
// multiple of 64.
// Partial-density work area, element offsets from its start: the partial
// density (V floats), the edge records (16 floats per (z, y, 64-wide x
// segment)), then the two ghost-row arrays (receivers below a tile's first
// row, then above its last row), each sized for tiles of two rows
// (nz ceil(ny / 2) nx floats, indexed (z, tile row, x)).
struct PdLayout {
    size_t edge, ghost_bot, ghost_top, total;
};
__host__ __device__ inline PdLayout pd_layout(int nx, int ny, int nz) {
    const size_t V = (size_t)nx * ny * nz;
    const size_t nseg = ((size_t)nx + 63) / 64;
    const size_t e = (V + 63) / 64 * 64;
    const size_t gb = e + ((size_t)nz * ny * nseg * 16 + 63) / 64 * 64;
    const size_t gn = ((size_t)nz * ((ny + 1) / 2) * nx + 63) / 64 * 64;
    return PdLayout{e, gb, gb + gn, gb + 2 * gn};
}

template <int TX, int TY>
struct MarchDensity {
    using L = Lattice<1>;
    static_assert(TX % 64 == 0, "wavefront rows");
    static constexpr int NT = TX * TY, PAD = TX + 1;
    // with two rows each row sends in one direction only, so the two
    // directions share slots
    static constexpr int NYS = TY == 2 ? 5 : 10;
    static constexpr int LDS = NYS * NT + 2 * PAD;
    static constexpr int WAVE_SHL1 = 0x130, WAVE_SHR1 = 0x138;
    // slot of population i (c_y != 0): its rank among the five of its c_y sign
    static constexpr int yslot(int i) {
        return (i == 3 || i == 4) ? 0 : (i == 7 || i == 8) ? 1 : (i == 9 || i == 10) ? 2
             : (i == 15 || i == 17) ? 3 : 4;
    }
    static constexpr int ybase(int i) { return (TY == 2 || L::cy[i] == 1) ? 0 : 5; }
    // the in-plane exchange of the plane just computed: the x-only movers
    // into the sums (am: plane below, a0: this plane, ap: plane above), the
    // others into LDS.  Called by the lanes inside the box; a lane discards
    // what the shift brings from a neighbour outside its wavefront row or the
    // box (vxm, vxp false); up / down: this row has a receiver row above /
    // below in the tile.
    static __device__ __forceinline__ void put(float* lx, const float (&f)[L::Q], bool vxm, bool vxp,
                                               bool up, bool down, float& am, float& a0, float& ap) {
        // lane l receives from l - 1 (c_x = +1) and from l + 1 (c_x = -1)
        const float r1 = dpp_shift<WAVE_SHR1>(f[1]), r2 = dpp_shift<WAVE_SHL1>(f[2]);
        const float r11 = dpp_shift<WAVE_SHR1>(f[11]), r13 = dpp_shift<WAVE_SHL1>(f[13]);
        const float r12 = dpp_shift<WAVE_SHR1>(f[12]), r14 = dpp_shift<WAVE_SHL1>(f[14]);
        a0 += (vxm ? r1 : 0.f) + (vxp ? r2 : 0.f);
        ap += (vxm ? r11 : 0.f) + (vxp ? r13 : 0.f);
        am += (vxm ? r12 : 0.f) + (vxp ? r14 : 0.f);
#pragma unroll
        for (int i = 3; i < L::Q; ++i) {
            if (L::cy[i] == 0) continue;
            if (L::cy[i] == 1 ? up : down)
                lx[PAD + (ybase(i) + yslot(i)) * NT + (int)threadIdx.x] = f[i];
        }
    }
    // Edge records, one per (z, y, 64-wide x segment), EDGE floats: [0, 5)
    // the populations (1, 7, 8, 11, 12) (c_x = +1) of the segment's last
    // site (x & 63 == 63, or the box's last x), [8, 13) the populations
    // (2, 9, 10, 13, 14) (c_x = -1) of its first site.  These are the
    // sources that a segment's neighbours need and MarchDensity leaves out.
    static constexpr int EDGE = 16;
    static __device__ __forceinline__ uint32_t edge_record(int x, int y, int z, const Geom& g) {
        const uint32_t nseg = ((uint32_t)g.nx + 63u) >> 6;
        return (((uint32_t)z * (uint32_t)g.ny + (uint32_t)y) * nseg + ((uint32_t)x >> 6)) * EDGE;
    }
    static __device__ __forceinline__ void put_edge(float* edge, const float (&f)[L::Q], int x, int y,
                                                    int z, const Geom& g) {
        if ((x & 63) == 63 || x == g.nx - 1) {
            float* r = edge + edge_record(x, y, z, g);
            *(float4*)r = make_float4(f[1], f[7], f[8], f[11]);
            r[4] = f[12];
        }
        if ((x & 63) == 0) {
            float* r = edge + edge_record(x, y, z, g) + 8;
            *(float4*)r = make_float4(f[2], f[9], f[10], f[13]);
            r[4] = f[14];
        }
    }
    // Ghost-row sums of this row's plane z: bottom (the tile's first row):
    // the c_y = -1 movers for the row below, (0,-1,0) here, (+1,-1,0) from
    // x - 1 and (-1,-1,0) from x + 1 by the shifts, (0,-1,+1) into the next
    // plane's sum and (0,-1,-1) into the previous one's; top (the tile's last
    // row in the box) likewise with the c_y = +1 movers.  g: sums of planes
    // z - 1, z, z + 1 (the last assigned here).
    static __device__ __forceinline__ void put_ghost(const float (&f)[L::Q], bool vxm, bool vxp,
                                                     bool bottom, bool top, float (&gb)[3],
                                                     float (&gt)[3]) {
        if (bottom) {
            const float r8 = dpp_shift<WAVE_SHR1>(f[8]), r10 = dpp_shift<WAVE_SHL1>(f[10]);
            gb[0] += f[18];
            gb[1] += f[4] + ((vxm ? r8 : 0.f) + (vxp ? r10 : 0.f));
            gb[2] = f[17];
        }
        if (top) {
            const float r7 = dpp_shift<WAVE_SHR1>(f[7]), r9 = dpp_shift<WAVE_SHL1>(f[9]);
            gt[0] += f[16];
            gt[1] += f[3] + ((vxm ? r7 : 0.f) + (vxp ? r9 : 0.f));
            gt[2] = f[15];
        }
    }
    // the previous plane's c_y != 0 movers from the rows below (vym) and
    // above (vyp), into am (c_z = -1), a0 (c_z = 0) and ap (c_z = +1)
    static __device__ __forceinline__ void take(const float* lx, bool vxm, bool vxp, bool vym,
                                                bool vyp, float& am, float& a0, float& ap) {
#pragma unroll
        for (int i = 3; i < L::Q; ++i) {
            if (L::cy[i] == 0) continue;
            if (!(L::cy[i] == 1 ? vym : vyp)) continue;
            const float v = lx[PAD + (ybase(i) + yslot(i)) * NT + (int)threadIdx.x - L::cy[i] * TX - L::cx[i]];
            const float u = L::cx[i] == 1 ? (vxm ? v : 0.f) : (L::cx[i] == -1 ? (vxp ? v : 0.f) : v);
            if (L::cz[i] == -1) am += u;
            else if (L::cz[i] == 0) a0 += u;
            else ap += u;
        }
    }
};

template <bool PD, int TX, int TY>
struct MarchDensityLds { static constexpr int value = 1; };
template <int TX, int TY>
struct MarchDensityLds<true, TX, TY> { static constexpr int value = MarchDensity<TX, TY>::LDS; };

// D3Q19 force step, z-marching form: block b owns the column tile (x0, y0)
// of TX x TY sites and the planes [zb, zb + ZC) of it (ZC = g.zc).  The density
// and chemical potential live in LDS ring buffers (ForceMarch); the density
// plane two ahead is loaded into registers one plane early, and the
// populations of the current plane are requested before the barriers, so
// global loads overlap the LDS work.  NTS: populations stored with
// non-temporal hints (the state of a large lattice does not stay in the cache).
// PD: the block also writes the next step's density from its own sources to
// rho_part (MarchDensity), and the outflow of each 64-wide x segment's first
// and last site to edge records (MarchDensity::EDGE), which k_density_fix
// uses to complete it.
template <typename Real, bool STATS, int TX, int TY, bool NTS = false, bool PD = false>
__global__ __launch_bounds__(TX* TY) void k_step_march(
    const Real* __restrict__ fin, Real* __restrict__ fout, const Real* __restrict__ drho, Geom g,
    CollideParams<Real> P, ForceParams<Real> fp, StepIndex st, double* __restrict__ partial,
    Real* __restrict__ rho_part, Real* __restrict__ edge, Real* __restrict__ ghost_bot,
    Real* __restrict__ ghost_top) {
    using L = Lattice<1>;
    using M = Moments<1, Real>;
    using FM = ForceMarch<Real, TX, TY>;
    using MD = MarchDensity<TX, TY>;
    static_assert(!PD || std::is_same<Real, float>::value, "partial density: FP32");
    constexpr int Q = L::Q, NT = TX * TY;
    constexpr bool ROWS = (TX % 64) == 0;
    constexpr int LDS_S = STATS ? 4 * ((NT + 63) / 64) * 2 * Q : 1;
    __shared__ Real lds_r[5 * FM::NRP];
    __shared__ Real lds_m[3 * FM::NMP];
    __shared__ double lds_stats[LDS_S];
    __shared__ Real lds_x[MarchDensityLds<PD, TX, TY>::value];

    const uint32_t b = xcd_remap(blockIdx.x, g.nblocks);
    const uint32_t ncol = (uint32_t)g.nbx * (uint32_t)g.nby;
    const uint32_t col = b % ncol, chunk = b / ncol;
    const int x0 = (int)(col % (uint32_t)g.nbx) * TX, y0 = (int)(col / (uint32_t)g.nbx) * TY;
    const int zb = (int)chunk * g.zc;
    const int ze = min(zb + g.zc, g.nz);
    const int tx = threadIdx.x % TX;
    int ty = threadIdx.x / TX;
    if constexpr (ROWS) ty = __builtin_amdgcn_readfirstlane(ty);
    const int x = x0 + tx, y = y0 + ty;
    const bool inxy = x < g.nx && y < g.ny;

    uint32_t off[FM::NLD];
    FM::plane_offsets(g, x0, y0, off);
    Real rreg[FM::NLD];
#pragma unroll 1
    for (int z = zb - 2; z <= zb + 1; ++z) {
        FM::load_plane(drho, g, off, z, rreg);
        FM::store_plane(rreg, lds_r + FM::rslot(z, zb) * FM::NRP);
    }
    __syncthreads();
    FM::mu_plane(lds_r, lds_m, zb - 1, zb, fp);
    FM::mu_plane(lds_r, lds_m, zb, zb, fp);
    FM::load_plane(drho, g, off, zb + 2, rreg);

    Real v[2 * Q];
    if constexpr (STATS) {
#pragma unroll
        for (int k = 0; k < 2 * Q; ++k) v[k] = Real(0);
    }
    // PD: sums of the next density at planes z - 2 .. z + 1 of this column
    // (at the top of iteration z); which in-plane neighbours are sources
    // (x - 1, x + 1 in this wavefront row, y - 1, y + 1 in the tile, in the
    // box) and which neighbour rows of the tile receive from this one
    Real a_m2 = Real(0), a_m1 = Real(0), a_0 = Real(0), a_p1 = Real(0);
    const bool vxm = (x & 63) != 0, vxp = (x & 63) != 63 && x + 1 < g.nx;
    const bool vym = ty >= 1, vyp = ty + 1 < TY && y + 1 < g.ny;
    const bool up = ty + 1 < TY, down = ty >= 1;
    // ghost rows: this row is the tile's first / last row in the box
    const bool gbot = ty == 0, gtop = ty == min(TY, g.ny - y0) - 1;
    Real gsb[3] = {Real(0), Real(0), Real(0)}, gst[3] = {Real(0), Real(0), Real(0)};
    const uint32_t grow = (uint32_t)(y0 / TY);
    const uint32_t step = st.get();
#pragma unroll 1
    for (int z = zb; z < ze; ++z) {
        FM::store_plane(rreg, lds_r + FM::rslot(z + 2, zb) * FM::NRP);
        if (z + 1 < ze) FM::load_plane(drho, g, off, z + 3, rreg);
        // x is re-read each plane, so that per-plane lane addresses are not
        // hoisted out of the loop (they would hold two VGPRs per plane); the
        // plane stride likewise, so that the 19 64-bit plane bases are formed
        // by scalar arithmetic next to their accesses instead of being held
        // in SGPRs through the loop (which spills them to VGPR lanes)
        int xl = x;
        asm volatile("" : "+v"(xl));
        Geom gz = g;
        asm volatile("" : "+s"(gz.V));
        Real f[Q];
        if (inxy) {
            if constexpr (ROWS) pull_rows<1, Real>(fin, xl, y, z, gz, f);
            else pull<1, Real>(fin, xl, y, z, gz, f);
        }
        __syncthreads();
        FM::mu_plane(lds_r, lds_m, z + 1, zb, fp);
        if constexpr (PD) {
            // plane z - 1's exchange; plane z - 2 then has all its sources
            if (z > zb) {
                MD::take(lds_x, vxm, vxp, vym, vyp, a_m2, a_m1, a_0);
                if (z - 2 >= zb && inxy)
                    plane_st(rho_part + (size_t)(uint32_t)(((z - 2) * g.ny + y) * g.nx), (uint32_t)xl, a_m2);
            }
        }
        __syncthreads();
        if (inxy) {
            Real F[3];
            FM::force(lds_r, lds_m, z, zb, fp, P.rho0, tx, ty, F);
            Real m[Q];
            M::forward(f, m);
            if constexpr (STATS) {
#pragma unroll
                for (int a = 0; a < Q; ++a) {
                    v[a] += m[a];
                    v[Q + a] += m[a] * m[a];
                }
            }
            const uint32_t site = (uint32_t)((z * g.ny + y) * g.nx + xl);
            Real zn[2 * L::NPAIR];
            if (P.noise_on) {
                // the key is re-read each plane, so that Philox's round keys are
                // formed next to their use instead of being held in SGPRs through
                // the loop (which spills them to VGPR lanes)
                uint32_t k0 = P.key0, k1 = P.key1;
                asm volatile("" : "+s"(k0), "+s"(k1));
                site_normals<L::NPAIR, Real>(site, step, 0u, P.replica, k0, k1, zn);
            }
            collide_moments<1, Real, true>(m, F, zn, P);
            M::inverse(m, f);
            if constexpr (PD) {
                a_m1 += f[6];   // (0, 0, -1) reaches plane z - 1
                a_0 += f[0];
                a_p1 = f[5];    // (0, 0, +1) reaches plane z + 1
                MD::put(lds_x, f, vxm, vxp, up, down, a_m1, a_0, a_p1);
                MD::put_edge(edge, f, x, y, z, g);
                MD::put_ghost(f, vxm, vxp, gbot, gtop, gsb, gst);
                // ghost plane z - 1 has all its sources
                if (z - 1 >= zb) {
                    const uint32_t gi = ((uint32_t)(z - 1) * (uint32_t)g.nby + grow) * (uint32_t)g.nx + (uint32_t)x;
                    if (gbot) ghost_bot[gi] = gsb[0];
                    if (gtop) ghost_top[gi] = gst[0];
                }
            }
            if constexpr (ROWS) {
                const size_t row = (size_t)(uint32_t)((z * g.ny + y) * g.nx);
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if constexpr (NTS) plane_st_nt(fout + ((size_t)i * gz.V + row), (uint32_t)xl, f[i]);
                    else plane_st(fout + ((size_t)i * gz.V + row), (uint32_t)xl, f[i]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) plane_st(fout + (size_t)i * gz.V, site, f[i]);
            }
        }
        if constexpr (PD) {
            a_m2 = a_m1;
            a_m1 = a_0;
            a_0 = a_p1;
            gsb[0] = gsb[1];
            gsb[1] = gsb[2];
            gst[0] = gst[1];
            gst[1] = gst[2];
        }
    }
    if constexpr (PD) {
        // the last plane's exchange completes planes ze - 2 and ze - 1 (the
        // sources of ze - 1 in plane ze belong to the next block in z)
        __syncthreads();
        MD::take(lds_x, vxm, vxp, vym, vyp, a_m2, a_m1, a_0);
        if (inxy) {
            if (ze - 2 >= zb)
                plane_st(rho_part + (size_t)(uint32_t)(((ze - 2) * g.ny + y) * g.nx), (uint32_t)x, a_m2);
            plane_st(rho_part + (size_t)(uint32_t)(((ze - 1) * g.ny + y) * g.nx), (uint32_t)x, a_m1);
            // ghost plane ze - 1 (its sources in plane ze belong to the next block)
            const uint32_t gi = ((uint32_t)(ze - 1) * (uint32_t)g.nby + grow) * (uint32_t)g.nx + (uint32_t)x;
            if (gbot) ghost_bot[gi] = gsb[0];
            if (gtop) ghost_top[gi] = gst[0];
        }
    }
    if constexpr (STATS) block_accumulate<2 * Q, NT>(v, partial + (size_t)b * 2 * Q, lds_stats);
}

// Completes the march's partial density: adds to rho_part(x) the streamed
// populations S*_i(x - c_i) whose source the forming block left out (outside
// the 64-wide x segment of x, the TY rows of its tile from the origin, its
// run of g.zc planes, as in k_step_march / MarchDensity).  A block of four
// wavefronts covers 64 SPL sites of x (from 64 SPL bx) in RY rows of plane z,
// each wavefront RY / 4 rows, SPL sites per lane.  A tile's first (last) row
// adds the ghost row that the march of the tile below (above) formed for it:
// the sources across the y edge in the same segment and plane run.  Whether
// a population crosses the plane run's edge is uniform, so those
// populations are read as whole rows under scalar branches.  A segment's
// first lane (x & 63 == 0) and last lane (x & 63 == 63, or the box's last x)
// take the other x movers from the neighbouring segments' edge records.
// The sum runs over the partial density, the ghost rows, then the
// populations in the order i = 1 .. Q - 1.
constexpr int FIX_SPL = 2;   // sites per lane of k_density_fix (2 measured best of 1, 2, 4)
template <int TY>
__global__ __launch_bounds__(256) void k_density_fix(const float* __restrict__ fin,
                                                     const float* __restrict__ rho_part,
                                                     const float* __restrict__ edge,
                                                     const float* __restrict__ ghost_bot,
                                                     const float* __restrict__ ghost_top,
                                                     float* __restrict__ out, Geom g) {
    using L = Lattice<1>;
    constexpr int SPL = FIX_SPL, RY = 16;
    const int z = (int)blockIdx.z;
    const int zb = z - z % g.zc;
    const bool zlo = z == zb, zhi = z + 1 == min(zb + g.zc, g.nz);
    const uint32_t nxy = (uint32_t)g.nx * (uint32_t)g.ny;
    const uint32_t nseg = ((uint32_t)g.nx + 63u) >> 6;
    const uint32_t szm = z == 0 ? (uint32_t)(g.nz - 1) * nxy : 0u - nxy;
    const uint32_t szp = z == g.nz - 1 ? 0u - (uint32_t)(g.nz - 1) * nxy : nxy;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    const int lane = (int)threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    // lanes past the box's last x read at the last x (valid addresses) and
    // store nothing
    int xs[SPL];
    uint32_t sxm[SPL], sxp[SPL];
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
        const int x = min((int)(blockIdx.x * (64u * SPL)) + 64 * k + lane, g.nx - 1);
        xs[k] = x;
        sxm[k] = x == 0 ? (uint32_t)(g.nx - 1) : 0u - 1u;
        sxp[k] = x == g.nx - 1 ? 0u - (uint32_t)(g.nx - 1) : 1u;
    }
#pragma unroll 1
    for (int y = (int)blockIdx.y * RY + wave; y < min((int)(blockIdx.y + 1) * RY, g.ny); y += 4) {
        const int y0 = y - y % TY;
        const bool ylo = y == y0, yhi = y + 1 == min(y0 + TY, g.ny);
        const uint32_t row = (uint32_t)z * nxy + (uint32_t)y * (uint32_t)g.nx;
        const uint32_t sym = y == 0 ? (uint32_t)(g.ny - 1) * (uint32_t)g.nx : 0u - (uint32_t)g.nx;
        const uint32_t syp = y == g.ny - 1 ? 0u - (uint32_t)(g.ny - 1) * (uint32_t)g.nx : (uint32_t)g.nx;
        const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
        auto src = [&](int i, int k) {
            return row + (uint32_t)xs[k] + (L::cx[i] == 0 ? 0u : (L::cx[i] > 0 ? sxm[k] : sxp[k])) +
                   (L::cy[i] == 0 ? 0u : (L::cy[i] > 0 ? sym : syp)) +
                   (L::cz[i] == 0 ? 0u : (L::cz[i] > 0 ? szm : szp));
        };
        // the edge record of the source of population i (c_x != 0) at x
        auto rec = [&](int i, int x) {
            const int sx = L::cx[i] > 0 ? (x == 0 ? g.nx - 1 : x - 1) : (x == g.nx - 1 ? 0 : x + 1);
            const int sy = L::cy[i] == 0 ? y : (L::cy[i] > 0 ? ym : yp);
            const int sz = L::cz[i] == 0 ? z : (L::cz[i] > 0 ? zm : zp);
            constexpr int slot[L::Q] = {0, 0, 8, 0, 0, 0, 0, 1, 2, 9, 10, 3, 4, 11, 12, 0, 0, 0, 0};
            return ((uint32_t)sz * (uint32_t)g.ny + (uint32_t)sy) * nseg * 16u +
                   ((uint32_t)sx >> 6) * 16u + (uint32_t)slot[i];
        };
        float v[SPL][L::Q], gv[SPL][2];
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            gv[k][0] = gv[k][1] = 0.f;
#pragma unroll
            for (int i = 1; i < L::Q; ++i) v[k][i] = 0.f;
        }
        // a tile's edge row: the ghost row that the neighbouring tile's march
        // formed for it (sources across the y edge, same segment and run)
        if (ylo) {
            const uint32_t gi = ((uint32_t)z * (uint32_t)g.nby + (uint32_t)(ym / TY)) * (uint32_t)g.nx;
#pragma unroll
            for (int k = 0; k < SPL; ++k) gv[k][0] = ghost_top[gi + (uint32_t)xs[k]];
        }
        if (yhi) {
            const uint32_t gi = ((uint32_t)z * (uint32_t)g.nby + (uint32_t)(yp / TY)) * (uint32_t)g.nx;
#pragma unroll
            for (int k = 0; k < SPL; ++k) gv[k][1] = ghost_bot[gi + (uint32_t)xs[k]];
        }
        // whole rows: sources across the plane run's z edge
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const bool oz = (L::cz[i] == 1 && zlo) || (L::cz[i] == -1 && zhi);
            if (oz) {
#pragma unroll
                for (int k = 0; k < SPL; ++k) v[k][i] = plane_ld(fin + (size_t)i * g.V, src(i, k));
            }
        }
        // segment edges, for the x movers not read as whole rows (also those
        // crossing the y edge: the ghost rows leave them out)
        if (lane == 0) {
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                if (L::cx[i] != 1) continue;
                const bool oz = (L::cz[i] == 1 && zlo) || (L::cz[i] == -1 && zhi);
                if (!oz) {
#pragma unroll
                    for (int k = 0; k < SPL; ++k) v[k][i] = edge[rec(i, xs[k])];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            if (lane == 63 || xs[k] + 1 == g.nx) {
#pragma unroll
                for (int i = 1; i < L::Q; ++i) {
                    if (L::cx[i] != -1) continue;
                    const bool oz = (L::cz[i] == 1 && zlo) || (L::cz[i] == -1 && zhi);
                    if (!oz) v[k][i] = edge[rec(i, xs[k])];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            if ((int)(blockIdx.x * (64u * SPL)) + 64 * k + lane >= g.nx) break;
            const uint32_t site = row + (uint32_t)xs[k];
            float acc = plane_ld(rho_part, site) + gv[k][0] + gv[k][1];
#pragma unroll
            for (int i = 1; i < L::Q; ++i) acc += v[k][i];
            plane_st(out, site, acc);
        }
    }
}

// rho and rho u = sum c f + F/2 after streaming of state fin.
template <int LAT, typename Real, bool FORCE, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX* TY* TZ) void k_fields(const Real* __restrict__ fin,
                                                        const Real* __restrict__ drho,
                                                        Real* __restrict__ out, Geom g, Real rho0,
                                                        ForceParams<Real> fp) {
    using L = Lattice<LAT>;
    using FT = ForceTile<LAT, Real, TX, TY, TZ>;
    constexpr int Q = L::Q, D = L::D;
    constexpr int LDS_F = FORCE ? (FT::NR + FT::NM) : 1;
    __shared__ Real lds_force[LDS_F];
    int x0, y0, z0;
    tile_origin<LAT, TX, TY, TZ>(g, x0, y0, z0);
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    const bool inside = x < g.nx && y < g.ny && z < g.nz;
    Real F[D];
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] = Real(0);
    if constexpr (FORCE) {
        FT::stage(drho, g, fp, x0, y0, z0, lds_force, lds_force + FT::NR);
        if (inside) FT::force(lds_force, lds_force + FT::NR, fp, rho0, tx, ty, tz, F);
    }
    if (!inside) return;
    Real f[Q];
    pull<LAT, Real>(fin, x, y, z, g, f);
    Real rho = Real(0), j[D];
#pragma unroll
    for (int a = 0; a < D; ++a) j[a] = Real(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        const int c3[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (c3[a] == 1) j[a] += f[i];
            else if (c3[a] == -1) j[a] -= f[i];
        }
    }
    const uint32_t s = site_index<LAT>(x, y, z, g);
    out[s] = rho0 + rho;
#pragma unroll
    for (int a = 0; a < D; ++a) out[(size_t)(1 + a) * g.V + s] = j[a] + Real(0.5) * F[a];
}

// Fixed-order reduction of the statistics slots: out[k] = sum_b partial[b][k].
__global__ void k_stats_finalize(const double* __restrict__ partial, uint32_t nslots, int nvals,
                                 double* __restrict__ out) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (uint32_t b = threadIdx.x; b < nslots; b += 256) acc += partial[(size_t)b * nvals + k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
}

__global__ void k_noise_words(unsigned long long site0, unsigned long long nsites, uint32_t step,
                              uint32_t word2, uint32_t replica, uint32_t k0, uint32_t k1,
                              uint32_t* __restrict__ out) {
    const unsigned long long s = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsites) return;
    const Philox4 r = philox4x32_10((uint32_t)(site0 + s), step, word2, replica, k0, k1);
    out[4 * s + 0] = r.x;
    out[4 * s + 1] = r.y;
    out[4 * s + 2] = r.z;
    out[4 * s + 3] = r.w;
}

// The 2 NPAIR Box-Muller normals of sites site0 .. site0 + nsites - 1 (tag 0).
template <int NPAIR, typename Real>
__global__ void k_noise_normals(unsigned long long site0, unsigned long long nsites, uint32_t step,
                                uint32_t replica, uint32_t k0, uint32_t k1,
                                Real* __restrict__ out) {
    const unsigned long long s = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsites) return;
    Real z[2 * NPAIR];
    site_normals<NPAIR, Real>((uint32_t)(site0 + s), step, 0u, replica, k0, k1, z);
#pragma unroll
    for (int k = 0; k < 2 * NPAIR; ++k) out[(size_t)(2 * NPAIR) * s + k] = z[k];
}

__global__ void k_add_u64(unsigned long long* ctr, unsigned long long inc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr += inc;
}

__global__ void k_set_u64(unsigned long long* ctr, unsigned long long v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = v;
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------------ launchers

int n_configs(int lat, int force) {
    if (!force) return N_IDEAL_CFG;
    return lat == 1 ? N_FORCE3_CFG : N_FORCE2_CFG;
}

TileShape config_shape(int lat, int force, int cfg) {
    if (!force) return IDEAL_CFG[cfg];
    return lat == 1 ? FORCE3_CFG[cfg] : FORCE2_CFG[cfg];
}

static Geom make_geom(const StepSpec& s, TileShape t) {
    Geom g{};
    g.nx = s.nx;
    g.ny = s.ny;
    g.nz = s.nz;
    const int ty = t.ty * (t.spt > 1 ? t.spt : 1);
    const int tz = t.zc > 0 ? t.zc : t.tz;
    g.nbx = (s.nx + t.tx - 1) / t.tx;
    g.nby = (s.ny + ty - 1) / ty;
    g.nbz = (s.nz + tz - 1) / tz;
    g.zc = t.zc;
    g.nblocks = (uint32_t)g.nbx * g.nby * g.nbz;
    g.V = (uint32_t)s.nx * s.ny * s.nz;
    return g;
}

uint32_t config_blocks(const StepSpec& s, int cfg) {
    return make_geom(s, config_shape(s.lat, s.force, cfg)).nblocks;
}

template <typename Real>
static CollideParams<Real> collide_params(const StepSpec& s) {
    CollideParams<Real> P;
    P.rho0 = (Real)s.rho0;
    P.lam_bulk = (Real)s.lam_bulk;
    P.lam_shear = (Real)s.lam_shear;
    P.lam_ghost = (Real)s.lam_ghost;
    for (int c = 0; c < 3; ++c) P.amp_cls[c] = (Real)s.amp_cls[c];
    P.noise_on = s.noise_on;
    P.noise_local = s.noise_local;
    P.key0 = s.key0;
    P.key1 = s.key1;
    P.replica = s.replica;
    P.nonfinite = s.nonfinite;
    return P;
}

template <typename Real>
static ForceParams<Real> force_params(const StepSpec& s) {
    ForceParams<Real> f;
    f.a = (Real)s.a;
    f.b = (Real)s.b;
    f.shift = (Real)(s.rho0 - s.rho_c);
    f.kappa = (Real)s.kappa;
    f.eta = (Real)s.eta;
    return f;
}

hipError_t launch_init(const StepSpec& s, void* f, const double* drho, hipStream_t st) {
    const uint32_t V = (uint32_t)s.nx * s.ny * s.nz;
    const dim3 grid((V + 255) / 256), block(256);
    if (s.lat == 0 && s.prec == 0) hipLaunchKernelGGL((k_init<0, float>), grid, block, 0, st, (float*)f, drho, V);
    else if (s.lat == 0) hipLaunchKernelGGL((k_init<0, double>), grid, block, 0, st, (double*)f, drho, V);
    else if (s.prec == 0) hipLaunchKernelGGL((k_init<1, float>), grid, block, 0, st, (float*)f, drho, V);
    else hipLaunchKernelGGL((k_init<1, double>), grid, block, 0, st, (double*)f, drho, V);
    return hipGetLastError();
}

hipError_t launch_density(const StepSpec& s, const void* fin, void* out, hipStream_t st) {
    const Geom g = make_geom(s, TileShape{1, 1, 1, 1, 0, 0, 0});
    const dim3 grid((g.V + 255) / 256), block(256);
    if (s.lat == 0 && s.prec == 0) hipLaunchKernelGGL((k_density<0, float>), grid, block, 0, st, (const float*)fin, (float*)out, g);
    else if (s.lat == 0) hipLaunchKernelGGL((k_density<0, double>), grid, block, 0, st, (const double*)fin, (double*)out, g);
    else if (s.prec == 0) hipLaunchKernelGGL((k_density<1, float>), grid, block, 0, st, (const float*)fin, (float*)out, g);
    else hipLaunchKernelGGL((k_density<1, double>), grid, block, 0, st, (const double*)fin, (double*)out, g);
    return hipGetLastError();
}

template <int LAT, typename Real, bool FORCE, int TX, int TY, int TZ, int SPT = 1, bool NTS = false,
          bool FUSED = false>
static void step_tile(const StepSpec& s, const void* fin, void* fout, const void* drho,
                      StepIndex si, double* partial, hipStream_t st, void* rho_out = nullptr) {
    const Geom g = make_geom(s, TileShape{TX, TY, TZ, SPT, NTS, 0, 0});
    const dim3 grid(g.nblocks), block(TX * TY * TZ);
    const CollideParams<Real> P = collide_params<Real>(s);
    const ForceParams<Real> fp = force_params<Real>(s);
    Real* ro = FUSED ? (Real*)rho_out : nullptr;
    if (partial)
        hipLaunchKernelGGL((k_step<LAT, Real, FORCE, true, TX, TY, TZ, SPT, NTS, FUSED>), grid, block, 0, st,
                           (const Real*)fin, (Real*)fout, (const Real*)drho, g, P, fp, si, partial, ro);
    else
        hipLaunchKernelGGL((k_step<LAT, Real, FORCE, false, TX, TY, TZ, SPT, NTS, FUSED>), grid, block, 0, st,
                           (const Real*)fin, (Real*)fout, (const Real*)drho, g, P, fp, si, partial, ro);
}

// rho_part: the partial next density (partial-density shapes: FP32, TX a
// multiple of 64; null runs the plain march of the same shape).
template <typename Real, int TX, int TY, bool NTS = false>
static void step_march(const StepSpec& s, int zc, const void* fin, void* fout, const void* drho,
                       StepIndex si, double* partial, hipStream_t st, void* rho_part = nullptr) {
    const Geom g = make_geom(s, TileShape{TX, TY, 1, 1, NTS, zc, 0});
    const dim3 grid(g.nblocks), block(TX * TY);
    const CollideParams<Real> P = collide_params<Real>(s);
    const ForceParams<Real> fp = force_params<Real>(s);
    if constexpr (std::is_same<Real, float>::value && TX % 64 == 0) {
        Real* rp = (Real*)rho_part;
        const PdLayout lay = pd_layout(s.nx, s.ny, s.nz);
        Real* ed = rp ? rp + lay.edge : nullptr;
        Real* gb = rp ? rp + lay.ghost_bot : nullptr;
        Real* gt = rp ? rp + lay.ghost_top : nullptr;
        if (rp && partial) {
            hipLaunchKernelGGL((k_step_march<Real, true, TX, TY, NTS, true>), grid, block, 0, st,
                               (const Real*)fin, (Real*)fout, (const Real*)drho, g, P, fp, si, partial, rp, ed,
                               gb, gt);
            return;
        }
        if (rp) {
            hipLaunchKernelGGL((k_step_march<Real, false, TX, TY, NTS, true>), grid, block, 0, st,
                               (const Real*)fin, (Real*)fout, (const Real*)drho, g, P, fp, si, partial, rp, ed,
                               gb, gt);
            return;
        }
    }
    Real* const none = nullptr;
    if (partial) {
        hipLaunchKernelGGL((k_step_march<Real, true, TX, TY, NTS>), grid, block, 0, st, (const Real*)fin,
                           (Real*)fout, (const Real*)drho, g, P, fp, si, partial, none, none, none, none);
    } else {
        hipLaunchKernelGGL((k_step_march<Real, false, TX, TY, NTS>), grid, block, 0, st, (const Real*)fin,
                           (Real*)fout, (const Real*)drho, g, P, fp, si, partial, none, none, none, none);
    }
}

template <int LAT, typename Real>
static void step_dispatch(const StepSpec& s, int cfg, const void* fin, void* fout,
                          const void* drho, StepIndex si, double* partial, hipStream_t st,
                          void* rho_out, void* rho_part) {
    if (!s.force) {
        switch (cfg) {
            case 0: step_tile<LAT, Real, false, 64, 4, 1, 1>(s, fin, fout, drho, si, partial, st); break;
            case 1: step_tile<LAT, Real, false, 128, 2, 1, 1>(s, fin, fout, drho, si, partial, st); break;
            case 2: step_tile<LAT, Real, false, 256, 1, 1, 1>(s, fin, fout, drho, si, partial, st); break;
            case 3: step_tile<LAT, Real, false, 32, 8, 1, 1>(s, fin, fout, drho, si, partial, st); break;
            case 4: step_tile<LAT, Real, false, 128, 2, 1, 2>(s, fin, fout, drho, si, partial, st); break;
            case 5: step_tile<LAT, Real, false, 64, 4, 1, 2>(s, fin, fout, drho, si, partial, st); break;
            case 6: step_tile<LAT, Real, false, 128, 2, 1, 4>(s, fin, fout, drho, si, partial, st); break;
            case 7: step_tile<LAT, Real, false, 256, 1, 1, 2>(s, fin, fout, drho, si, partial, st); break;
            case 8: step_tile<LAT, Real, false, 128, 2, 1, 1, true>(s, fin, fout, drho, si, partial, st); break;
            case 9: step_tile<LAT, Real, false, 256, 1, 1, 1, true>(s, fin, fout, drho, si, partial, st); break;
            // in-place shapes: a lone step (not part of a pair) uses the ordinary kernel
            case 10: step_tile<LAT, Real, false, 128, 2, 1, 1>(s, fin, fout, drho, si, partial, st); break;
            case 11: step_tile<LAT, Real, false, 64, 4, 1, 1>(s, fin, fout, drho, si, partial, st); break;
            case 12: step_tile<LAT, Real, false, 256, 1, 1, 1>(s, fin, fout, drho, si, partial, st); break;
            case 13: step_tile<LAT, Real, false, 128, 2, 1, 2>(s, fin, fout, drho, si, partial, st); break;
            default: step_tile<LAT, Real, false, 64, 4, 1, 2>(s, fin, fout, drho, si, partial, st); break;
        }
    } else if constexpr (LAT == 1) {
        switch (cfg) {
            case 0: step_tile<LAT, Real, true, 32, 4, 2>(s, fin, fout, drho, si, partial, st); break;
            case 1: step_tile<LAT, Real, true, 16, 4, 4>(s, fin, fout, drho, si, partial, st); break;
            case 2: step_tile<LAT, Real, true, 64, 2, 2>(s, fin, fout, drho, si, partial, st); break;
            case 3: step_march<Real, 64, 4>(s, 16, fin, fout, drho, si, partial, st); break;
            case 4: step_march<Real, 64, 4>(s, 32, fin, fout, drho, si, partial, st); break;
            case 5: step_march<Real, 32, 8>(s, 16, fin, fout, drho, si, partial, st); break;
            case 6: step_march<Real, 64, 8>(s, 16, fin, fout, drho, si, partial, st); break;
            case 7: step_march<Real, 128, 2>(s, 16, fin, fout, drho, si, partial, st); break;
            case 8: step_march<Real, 128, 2, true>(s, 16, fin, fout, drho, si, partial, st); break;
            // the march also forms the next density (rho_part, completed by k_density_fix)
            case 9: step_march<Real, 128, 2, true>(s, 16, fin, fout, drho, si, partial, st, rho_part); break;
            case 10: step_march<Real, 64, 4>(s, 16, fin, fout, drho, si, partial, st, rho_part); break;
            default: step_march<Real, 64, 8>(s, 16, fin, fout, drho, si, partial, st, rho_part); break;
        }
    } else {
        switch (cfg) {
            case 0: step_tile<LAT, Real, true, 64, 4, 1>(s, fin, fout, drho, si, partial, st); break;
            case 1: step_tile<LAT, Real, true, 32, 8, 1>(s, fin, fout, drho, si, partial, st); break;
            case 2: step_tile<LAT, Real, true, 128, 2, 1>(s, fin, fout, drho, si, partial, st); break;
            case 3: step_tile<LAT, Real, true, 64, 4, 1, 1, false, true>(s, fin, fout, drho, si, partial, st, rho_out); break;
            case 4: step_tile<LAT, Real, true, 32, 8, 1, 1, false, true>(s, fin, fout, drho, si, partial, st, rho_out); break;
            default: step_tile<LAT, Real, true, 128, 2, 1, 1, false, true>(s, fin, fout, drho, si, partial, st, rho_out); break;
        }
    }
}

template <int LAT, typename Real, int TX, int TY, int SPT = 1>
static void step_ip(const StepSpec& s, int phase, void* f, StepIndex si, double* partial,
                    hipStream_t st) {
    const Geom g = make_geom(s, TileShape{TX, TY, 1, SPT, 0, 0, 1});
    const dim3 grid(g.nblocks), block(TX * TY);
    const CollideParams<Real> P = collide_params<Real>(s);
    if (phase == 0) {
        if (partial) hipLaunchKernelGGL((k_step_ip<LAT, Real, true, 0, TX, TY, SPT>), grid, block, 0, st, (Real*)f, g, P, si, partial);
        else hipLaunchKernelGGL((k_step_ip<LAT, Real, false, 0, TX, TY, SPT>), grid, block, 0, st, (Real*)f, g, P, si, partial);
    } else {
        if (partial) hipLaunchKernelGGL((k_step_ip<LAT, Real, true, 1, TX, TY, SPT>), grid, block, 0, st, (Real*)f, g, P, si, partial);
        else hipLaunchKernelGGL((k_step_ip<LAT, Real, false, 1, TX, TY, SPT>), grid, block, 0, st, (Real*)f, g, P, si, partial);
    }
}

template <int LAT, typename Real>
static void ip_dispatch(const StepSpec& s, int cfg, int phase, void* f, StepIndex si,
                        double* partial, hipStream_t st) {
    switch (cfg) {
        case 10: step_ip<LAT, Real, 128, 2>(s, phase, f, si, partial, st); break;
        case 11: step_ip<LAT, Real, 64, 4>(s, phase, f, si, partial, st); break;
        case 13: step_ip<LAT, Real, 128, 2, 2>(s, phase, f, si, partial, st); break;
        case 14: step_ip<LAT, Real, 64, 4, 2>(s, phase, f, si, partial, st); break;
        default: step_ip<LAT, Real, 256, 1>(s, phase, f, si, partial, st); break;
    }
}

bool config_partial_density(const StepSpec& s, int cfg) {
    // the completion pass launches one block per plane in grid z and one per
    // 16 rows in grid y (each below 2^16); otherwise the plain march runs
    return s.force && s.prec == 0 && s.nz <= 65535 && (s.ny + 15) / 16 <= 65535 && cfg >= 0 &&
           cfg < n_configs(s.lat, s.force) && config_shape(s.lat, s.force, cfg).pd;
}

size_t partial_density_bytes(const StepSpec& s) {
    if (!(s.force && s.lat == 1 && s.prec == 0)) return 0;
    return pd_layout(s.nx, s.ny, s.nz).total * 4;
}

hipError_t launch_density_fix(const StepSpec& s, int cfg, const void* fin, const void* rho_part,
                              void* out, hipStream_t st) {
    if (!config_partial_density(s, cfg)) return hipErrorInvalidValue;
    const TileShape t = config_shape(s.lat, s.force, cfg);
    const Geom g = make_geom(s, t);
    const dim3 grid((s.nx + 64 * FIX_SPL - 1) / (64 * FIX_SPL), (s.ny + 15) / 16, s.nz), block(256);
    const float* f = (const float*)fin;
    const float* rp = (const float*)rho_part;
    const PdLayout lay = pd_layout(s.nx, s.ny, s.nz);
    const float* ed = rp + lay.edge;
    const float* gb = rp + lay.ghost_bot;
    const float* gt = rp + lay.ghost_top;
    float* o = (float*)out;
    if (t.tx % 64 != 0) return hipErrorInvalidValue;
    if (t.ty == 2) hipLaunchKernelGGL((k_density_fix<2>), grid, block, 0, st, f, rp, ed, gb, gt, o, g);
    else if (t.ty == 4) hipLaunchKernelGGL((k_density_fix<4>), grid, block, 0, st, f, rp, ed, gb, gt, o, g);
    else if (t.ty == 8) hipLaunchKernelGGL((k_density_fix<8>), grid, block, 0, st, f, rp, ed, gb, gt, o, g);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

bool config_fused(const StepSpec& s, int cfg) {
    return s.force && cfg >= 0 && cfg < n_configs(s.lat, s.force) &&
           config_shape(s.lat, s.force, cfg).fd;
}

bool config_in_place(const StepSpec& s, int cfg) {
    return cfg >= 0 && cfg < n_configs(s.lat, s.force) && config_shape(s.lat, s.force, cfg).ip;
}

hipError_t launch_step_in_place(const StepSpec& s, int cfg, int phase, void* f,
                                const unsigned long long* step_dev, unsigned long long step_host,
                                double* partial, hipStream_t st) {
    if (!config_in_place(s, cfg) || phase < 0 || phase > 1) return hipErrorInvalidValue;
    StepIndex si{step_dev, step_host};
    if (s.lat == 0 && s.prec == 0) ip_dispatch<0, float>(s, cfg, phase, f, si, partial, st);
    else if (s.lat == 0) ip_dispatch<0, double>(s, cfg, phase, f, si, partial, st);
    else if (s.prec == 0) ip_dispatch<1, float>(s, cfg, phase, f, si, partial, st);
    else ip_dispatch<1, double>(s, cfg, phase, f, si, partial, st);
    return hipGetLastError();
}

hipError_t launch_step(const StepSpec& s, int cfg, const void* fin, void* fout, const void* drho,
                       const unsigned long long* step_dev, unsigned long long step_host,
                       double* partial, hipStream_t st, void* rho_out, void* rho_part) {
    StepIndex si{step_dev, step_host};
    if (s.lat == 0 && s.prec == 0) step_dispatch<0, float>(s, cfg, fin, fout, drho, si, partial, st, rho_out, rho_part);
    else if (s.lat == 0) step_dispatch<0, double>(s, cfg, fin, fout, drho, si, partial, st, rho_out, rho_part);
    else if (s.prec == 0) step_dispatch<1, float>(s, cfg, fin, fout, drho, si, partial, st, rho_out, rho_part);
    else step_dispatch<1, double>(s, cfg, fin, fout, drho, si, partial, st, rho_out, rho_part);
    return hipGetLastError();
}

// All Q mode densities of fin after streaming, in FP64: out[a V + s] =
// sum_i T_ai df_i(s) (shifted populations, so row 0 is rho - rho0), with the
// momentum rows replaced by rho u = j + F/2.
template <int LAT, typename Real, bool FORCE, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX* TY* TZ) void k_mode_fields(const Real* __restrict__ fin,
                                                             const Real* __restrict__ drho,
                                                             double* __restrict__ out, Geom g,
                                                             Real rho0, ForceParams<Real> fp) {
    using L = Lattice<LAT>;
    using FT = ForceTile<LAT, Real, TX, TY, TZ>;
    constexpr int Q = L::Q, D = L::D;
    constexpr int LDS_F = FORCE ? (FT::NR + FT::NM) : 1;
    __shared__ Real lds_force[LDS_F];
    int x0, y0, z0;
    tile_origin<LAT, TX, TY, TZ>(g, x0, y0, z0);
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    const bool inside = x < g.nx && y < g.ny && z < g.nz;
    Real F[D];
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] = Real(0);
    if constexpr (FORCE) {
        FT::stage(drho, g, fp, x0, y0, z0, lds_force, lds_force + FT::NR);
        if (inside) FT::force(lds_force, lds_force + FT::NR, fp, rho0, tx, ty, tz, F);
    }
    if (!inside) return;
    Real f[Q];
    pull<LAT, Real>(fin, x, y, z, g, f);
    const uint32_t s = site_index<LAT>(x, y, z, g);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        double m = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (L::T[a][i] != 0) m += (double)L::T[a][i] * (double)f[i];
        }
        if (a >= 1 && a <= D) m += 0.5 * (double)F[a - 1];
        out[(size_t)a * g.V + s] = m;
    }
}

template <int LAT, typename Real, bool FORCE>
static void fields_launch(const StepSpec& s, const void* fin, const void* drho, void* out,
                          hipStream_t st) {
    constexpr int TX = (LAT == 1) ? 32 : 64, TY = 4, TZ = (LAT == 1) ? 2 : 1;
    const Geom g = make_geom(s, TileShape{TX, TY, TZ, 1, 0, 0, 0});
    hipLaunchKernelGGL((k_fields<LAT, Real, FORCE, TX, TY, TZ>), dim3(g.nblocks),
                       dim3(TX * TY * TZ), 0, st, (const Real*)fin, (const Real*)drho, (Real*)out,
                       g, (Real)s.rho0, force_params<Real>(s));
}

hipError_t launch_fields(const StepSpec& s, const void* fin, const void* drho, void* out,
                         hipStream_t st) {
    if (s.lat == 0 && s.prec == 0) {
        if (s.force) fields_launch<0, float, true>(s, fin, drho, out, st);
        else fields_launch<0, float, false>(s, fin, drho, out, st);
    } else if (s.lat == 0) {
        if (s.force) fields_launch<0, double, true>(s, fin, drho, out, st);
        else fields_launch<0, double, false>(s, fin, drho, out, st);
    } else if (s.prec == 0) {
        if (s.force) fields_launch<1, float, true>(s, fin, drho, out, st);
        else fields_launch<1, float, false>(s, fin, drho, out, st);
    } else {
        if (s.force) fields_launch<1, double, true>(s, fin, drho, out, st);
        else fields_launch<1, double, false>(s, fin, drho, out, st);
    }
    return hipGetLastError();
}

template <int LAT, typename Real, bool FORCE>
static void mode_fields_launch(const StepSpec& s, const void* fin, const void* drho, double* out,
                               hipStream_t st) {
    constexpr int TX = (LAT == 1) ? 32 : 64, TY = 4, TZ = (LAT == 1) ? 2 : 1;
    const Geom g = make_geom(s, TileShape{TX, TY, TZ, 1, 0, 0, 0});
    hipLaunchKernelGGL((k_mode_fields<LAT, Real, FORCE, TX, TY, TZ>), dim3(g.nblocks),
                       dim3(TX * TY * TZ), 0, st, (const Real*)fin, (const Real*)drho, out, g,
                       (Real)s.rho0, force_params<Real>(s));
}

hipError_t launch_mode_fields(const StepSpec& s, const void* fin, const void* drho, double* out,
                              hipStream_t st) {
    if (s.lat == 0 && s.prec == 0) {
        if (s.force) mode_fields_launch<0, float, true>(s, fin, drho, out, st);
        else mode_fields_launch<0, float, false>(s, fin, drho, out, st);
    } else if (s.lat == 0) {
        if (s.force) mode_fields_launch<0, double, true>(s, fin, drho, out, st);
        else mode_fields_launch<0, double, false>(s, fin, drho, out, st);
    } else if (s.prec == 0) {
        if (s.force) mode_fields_launch<1, float, true>(s, fin, drho, out, st);
        else mode_fields_launch<1, float, false>(s, fin, drho, out, st);
    } else {
        if (s.force) mode_fields_launch<1, double, true>(s, fin, drho, out, st);
        else mode_fields_launch<1, double, false>(s, fin, drho, out, st);
    }
    return hipGetLastError();
}

hipError_t launch_stats_finalize(const double* partial, uint32_t nslots, int nvals, double* out,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_stats_finalize, dim3(nvals), dim3(256), 0, st, partial, nslots, nvals,
                       out);
    return hipGetLastError();
}

hipError_t launch_noise_words(const StepSpec& s, unsigned long long step, uint32_t block,
                              uint32_t tag, unsigned long long site0, unsigned long long nsites,
                              uint32_t* out, hipStream_t st) {
    if (nsites == 0) return hipSuccess;
    const dim3 grid((unsigned)((nsites + 255) / 256)), blk(256);
    hipLaunchKernelGGL(k_noise_words, grid, blk, 0, st, site0, nsites, (uint32_t)step,
                       block | (tag << 16), s.replica, s.key0, s.key1, out);
    return hipGetLastError();
}

hipError_t launch_noise_normals(const StepSpec& s, unsigned long long step,
                                unsigned long long site0, unsigned long long nsites, void* out,
                                hipStream_t st) {
    if (nsites == 0) return hipSuccess;
    const dim3 grid((unsigned)((nsites + 255) / 256)), blk(256);
    const uint32_t t = (uint32_t)step;
    if (s.lat == 0 && s.prec == 0)
        hipLaunchKernelGGL((k_noise_normals<Lattice<0>::NPAIR, float>), grid, blk, 0, st, site0, nsites, t, s.replica, s.key0, s.key1, (float*)out);
    else if (s.lat == 0)
        hipLaunchKernelGGL((k_noise_normals<Lattice<0>::NPAIR, double>), grid, blk, 0, st, site0, nsites, t, s.replica, s.key0, s.key1, (double*)out);
    else if (s.prec == 0)
        hipLaunchKernelGGL((k_noise_normals<Lattice<1>::NPAIR, float>), grid, blk, 0, st, site0, nsites, t, s.replica, s.key0, s.key1, (float*)out);
    else
        hipLaunchKernelGGL((k_noise_normals<Lattice<1>::NPAIR, double>), grid, blk, 0, st, site0, nsites, t, s.replica, s.key0, s.key1, (double*)out);
    return hipGetLastError();
}

hipError_t launch_add_u64(unsigned long long* ctr, unsigned long long inc, hipStream_t st) {
    hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(64), 0, st, ctr, inc);
    return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long* ctr, unsigned long long v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, st, ctr, v);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (uint32_t*)p, n);
    return hipGetLastError();
}

}  // namespace flb
