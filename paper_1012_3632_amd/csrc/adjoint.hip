// Adjoint (reverse-mode) kernels of the fluctuating LB step.
//
// Given abar_{n+1} = dL/dS_{n+1} and the state S_n, they produce
// abar_n = dL/dS_n and the derivatives of the step w.r.t. the relaxation rates
// and kT, with the noise of step n regenerated from the same Philox counters.
// The forward step is S_{n+1} = Tinv C(T P S_n, F), with P the pull, T the
// moment transform (Sec. III eq. moments), C the moment-space update of
// Sec. V eq. lbe-mom and, for the square-gradient fluid, the force
// F = -rho grad_h mu + eta grad_h rho built from rho = sum_i (P S_n)_i
// (App. A eq. he-force).  Reverse mode, per site x:
//   mbar*  = N^-1 T (w . abar_{n+1})              (transpose of Tinv)
//   mbar, Fbar  = C^T(mbar*)                      (collision Jacobian, incl. u = (j + F/2)/rho,
//                                                  m^eq, m^F and sigma_a ~ sqrt(rho))
//   fbar_i = sum_a T_ai mbar_a                    (transpose of T)
//   abar_n,i(x - c_i) = fbar_i(x)                 (transpose of the pull: a conflict-free push)
// and, for the force, rhobar = (dF/drho)^T Fbar through the stencil transposes
//   mubar = -grad_h^T (rho Fbar),  rhobar = -Fbar.grad_h mu + eta cs2 grad_h^T Fbar
//                                            + psi''(rho) mubar - kappa lap_h mubar
// (grad_h^T phi(y) = 3 sum_i w_i c_i phi(y - c_i); lap_h is self-adjoint), added
// to every population of the site: abar_n,i(y) += rhobar(y + c_i).  In a
// reverse sweep that last spread is deferred: the next (earlier) step's
// collision adjoint adds rhobar(y + c_i) as it reads abar, which saves a pass.
// For the D2Q9 force that rhobar is not stored either: the collision adjoint
// forms it on its tile plus a one-site halo from the later step's Fbar and
// density, staged in LDS, so a reverse step is a single launch.
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"

namespace flb {

// Reverse mode of collide_moments at one site.  m: pre-collision moments
// (m_0 = delta rho), F: force, z: normals, mbs: dL/dm*.  Outputs mb = dL/dm,
// Fb = dL/dF and adds the parameter derivatives to pg (shear, kT, bulk, ghost).
template <int LAT, typename Real, bool FORCE>
__device__ __forceinline__ void collide_adjoint(const Real (&m)[Lattice<LAT>::Q],
                                                const Real (&F)[Lattice<LAT>::D], const Real* z,
                                                const CollideParams<Real>& P, Real inv2kT,
                                                const Real (&mbs)[Lattice<LAT>::Q],
                                                Real (&mb)[Lattice<LAT>::Q],
                                                Real (&Fb)[Lattice<LAT>::D], double (&pg)[4]) {
    using L = Lattice<LAT>;
    using S = Stress<LAT, Real>;
    constexpr int D = L::D, Q = L::Q;
    const Real rho = P.rho0 + m[0];
    const Real inv_rho = Real(1) / rho;
    Real u[D];
#pragma unroll
    for (int a = 0; a < D; ++a) u[a] = (FORCE ? (m[1 + a] + Real(0.5) * F[a]) : m[1 + a]) * inv_rho;
    Real meq[S::count], mF[S::count];
    S::eval(rho, u, F, meq, mF);
    const Real sr = P.noise_local ? sqrt(rho) : sqrt(P.rho0);
    const Real tc[3] = {sr * P.amp_cls[0], sr * P.amp_cls[1], sr * P.amp_cls[2]};
    Real rho_b = Real(0), u_b[D];
    mb[0] = mbs[0];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        u_b[a] = Real(0);
        mb[1 + a] = mbs[1 + a];
        Fb[a] = FORCE ? mbs[1 + a] : Real(0);   // j* = j + F
    }
    Real meq_b[S::count], mF_b[S::count];
#pragma unroll
    for (int k = 0; k < S::count; ++k) {
        const int a = S::first + k;
        const bool bulk = L::cls[a] == CLS_BULK;
        const Real lam = bulk ? P.lam_bulk : P.lam_shear;
        const Real gb = mbs[a];
        mb[a] = (Real(1) - lam) * gb;
        meq_b[k] = lam * gb;
        mF_b[k] = FORCE ? (Real(1) - Real(0.5) * lam) * gb : Real(0);
        Real g = meq[k] - m[a];
        if (FORCE) g -= Real(0.5) * mF[k];
        g *= gb;
        if (P.noise_on) {
            const int kk = a - D - 1;
            const Real sz = mode_amp<LAT, Real>(tc, a) * z[kk] * gb;
            g += sz * (Real(1) - lam) / (lam * (Real(2) - lam));
            pg[1] += (double)(sz * inv2kT);
            if (P.noise_local) rho_b += Real(0.5) * sz * inv_rho;
        }
        pg[bulk ? 2 : 0] += (double)g;
    }
#pragma unroll
    for (int a = S::first + S::count; a < Q; ++a) {
        const Real lam = P.lam_ghost;
        const Real gb = mbs[a];
        mb[a] = (Real(1) - lam) * gb;
        Real g = -m[a] * gb;
        if (P.noise_on) {
            const int kk = a - D - 1;
            const Real sz = mode_amp<LAT, Real>(tc, a) * z[kk] * gb;
            g += sz * (Real(1) - lam) / (lam * (Real(2) - lam));
            pg[1] += (double)(sz * inv2kT);
            if (P.noise_local) rho_b += Real(0.5) * sz * inv_rho;
        }
        pg[3] += (double)g;
    }
    StressAdj<LAT, Real>::apply(rho, u, F, meq, meq_b, mF_b, rho_b, u_b, Fb);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        mb[1 + a] += u_b[a] * inv_rho;
        if (FORCE) Fb[a] += Real(0.5) * u_b[a] * inv_rho;
        rho_b -= u_b[a] * u[a] * inv_rho;
    }
    mb[0] += rho_b;
}

// The density adjoint of the force on a tile (P2's arithmetic, shared by
// k_adj_force and the fused collision adjoint).  With rs, ms the density and
// mu staged by ForceTile<TX, TY, TZ>::stage (tile plus halos 2 and 1) and fbs
// the force adjoint staged on the same region as rs:
//   mubar(y) = -3 sum_i w_i c_i . (rho Fbar)(y - c_i)  on the tile plus halo 1,
//   rhobar   = -Fbar . 3 grad_h mu + eta grad_h^T Fbar + psi''(rho) mubar - kappa lap_h mubar.
template <int LAT, typename Real, int TX, int TY, int TZ>
struct ForceAdjointTile {
    using L = Lattice<LAT>;
    using FT = ForceTile<LAT, Real, TX, TY, TZ>;
    static constexpr int Q = L::Q, D = L::D, HZ = FT::HZ;
    static constexpr int RX = FT::RX, RY = FT::RY, NR = FT::NR, MX = FT::MX, MY = FT::MY,
                         NM = FT::NM;

    // fbs[a NR + l] = Fbar_a at the staged site l (tile origin x0, y0, z0)
    static __device__ __forceinline__ void load_fbar(const Real* __restrict__ Fbar, const Geom& g,
                                                     int x0, int y0, int z0, Real* fbs,
                                                     int nthreads) {
        for (int l = threadIdx.x; l < NR; l += nthreads) {
            const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
            const int gx = wrap_any(x0 + lx - 2, g.nx);
            const int gy = wrap_any(y0 + ly - 2, g.ny);
            const int gz = wrap_any(z0 + lz - 2 * HZ, g.nz);
            const uint32_t s = (uint32_t)((gz * g.ny + gy) * g.nx + gx);
#pragma unroll
            for (int a = 0; a < D; ++a) fbs[a * NR + l] = Fbar[(size_t)a * g.V + s];
        }
    }

    static __device__ __forceinline__ void mubar(const Real* rs, const Real* fbs, Real* mubs,
                                                 Real rho0, int nthreads) {
        for (int l = threadIdx.x; l < NM; l += nthreads) {
            const int mx = l % MX, my = (l / MX) % MY, mz = l / (MX * MY);
            const int c = ((mz + HZ) * RY + (my + 1)) * RX + (mx + 1);
            Real acc = Real(0);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int n = c - (L::cz[i] * RY + L::cy[i]) * RX - L::cx[i];
                const Real rn = rho0 + rs[n];
                const int c3[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    if (c3[a] == 0) continue;
                    acc += Real(L::w[i] * c3[a]) * rn * fbs[a * NR + n];
                }
            }
            mubs[l] = Real(-3) * acc;
        }
    }

    // rhobar at tile-local site (tx, ty, tz)
    static __device__ __forceinline__ Real rhobar(const Real* rs, const Real* ms, const Real* fbs,
                                                  const Real* mubs, const ForceParams<Real>& fp,
                                                  int tx, int ty, int tz) {
        const int cm = ((tz + HZ) * MY + (ty + 1)) * MX + (tx + 1);
        const int cr = ((tz + 2 * HZ) * RY + (ty + 2)) * RX + (tx + 2);
        Real gmu[D], eterm = Real(0), lap = Real(0);
#pragma unroll
        for (int a = 0; a < D; ++a) gmu[a] = Real(0);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int om = (L::cz[i] * MY + L::cy[i]) * MX + L::cx[i];
            const int orr = (L::cz[i] * RY + L::cy[i]) * RX + L::cx[i];
            lap += Real(L::w[i]) * (mubs[cm + om] - mubs[cm]);
            const int c3[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
            for (int a = 0; a < D; ++a) {
                if (c3[a] == 0) continue;
                const Real wc = Real(L::w[i] * c3[a]);
                gmu[a] += wc * ms[cm + om];
                eterm += wc * fbs[a * NR + cr - orr];
            }
        }
        Real t1 = Real(0);
#pragma unroll
        for (int a = 0; a < D; ++a) t1 -= fbs[a * NR + cr] * Real(3) * gmu[a];
        const Real d = rs[cr] + fp.shift;
        const Real psi2 = Real(2) * fp.a + Real(12) * fp.b * d * d;
        // eta cs2 grad_h rho = eta sum_i w_i c_i rho(x + c_i): its transpose carries no factor 3
        return t1 + fp.eta * eterm + psi2 * mubs[cm] - fp.kappa * Real(6) * lap;
    }
};

// Collision adjoint + transposed transforms + push (P1).
// FUSE (D2Q9 force only): instead of reading the later step's rhobar (rb_prev),
// form it here on the tile plus one site from that step's force adjoint
// Fbar_next and density drho_next (the arithmetic of k_adj_force on a tile
// two sites wider), so the reverse sweep needs no separate P2 per step.
template <int LAT, typename Real, bool FORCE, int TX, int TY, int TZ, bool FUSE = false>
__global__ __launch_bounds__(TX* TY* TZ) void k_adj_collide(
    const Real* __restrict__ s_n, const Real* __restrict__ abar, const Real* __restrict__ rb_prev,
    Real* __restrict__ abar_out, const Real* __restrict__ drho, Real* __restrict__ Fbar, Geom g,
    CollideParams<Real> P, ForceParams<Real> fp, Real inv2kT, uint32_t step,
    double* __restrict__ gpartial, const Real* __restrict__ drho_next,
    const Real* __restrict__ Fbar_next) {
    using L = Lattice<LAT>;
    using M = Moments<LAT, Real>;
    using FT = ForceTile<LAT, Real, TX, TY, TZ>;
    using FA = ForceAdjointTile<LAT, Real, TX + 2, TY + 2, TZ>;
    constexpr int Q = L::Q, D = L::D, NT = TX * TY * TZ;
    static_assert(!FUSE || (FORCE && LAT == 0), "the fused sweep is the D2Q9 force path");
    constexpr int LDS_F = FORCE ? (FT::NR + FT::NM) : 1;
    constexpr int NRB = (TX + 2) * (TY + 2);
    constexpr int LDS_A = FUSE ? ((D + 1) * FA::NR + 2 * FA::NM + NRB) : 1;
    __shared__ Real lds_force[LDS_F];
    __shared__ Real lds_adj[LDS_A];
    __shared__ double lds_red[4 * ((NT + 63) / 64) * 4];

    int x0, y0, z0;
    tile_origin<LAT, TX, TY, TZ>(g, x0, y0, z0);
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    const bool inside = x < g.nx && y < g.ny && z < g.nz;
    const uint32_t site = (uint32_t)((z * g.ny + y) * g.nx + x);
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    // global loads first, so that their latency overlaps the force tile's
    Real f[Q], ab[Q];
    if (inside) {
        pull<LAT, Real>(s_n, x, y, z, g, f);
#pragma unroll
        for (int i = 0; i < Q; ++i) ab[i] = abar[(size_t)i * g.V + site];
        if (FORCE && !FUSE && rb_prev) {
            // the density adjoint of the later step not yet spread over the
            // populations: abar_i(y) += rhobar(y + c_i)
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int sx = L::cx[i] == 0 ? x : (L::cx[i] > 0 ? xp : xm);
                const int sy = L::cy[i] == 0 ? y : (L::cy[i] > 0 ? yp : ym);
                const int sz = L::cz[i] == 0 ? z : (L::cz[i] > 0 ? zp : zm);
                ab[i] += rb_prev[(uint32_t)((sz * g.ny + sy) * g.nx + sx)];
            }
        }
    }
    Real F[D];
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] = Real(0);
    if constexpr (FUSE) {
        // every staged field is requested at once: this step's density tile,
        // and the later step's Fbar and density on the tile two sites wider;
        // then the chemical potentials and mubar in one phase
        const bool next = Fbar_next != nullptr;   // uniform over the grid
        Real* rs2 = lds_adj;
        Real* fbs2 = rs2 + FA::NR;
        Real* ms2 = fbs2 + D * FA::NR;
        Real* mubs2 = ms2 + FA::NM;
        Real* rbs = mubs2 + FA::NM;
        FT::load_rho(drho, g, x0, y0, z0, lds_force, NT);
        if (next) {
            FA::load_fbar(Fbar_next, g, x0 - 1, y0 - 1, z0, fbs2, NT);
            FA::FT::load_rho(drho_next, g, x0 - 1, y0 - 1, z0, rs2, NT);
        }
        __syncthreads();
        if (next) {
            FA::FT::mu_rows(fp, rs2, ms2, NT);
            FA::mubar(rs2, fbs2, mubs2, P.rho0, NT);
        }
        FT::mu_from_rho(fp, lds_force, lds_force + FT::NR, NT);   // ends with a barrier
        if (next) {
            for (int l = threadIdx.x; l < NRB; l += NT)
                rbs[l] = FA::rhobar(rs2, ms2, fbs2, mubs2, fp, l % (TX + 2), l / (TX + 2), 0);
            __syncthreads();
            if (inside) {
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    ab[i] += rbs[(ty + 1 + L::cy[i]) * (TX + 2) + (tx + 1 + L::cx[i])];
            }
        }
        if (inside) FT::force(lds_force, lds_force + FT::NR, fp, P.rho0, tx, ty, tz, F);
    } else if constexpr (FORCE) {
        FT::stage(drho, g, fp, x0, y0, z0, lds_force, lds_force + FT::NR);
        if (inside) FT::force(lds_force, lds_force + FT::NR, fp, P.rho0, tx, ty, tz, F);
    }
    double pg[4] = {0.0, 0.0, 0.0, 0.0};
    if (inside) {
        Real m[Q];
        M::forward(f, m);
        Real zn[2 * L::NPAIR];
        if (P.noise_on) site_normals<L::NPAIR, Real>(site, step, 0u, P.replica, P.key0, P.key1, zn);
        Real mbs[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) ab[i] *= Real(L::w[i]);
        M::forward(ab, mbs);
#pragma unroll
        for (int a = 0; a < Q; ++a) mbs[a] *= Real(1.0 / L::N[a]);
        Real mb[Q], Fb[D];
        collide_adjoint<LAT, Real, FORCE>(m, F, zn, P, inv2kT, mbs, mb, Fb, pg);
        Real fb[Q];
        M::transpose(mb, fb);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int dx = L::cx[i] == 0 ? x : (L::cx[i] > 0 ? xm : xp);
            const int dy = L::cy[i] == 0 ? y : (L::cy[i] > 0 ? ym : yp);
            const int dz = L::cz[i] == 0 ? z : (L::cz[i] > 0 ? zm : zp);
            abar_out[(size_t)i * g.V + (uint32_t)((dz * g.ny + dy) * g.nx + dx)] = fb[i];
        }
        if constexpr (FORCE) {
#pragma unroll
            for (int a = 0; a < D; ++a) Fbar[(size_t)a * g.V + site] = Fb[a];
        }
    }
    const uint32_t b = xcd_remap(blockIdx.x, g.nblocks);
    block_accumulate<4, NT>(pg, gpartial + (size_t)b * 4, lds_red);
}

// Force adjoint through the stencils (P2): rhobar at every site.
template <int LAT, typename Real, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX* TY* TZ) void k_adj_force(const Real* __restrict__ drho,
                                                           const Real* __restrict__ Fbar,
                                                           Real* __restrict__ rhobar, Geom g,
                                                           Real rho0, ForceParams<Real> fp) {
    using FA = ForceAdjointTile<LAT, Real, TX, TY, TZ>;
    constexpr int D = FA::D, NT = TX * TY * TZ;
    __shared__ Real rs[FA::NR];
    __shared__ Real ms[FA::NM];
    __shared__ Real fbs[D * FA::NR];
    __shared__ Real mubs[FA::NM];
    int x0, y0, z0;
    tile_origin<LAT, TX, TY, TZ>(g, x0, y0, z0);
    FA::load_fbar(Fbar, g, x0, y0, z0, fbs, NT);
    FA::FT::stage(drho, g, fp, x0, y0, z0, rs, ms);   // synchronizes
    FA::mubar(rs, fbs, mubs, rho0, NT);
    __syncthreads();
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    rhobar[(uint32_t)((z * g.ny + y) * g.nx + x)] = FA::rhobar(rs, ms, fbs, mubs, fp, tx, ty, tz);
}

// out_i(y) (+)= r(y + c_i) for every population (P3 and the density seed).
template <int LAT, typename Real, bool ADD>
__global__ void k_adj_spread(const Real* __restrict__ r, Real* __restrict__ out, Geom g) {
    using L = Lattice<LAT>;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const int x = (int)(s % (uint32_t)g.nx);
    const uint32_t q = s / (uint32_t)g.nx;
    const int y = (int)(q % (uint32_t)g.ny), z = (int)(q / (uint32_t)g.ny);
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int sx = L::cx[i] == 0 ? x : (L::cx[i] > 0 ? xp : xm);
        const int sy = L::cy[i] == 0 ? y : (L::cy[i] > 0 ? yp : ym);
        const int sz = L::cz[i] == 0 ? z : (L::cz[i] > 0 ? zp : zm);
        const Real v = r[(uint32_t)((sz * g.ny + sy) * g.nx + sx)];
        if (ADD) out[(size_t)i * g.V + s] += v;
        else out[(size_t)i * g.V + s] = v;
    }
}

// ------------------------------------------------------------------ launchers

template <int LAT, bool FORCE> struct AdjTile;
template <> struct AdjTile<0, false> { static constexpr int X = 64, Y = 4, Z = 1; };
template <> struct AdjTile<1, false> { static constexpr int X = 64, Y = 4, Z = 1; };
template <> struct AdjTile<0, true> { static constexpr int X = 64, Y = 4, Z = 1; };
template <> struct AdjTile<1, true> { static constexpr int X = 16, Y = 4, Z = 2; };

static Geom adj_geom(const StepSpec& s, int tx, int ty, int tz) {
    Geom g{};
    g.nx = s.nx;
    g.ny = s.ny;
    g.nz = s.nz;
    g.nbx = (s.nx + tx - 1) / tx;
    g.nby = (s.ny + ty - 1) / ty;
    g.nbz = (s.nz + tz - 1) / tz;
    g.nblocks = (uint32_t)g.nbx * g.nby * g.nbz;
    g.V = (uint32_t)s.nx * s.ny * s.nz;
    return g;
}

template <typename Real>
static CollideParams<Real> adj_collide_params(const StepSpec& s) {
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
    P.nonfinite = nullptr;
    return P;
}

template <typename Real>
static ForceParams<Real> adj_force_params(const StepSpec& s) {
    ForceParams<Real> f;
    f.a = (Real)s.a;
    f.b = (Real)s.b;
    f.shift = (Real)(s.rho0 - s.rho_c);
    f.kappa = (Real)s.kappa;
    f.eta = (Real)s.eta;
    return f;
}

// Force adjoint work space.  D3Q19: D planes of Fbar, then two rhobar planes
// (a step of a reverse sweep reads the later step's rhobar while writing its
// own).  D2Q9 (fused sweep): two sets of D Fbar planes (a step reads the later
// step's Fbar while writing its own), then one rhobar plane for a spread at
// the end of a sweep or of a single step.
static bool adj_fused(const StepSpec& s) { return s.force && s.lat == 0; }

size_t adjoint_work_bytes(const StepSpec& s) {
    if (!s.force) return 0;
    const size_t rb = s.prec ? 8 : 4;
    const size_t D = s.lat == 1 ? 3 : 2;
    const size_t planes = adj_fused(s) ? 2 * D + 1 : D + 2;
    return planes * (size_t)s.nx * s.ny * s.nz * rb;
}

uint32_t adjoint_slots(const StepSpec& s) {
    if (s.lat == 1 && s.force)
        return adj_geom(s, AdjTile<1, true>::X, AdjTile<1, true>::Y, AdjTile<1, true>::Z).nblocks;
    if (s.lat == 0 && s.force)
        return adj_geom(s, AdjTile<0, true>::X, AdjTile<0, true>::Y, AdjTile<0, true>::Z).nblocks;
    return adj_geom(s, AdjTile<0, false>::X, AdjTile<0, false>::Y, AdjTile<0, false>::Z).nblocks;
}

template <int LAT, typename Real, bool FORCE>
static void adj_launch(const StepSpec& s, const AdjointStepArgs& a, hipStream_t st) {
    using T = AdjTile<LAT, FORCE>;
    constexpr int D = Lattice<LAT>::D;
    const Geom g = adj_geom(s, T::X, T::Y, T::Z);
    const CollideParams<Real> P = adj_collide_params<Real>(s);
    const ForceParams<Real> fp = adj_force_params<Real>(s);
    const Real inv2kT = s.kT > 0.0 ? (Real)(0.5 / s.kT) : Real(0);
    const dim3 grid(g.nblocks), block(T::X * T::Y * T::Z);
    Real* base = (Real*)a.work;
    if constexpr (FORCE && LAT == 0) {
        // fused sweep: Fbar sets alternate; the later step's rhobar is formed
        // inside the collision adjoint
        Real* Fb_out = base + (size_t)a.rb_out * D * g.V;
        const Real* Fb_next = a.rb_in >= 0 ? base + (size_t)a.rb_in * D * g.V : nullptr;
        hipLaunchKernelGGL((k_adj_collide<LAT, Real, true, T::X, T::Y, T::Z, true>), grid, block,
                           0, st, (const Real*)a.s_n, (const Real*)a.abar_np1, (const Real*)nullptr,
                           (Real*)a.abar_n, (const Real*)a.drho, Fb_out, g, P, fp, inv2kT,
                           (uint32_t)a.step, a.gpartial, (const Real*)a.drho_next, Fb_next);
        if (a.spread) {
            Real* rbar = base + (size_t)2 * D * g.V;
            hipLaunchKernelGGL((k_adj_force<LAT, Real, T::X, T::Y, T::Z>), grid, block, 0, st,
                               (const Real*)a.drho, (const Real*)Fb_out, rbar, g, (Real)s.rho0, fp);
            hipLaunchKernelGGL((k_adj_spread<LAT, Real, true>), dim3((g.V + 255) / 256), dim3(256),
                               0, st, (const Real*)rbar, (Real*)a.abar_n, g);
        }
        return;
    }
    Real* Fbar = base;
    Real* rb_in = (FORCE && a.rb_in >= 0) ? Fbar + (size_t)(D + a.rb_in) * g.V : nullptr;
    Real* rb_out = FORCE ? Fbar + (size_t)(D + a.rb_out) * g.V : nullptr;
    hipLaunchKernelGGL((k_adj_collide<LAT, Real, FORCE, T::X, T::Y, T::Z>), grid, block, 0, st,
                       (const Real*)a.s_n, (const Real*)a.abar_np1, (const Real*)rb_in,
                       (Real*)a.abar_n, (const Real*)a.drho, Fbar, g, P, fp, inv2kT,
                       (uint32_t)a.step, a.gpartial, (const Real*)nullptr, (const Real*)nullptr);
    if constexpr (FORCE) {
        hipLaunchKernelGGL((k_adj_force<LAT, Real, T::X, T::Y, T::Z>), grid, block, 0, st,
                           (const Real*)a.drho, (const Real*)Fbar, rb_out, g, (Real)s.rho0, fp);
        if (a.spread)
            hipLaunchKernelGGL((k_adj_spread<LAT, Real, true>), dim3((g.V + 255) / 256),
                               dim3(256), 0, st, (const Real*)rb_out, (Real*)a.abar_n, g);
    }
}

hipError_t launch_adjoint_step(const StepSpec& s, const AdjointStepArgs& a, hipStream_t st) {
    if (s.force && (a.rb_out < 0 || a.rb_out > 1 || a.rb_in > 1 || a.rb_in == a.rb_out))
        return hipErrorInvalidValue;
    if (adj_fused(s) && a.rb_in >= 0 && !a.drho_next) return hipErrorInvalidValue;
    if (s.lat == 0 && s.prec == 0) {
        if (s.force) adj_launch<0, float, true>(s, a, st);
        else adj_launch<0, float, false>(s, a, st);
    } else if (s.lat == 0) {
        if (s.force) adj_launch<0, double, true>(s, a, st);
        else adj_launch<0, double, false>(s, a, st);
    } else if (s.prec == 0) {
        if (s.force) adj_launch<1, float, true>(s, a, st);
        else adj_launch<1, float, false>(s, a, st);
    } else {
        if (s.force) adj_launch<1, double, true>(s, a, st);
        else adj_launch<1, double, false>(s, a, st);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_spread(const StepSpec& s, void* work, int rb, const void* drho,
                                 void* abar, hipStream_t st) {
    if (!s.force) return hipSuccess;
    if (rb < 0 || rb > 1) return hipErrorInvalidValue;
    const Geom g = adj_geom(s, 1, 1, 1);
    const dim3 grid((g.V + 255) / 256), blk(256);
    if (adj_fused(s)) {
        // rhobar of the last step of the sweep from its Fbar set, then spread
        if (!drho) return hipErrorInvalidValue;
        using T = AdjTile<0, true>;
        const Geom gt = adj_geom(s, T::X, T::Y, T::Z);
        const dim3 tg(gt.nblocks), tb(T::X * T::Y * T::Z);
        const size_t fb = (size_t)rb * 2 * g.V, rr = (size_t)4 * g.V;
        if (s.prec == 0) {
            float* w = (float*)work;
            hipLaunchKernelGGL((k_adj_force<0, float, T::X, T::Y, T::Z>), tg, tb, 0, st,
                               (const float*)drho, (const float*)(w + fb), w + rr, gt,
                               (float)s.rho0, adj_force_params<float>(s));
            hipLaunchKernelGGL((k_adj_spread<0, float, true>), grid, blk, 0, st,
                               (const float*)(w + rr), (float*)abar, g);
        } else {
            double* w = (double*)work;
            hipLaunchKernelGGL((k_adj_force<0, double, T::X, T::Y, T::Z>), tg, tb, 0, st,
                               (const double*)drho, (const double*)(w + fb), w + rr, gt, s.rho0,
                               adj_force_params<double>(s));
            hipLaunchKernelGGL((k_adj_spread<0, double, true>), grid, blk, 0, st,
                               (const double*)(w + rr), (double*)abar, g);
        }
        return hipGetLastError();
    }
    const size_t off = (size_t)((s.lat == 1 ? 3 : 2) + rb) * g.V;
    if (s.lat == 0 && s.prec == 0)
        hipLaunchKernelGGL((k_adj_spread<0, float, true>), grid, blk, 0, st, (const float*)work + off, (float*)abar, g);
    else if (s.lat == 0)
        hipLaunchKernelGGL((k_adj_spread<0, double, true>), grid, blk, 0, st, (const double*)work + off, (double*)abar, g);
    else if (s.prec == 0)
        hipLaunchKernelGGL((k_adj_spread<1, float, true>), grid, blk, 0, st, (const float*)work + off, (float*)abar, g);
    else
        hipLaunchKernelGGL((k_adj_spread<1, double, true>), grid, blk, 0, st, (const double*)work + off, (double*)abar, g);
    return hipGetLastError();
}

hipError_t launch_adjoint_seed(const StepSpec& s, const void* rhobar, void* abar, hipStream_t st) {
    const Geom g = adj_geom(s, 1, 1, 1);
    const dim3 grid((g.V + 255) / 256), blk(256);
    if (s.lat == 0 && s.prec == 0)
        hipLaunchKernelGGL((k_adj_spread<0, float, false>), grid, blk, 0, st, (const float*)rhobar, (float*)abar, g);
    else if (s.lat == 0)
        hipLaunchKernelGGL((k_adj_spread<0, double, false>), grid, blk, 0, st, (const double*)rhobar, (double*)abar, g);
    else if (s.prec == 0)
        hipLaunchKernelGGL((k_adj_spread<1, float, false>), grid, blk, 0, st, (const float*)rhobar, (float*)abar, g);
    else
        hipLaunchKernelGGL((k_adj_spread<1, double, false>), grid, blk, 0, st, (const double*)rhobar, (double*)abar, g);
    return hipGetLastError();
}

}  // namespace flb
