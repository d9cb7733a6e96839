// Per-site collision of the fluctuating LB step in moment space (device side).
//
// Works on shifted populations delta f_i = f_i - w_i rho0.  Because
// sum_i T_ai w_i = N_a delta_a0, the moments of delta f equal those of f except
// m_0, which becomes delta rho = rho - rho0; the inverse transform maps the
// shifted moments back to shifted populations (Sec. III eqs. moments,
// moments-inv).
//
// The update is Sec. V eq. lbe-mom:
//   m*_a = m_a - lam_a (m_a - m^eq_a) + (1 - lam_a/2) m^F_a + sigma_a z_a,
// lam_a = 0 on rho and j (so rho* = rho and j* = j + F), with the equilibrium
// moments of Sec. III eq. feq (zero on ghosts for the w-weighted basis), the
// forcing moments {0, F, uF + Fu, 0} and u = (j + F/2)/rho (Sec. V
// eq. lbe-moments).  sigma_a^2 = rho kT N_a lam_a (2 - lam_a)/cs2 (Sec. V
// eq. noise-lbe), with rho the local density or rho0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"
#include "philox.h"

namespace flb {

constexpr int QMAX = 19;

// Physical parameters of the collision, uniform over a launch.
template <typename Real>
struct CollideParams {
    Real rho0;
    Real lam_bulk, lam_shear, lam_ghost;
    Real amp_cls[3];    // sqrt(kT lam (2 - lam) / cs2) of the bulk, shear and ghost rates
    int32_t noise_on;   // kT > 0
    int32_t noise_local;
    uint32_t key0, key1, replica;
    uint32_t* nonfinite;  // set to 1 when a site's pulled density is not finite (nullable)
};

// sqrt(x) of a positive constant by Newton's iteration (compile time).
constexpr double const_sqrt(double x, double r = 1.0, int n = 0) {
    return n == 60 ? r : const_sqrt(x, 0.5 * (r + x / r), n + 1);
}

// sqrt(N_a) for every mode of a lattice, evaluated by the compiler.
template <int LAT>
struct ModeSqrtN {
    struct Tab {
        double v[Lattice<LAT>::Q];
    };
    static constexpr Tab make() {
        Tab t{};
        for (int a = 0; a < Lattice<LAT>::Q; ++a) t.v[a] = const_sqrt(Lattice<LAT>::N[a]);
        return t;
    }
    static constexpr Tab tab = make();
};

// Rate class of mode a for the class amplitudes: 0 bulk, 1 shear, 2 ghost.
template <int LAT>
__host__ __device__ constexpr int amp_class(int a) {
    return Lattice<LAT>::cls[a] == CLS_BULK ? 0 : (Lattice<LAT>::cls[a] == CLS_SHEAR ? 1 : 2);
}

// Noise amplitude of mode a: the per-mode variance rho kT N_a lam_a
// (2 - lam_a) / cs2 of Sec. V eq. noise-lbe is N_a times a rate-class factor,
// so sigma_a = sqrt(N_a) tc[class], tc = sqrt(rho) times the class
// amplitudes.  a is a constant of an unrolled loop.
template <int LAT, typename Real>
__host__ __device__ __forceinline__ Real mode_amp(const Real (&tc)[3], int a) {
    return tc[amp_class<LAT>(a)] * Real(ModeSqrtN<LAT>::tab.v[a]);
}

template <int LAT, typename Real>
struct Moments {
    using L = Lattice<LAT>;
    static constexpr int Q = L::Q;
    static constexpr int NP = L::NP;

    // m_a = sum_i T_ai f_i via opposite-pair sums and differences.
    static __host__ __device__ __forceinline__ void forward(const Real (&f)[Q], Real (&m)[Q]) {
        if constexpr (LAT == 1) {
            forward19(f, m);
            return;
        }
        Real s[NP], d[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            s[p] = f[L::pair[p][0]] + f[L::pair[p][1]];
            d[p] = f[L::pair[p][0]] - f[L::pair[p][1]];
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            Real acc = Real(0);
            if (!L::odd[a] && L::T[a][0] != 0) acc = Real(L::T[a][0]) * f[0];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int t = L::T[a][L::pair[p][0]];
                if (t == 0) continue;
                const Real v = L::odd[a] ? d[p] : s[p];
                if (t == 1) acc += v;
                else if (t == -1) acc -= v;
                else acc += Real(t) * v;
            }
            m[a] = acc;
        }
    }

    // f_i = w_i sum_a T_ai m_a / N_a, pairwise: f_i = w (E + O), f_ibar = w (E - O).
    static __host__ __device__ __forceinline__ void inverse(const Real (&m)[Q], Real (&f)[Q]) {
        if constexpr (LAT == 1) {
            inverse19(m, f);
            return;
        }
        Real mt[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) mt[a] = m[a] * Real(1.0 / L::N[a]);
        {
            Real acc = Real(0);
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const int t = L::T[a][0];
                if (t == 0) continue;
                if (t == 1) acc += mt[a];
                else if (t == -1) acc -= mt[a];
                else acc += Real(t) * mt[a];
            }
            f[0] = Real(L::w[0]) * acc;
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int i = L::pair[p][0], j = L::pair[p][1];
            Real E = Real(0), O = Real(0);
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const int t = L::T[a][i];
                if (t == 0) continue;
                if (L::odd[a]) {
                    if (t == 1) O += mt[a];
                    else if (t == -1) O -= mt[a];
                    else O += Real(t) * mt[a];
                } else {
                    if (t == 1) E += mt[a];
                    else if (t == -1) E -= mt[a];
                    else E += Real(t) * mt[a];
                }
            }
            f[i] = Real(L::w[i]) * (E + O);
            f[j] = Real(L::w[i]) * (E - O);
        }
    }

    // D3Q19 forward transform with the sub-sums shared between the rows of
    // the basis (same result as the table, fewer additions).  Pair sums s and
    // differences d: axes A*/a*, plane edges P (++ with --), M (+- with -+).
    static __host__ __device__ __forceinline__ void forward19(const Real (&f)[Q], Real (&m)[Q]) {
        const Real Ax = f[1] + f[2], ax = f[1] - f[2];
        const Real Ay = f[3] + f[4], ay = f[3] - f[4];
        const Real Az = f[5] + f[6], az = f[5] - f[6];
        const Real Pxy = f[7] + f[10], dPxy = f[7] - f[10];
        const Real Mxy = f[8] + f[9], dMxy = f[8] - f[9];
        const Real Pxz = f[11] + f[14], dPxz = f[11] - f[14];
        const Real Mxz = f[12] + f[13], dMxz = f[12] - f[13];
        const Real Pyz = f[15] + f[18], dPyz = f[15] - f[18];
        const Real Myz = f[16] + f[17], dMyz = f[16] - f[17];
        // even rows
        const Real Exy = Pxy + Mxy, Exz = Pxz + Mxz, Eyz = Pyz + Myz;
        const Real A = Ax + (Ay + Az);
        const Real E = Exy + Exz + Eyz;
        m[0] = f[0] + A + E;                               // 1
        m[4] = E - f[0];                                   // c^2 - 1
        m[16] = f[0] + E - Real(2) * A;                    // 3c^4 - 6c^2 + 1
        const Real a5 = Real(2) * Ax - (Ay + Az);
        const Real a6 = Ay - Az;
        const Real B = (Exy + Exz) - Real(2) * Eyz;
        const Real Cc = Exy - Exz;
        m[5] = B + a5;                                     // 3cx^2 - c^2
        m[17] = B - a5;                                    // (2c^2 - 3)(3cx^2 - c^2)
        m[6] = Cc + a6;                                    // cy^2 - cz^2
        m[18] = Cc - a6;                                   // (2c^2 - 3)(cy^2 - cz^2)
        m[7] = Pxy - Mxy;                                  // cx cy
        m[8] = Pyz - Myz;                                  // cy cz
        m[9] = Pxz - Mxz;                                  // cz cx
        // odd rows
        const Real X1 = dPxy + dMxy, X2 = dPxz + dMxz;     // cx-odd edge parts
        const Real Y1 = dPxy - dMxy, Y2 = dPyz + dMyz;     // cy-odd edge parts
        const Real Z1 = dPxz - dMxz, Z2 = dPyz - dMyz;     // cz-odd edge parts
        const Real SX = X1 + X2, SY = Y1 + Y2, SZ = Z1 + Z2;
        m[1] = ax + SX;                                    // cx
        m[2] = ay + SY;
        m[3] = az + SZ;
        m[10] = SX - Real(2) * ax;                         // (3c^2 - 5) cx
        m[11] = SY - Real(2) * ay;
        m[12] = SZ - Real(2) * az;
        m[13] = X1 - X2;                                   // (cy^2 - cz^2) cx
        m[14] = Y2 - Y1;                                   // (cz^2 - cx^2) cy
        m[15] = Z1 - Z2;                                   // (cx^2 - cy^2) cz
    }

    // D3Q19 inverse f_i = w_i sum_a T_ai m_a / N_a with shared sub-sums: for
    // every opposite pair the even-row part E and odd-row part O, then
    // f_i = w (E + O), f_ibar = w (E - O).
    static __host__ __device__ __forceinline__ void inverse19(const Real (&m)[Q], Real (&f)[Q]) {
        Real t[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) t[a] = m[a] * Real(1.0 / L::N[a]);
        const Real G = t[0] - Real(2) * t[16];
        const Real H = t[17] - t[5];
        const Real K = t[6] - t[18];
        f[0] = Real(L::w[0]) * (t[0] - t[4] + t[16]);
        const Real Ex = G - Real(2) * H;
        const Real Ey = G + H + K;
        const Real Ez = G + H - K;
        const Real Ox = t[1] - Real(2) * t[10];
        const Real Oy = t[2] - Real(2) * t[11];
        const Real Oz = t[3] - Real(2) * t[12];
        const Real wa = Real(L::w[1]);
        f[1] = wa * (Ex + Ox);
        f[2] = wa * (Ex - Ox);
        f[3] = wa * (Ey + Oy);
        f[4] = wa * (Ey - Oy);
        f[5] = wa * (Ez + Oz);
        f[6] = wa * (Ez - Oz);
        const Real Ec = t[0] + t[4] + t[16];
        const Real U = t[5] + t[17], W = t[6] + t[18];
        const Real EcU = Ec + U;
        const Real Bxy = EcU + W, Bxz = EcU - W, Byz = Ec - Real(2) * U;
        const Real Sx = t[1] + t[10], Sy = t[2] + t[11], Sz = t[3] + t[12];
        const Real we = Real(L::w[7]);
        // xy plane: 7 (+,+) / 10 (-,-), 8 (+,-) / 9 (-,+)
        {
            const Real E7 = Bxy + t[7], E8 = Bxy - t[7];
            const Real O7 = (Sx + Sy) + (t[13] - t[14]);
            const Real O8 = (Sx - Sy) + (t[13] + t[14]);
            f[7] = we * (E7 + O7);
            f[10] = we * (E7 - O7);
            f[8] = we * (E8 + O8);
            f[9] = we * (E8 - O8);
        }
        // xz plane: 11 (+,+) / 14, 12 (+,-) / 13
        {
            const Real E11 = Bxz + t[9], E12 = Bxz - t[9];
            const Real O11 = (Sx + Sz) + (t[15] - t[13]);
            const Real O12 = (Sx - Sz) - (t[13] + t[15]);
            f[11] = we * (E11 + O11);
            f[14] = we * (E11 - O11);
            f[12] = we * (E12 + O12);
            f[13] = we * (E12 - O12);
        }
        // yz plane: 15 (+,+) / 18, 16 (+,-) / 17
        {
            const Real E15 = Byz + t[8], E16 = Byz - t[8];
            const Real O15 = (Sy + Sz) + (t[14] - t[15]);
            const Real O16 = (Sy - Sz) + (t[14] + t[15]);
            f[15] = we * (E15 + O15);
            f[18] = we * (E15 - O15);
            f[16] = we * (E16 + O16);
            f[17] = we * (E16 - O16);
        }
    }

    // g_i = sum_a T_ai h_a (transpose of the forward transform), pairwise.
    static __host__ __device__ __forceinline__ void transpose(const Real (&h)[Q], Real (&g)[Q]) {
        {
            Real acc = Real(0);
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const int t = L::T[a][0];
                if (t == 0) continue;
                if (t == 1) acc += h[a];
                else if (t == -1) acc -= h[a];
                else acc += Real(t) * h[a];
            }
            g[0] = acc;
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int i = L::pair[p][0], j = L::pair[p][1];
            Real E = Real(0), O = Real(0);
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const int t = L::T[a][i];
                if (t == 0) continue;
                Real& acc = L::odd[a] ? O : E;
                if (t == 1) acc += h[a];
                else if (t == -1) acc -= h[a];
                else acc += Real(t) * h[a];
            }
            g[i] = E + O;
            g[j] = E - O;
        }
    }
};

// Equilibrium (m^eq) and forcing (m^F) moments of the stress modes.
// Row a = sum Gamma_ab c_a c_b + gamma gives m^eq = Gamma:(rho cs2 I + rho u u) + gamma rho
// and m^F = Gamma:(uF + Fu).
template <int LAT, typename Real> struct Stress;

template <typename Real> struct Stress<0, Real> {
    static constexpr int first = 3, count = 3;
    static __device__ __forceinline__ void eval(Real rho, const Real (&u)[2], const Real (&F)[2],
                                                Real (&meq)[3], Real (&mF)[3]) {
        const Real uxx = u[0] * u[0], uyy = u[1] * u[1];
        meq[0] = Real(3) * rho * (uxx + uyy);          // e = 3c^2 - 2
        meq[1] = rho * (uxx - uyy);                    // p_ww = c_x^2 - c_y^2
        meq[2] = rho * u[0] * u[1];                    // p_xy = c_x c_y
        const Real fxx = u[0] * F[0], fyy = u[1] * F[1];
        mF[0] = Real(6) * (fxx + fyy);
        mF[1] = Real(2) * (fxx - fyy);
        mF[2] = u[0] * F[1] + u[1] * F[0];
    }
};

template <typename Real> struct Stress<1, Real> {
    static constexpr int first = 4, count = 6;
    static __device__ __forceinline__ void eval(Real rho, const Real (&u)[3], const Real (&F)[3],
                                                Real (&meq)[6], Real (&mF)[6]) {
        const Real uxx = u[0] * u[0], uyy = u[1] * u[1], uzz = u[2] * u[2];
        const Real usq = uxx + uyy + uzz;
        meq[0] = rho * usq;                            // c^2 - 1
        meq[1] = rho * (Real(3) * uxx - usq);          // 3c_x^2 - c^2
        meq[2] = rho * (uyy - uzz);                    // c_y^2 - c_z^2
        meq[3] = rho * u[0] * u[1];                    // c_x c_y
        meq[4] = rho * u[1] * u[2];                    // c_y c_z
        meq[5] = rho * u[2] * u[0];                    // c_z c_x
        const Real fxx = u[0] * F[0], fyy = u[1] * F[1], fzz = u[2] * F[2];
        const Real uF = fxx + fyy + fzz;
        mF[0] = Real(2) * uF;
        mF[1] = Real(2) * (Real(3) * fxx - uF);
        mF[2] = Real(2) * (fyy - fzz);
        mF[3] = u[0] * F[1] + u[1] * F[0];
        mF[4] = u[1] * F[2] + u[2] * F[1];
        mF[5] = u[2] * F[0] + u[0] * F[2];
    }
};

// Reverse mode of Stress::eval.  Every stress row has m^eq_k = rho u.G_k u and
// m^F_k = 2 u.G_k F for a symmetric 3x3 (2x2) matrix G_k, so given the adjoints
// meq_b, mF_b this adds d/d rho, d/d u and d/d F.
template <int LAT, typename Real> struct StressAdj;

template <typename Real> struct StressAdj<0, Real> {
    static __device__ __forceinline__ void apply(Real rho, const Real (&u)[2], const Real (&F)[2],
                                                 const Real (&meq)[3], const Real (&meq_b)[3],
                                                 const Real (&mF_b)[3], Real& rho_b,
                                                 Real (&u_b)[2], Real (&F_b)[2]) {
        // G_0 = 3 I, G_1 = diag(1, -1), G_2 = offdiag(1/2)
        const Real Gu[3][2] = {{Real(3) * u[0], Real(3) * u[1]}, {u[0], -u[1]},
                               {Real(0.5) * u[1], Real(0.5) * u[0]}};
        const Real GF[3][2] = {{Real(3) * F[0], Real(3) * F[1]}, {F[0], -F[1]},
                               {Real(0.5) * F[1], Real(0.5) * F[0]}};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            rho_b += meq_b[k] * meq[k] / rho;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                u_b[a] += Real(2) * (rho * meq_b[k] * Gu[k][a] + mF_b[k] * GF[k][a]);
                F_b[a] += Real(2) * mF_b[k] * Gu[k][a];
            }
        }
    }
};

template <typename Real> struct StressAdj<1, Real> {
    static __device__ __forceinline__ void apply(Real rho, const Real (&u)[3], const Real (&F)[3],
                                                 const Real (&meq)[6], const Real (&meq_b)[6],
                                                 const Real (&mF_b)[6], Real& rho_b,
                                                 Real (&u_b)[3], Real (&F_b)[3]) {
        // G_0 = I, G_1 = diag(2,-1,-1), G_2 = diag(0,1,-1), G_3..5 = offdiag(1/2) xy, yz, zx
        const Real h = Real(0.5);
        const Real Gu[6][3] = {{u[0], u[1], u[2]},          {Real(2) * u[0], -u[1], -u[2]},
                               {Real(0), u[1], -u[2]},      {h * u[1], h * u[0], Real(0)},
                               {Real(0), h * u[2], h * u[1]}, {h * u[2], Real(0), h * u[0]}};
        const Real GF[6][3] = {{F[0], F[1], F[2]},          {Real(2) * F[0], -F[1], -F[2]},
                               {Real(0), F[1], -F[2]},      {h * F[1], h * F[0], Real(0)},
                               {Real(0), h * F[2], h * F[1]}, {h * F[2], Real(0), h * F[0]}};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            rho_b += meq_b[k] * meq[k] / rho;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u_b[a] += Real(2) * (rho * meq_b[k] * Gu[k][a] + mF_b[k] * GF[k][a]);
                F_b[a] += Real(2) * mF_b[k] * Gu[k][a];
            }
        }
    }
};

// Collide the moments of one site in place.  m[0] is delta rho on entry and
// exit; F is the force density (zero for the ideal gas); z the site's normals.
template <int LAT, typename Real, bool FORCE>
__device__ __forceinline__ void collide_moments(Real (&m)[Lattice<LAT>::Q],
                                                const Real (&F)[Lattice<LAT>::D],
                                                const Real* z, const CollideParams<Real>& P) {
    using L = Lattice<LAT>;
    using S = Stress<LAT, Real>;
    constexpr int D = L::D;
    // every population of the site enters m_0, so a NaN or Inf pulled into
    // the site shows here (a plain vector store of the same value from any
    // number of lanes)
    if (P.nonfinite && !__builtin_isfinite(m[0])) *P.nonfinite = 1u;
    const Real rho = P.rho0 + m[0];
    const Real inv_rho = Real(1) / rho;
    Real u[D];
#pragma unroll
    for (int a = 0; a < D; ++a) u[a] = (FORCE ? (m[1 + a] + Real(0.5) * F[a]) : m[1 + a]) * inv_rho;
    Real meq[S::count], mF[S::count];
    S::eval(rho, u, F, meq, mF);
    // conserved: rho unchanged, j* = j + F
    if (FORCE) {
#pragma unroll
        for (int a = 0; a < D; ++a) m[1 + a] += F[a];
    }
    // stress modes
#pragma unroll
    for (int k = 0; k < S::count; ++k) {
        const int a = S::first + k;
        const Real lam = (L::cls[a] == CLS_BULK) ? P.lam_bulk : P.lam_shear;
        Real v = m[a] - lam * (m[a] - meq[k]);
        if (FORCE) v += (Real(1) - Real(0.5) * lam) * mF[k];
        m[a] = v;
    }
    // ghost modes: m^eq = m^F = 0
#pragma unroll
    for (int a = S::first + S::count; a < L::Q; ++a) m[a] = m[a] - P.lam_ghost * m[a];
    if (P.noise_on) {
        const Real sr = P.noise_local ? sqrt(rho) : sqrt(P.rho0);
        const Real tc[3] = {sr * P.amp_cls[0], sr * P.amp_cls[1], sr * P.amp_cls[2]};
#pragma unroll
        for (int k = 0; k < L::K; ++k) m[D + 1 + k] += mode_amp<LAT, Real>(tc, D + 1 + k) * z[k];
    }
}

}  // namespace flb
