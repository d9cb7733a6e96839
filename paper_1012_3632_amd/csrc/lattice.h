// Constant tables of the D2Q9 and D3Q19 velocity sets and their w-orthogonal
// moment bases, written out as literals.
//
// D2Q9: velocities, weights, basis and norms of App. B (table tab:modes-d2q9,
// matrix eq. TD2Q9).  Mode order rho, j_x, j_y, e, p_ww, p_xy, q_x, q_y, eps.
//
// D3Q19: the paper cites bases from the literature without printing one, so a
// w-orthogonal basis is fixed here.  Velocity order
//   0 | +x -x +y -y +z -z | xy: ++ +- -+ -- | xz: ++ +- -+ -- | yz: ++ +- -+ --
// weights 1/3, 1/18, 1/36; rows (polynomials in c)
//   1 | c_x c_y c_z | c^2-1 | 3c_x^2-c^2, c_y^2-c_z^2, c_xc_y, c_yc_z, c_zc_x |
//   (3c^2-5)c_x, (3c^2-5)c_y, (3c^2-5)c_z |
//   (c_y^2-c_z^2)c_x, (c_z^2-c_x^2)c_y, (c_x^2-c_y^2)c_z |
//   3c^4-6c^2+1 | (2c^2-3)(3c_x^2-c^2) | (2c^2-3)(c_y^2-c_z^2)
// with norms N_a = sum_i w_i T_ai^2 (Sec. III eq. T-orthog).
//
// Every row is a polynomial of definite parity in c, so with opposite
// velocities (i, ibar) the transform splits into sums s = f_i + f_ibar (even
// rows) and differences d = f_i - f_ibar (odd rows).
#pragma once

namespace flb {

enum ModeClass { CLS_RHO = 0, CLS_MOM = 1, CLS_BULK = 2, CLS_SHEAR = 3, CLS_GHOST = 4 };

template <int LAT> struct Lattice;

// ---------------------------------------------------------------- D2Q9
template <> struct Lattice<0> {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr int NP = 4;          // opposite pairs
    static constexpr int K = 6;           // non-conserved modes
    static constexpr int NPAIR = 3;       // Box-Muller pairs per site-step (K normals)
    static constexpr int cx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr int T[Q][Q] = {
        {1, 1, 1, 1, 1, 1, 1, 1, 1},
        {0, 1, 0, -1, 0, 1, -1, -1, 1},
        {0, 0, 1, 0, -1, 1, 1, -1, -1},
        {-2, 1, 1, 1, 1, 4, 4, 4, 4},
        {0, 1, -1, 1, -1, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 1, -1, 1, -1},
        {0, -1, 0, 1, 0, 2, -2, -2, 2},
        {0, 0, -1, 0, 1, 2, 2, -2, -2},
        {2, -4, -4, -4, -4, 8, 8, 8, 8},
    };
    static constexpr double N[Q] = {1.0, 1.0 / 3, 1.0 / 3, 4.0, 4.0 / 9, 1.0 / 9,
                                    2.0 / 3, 2.0 / 3, 16.0};
    static constexpr int cls[Q] = {CLS_RHO, CLS_MOM, CLS_MOM, CLS_BULK, CLS_SHEAR, CLS_SHEAR,
                                   CLS_GHOST, CLS_GHOST, CLS_GHOST};
    static constexpr int odd[Q] = {0, 1, 1, 0, 0, 0, 1, 1, 0};
    static constexpr int pair[NP][2] = {{1, 3}, {2, 4}, {5, 7}, {6, 8}};
    static constexpr int opp[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};   // c_opp(i) = -c_i
};

// ---------------------------------------------------------------- D3Q19
template <> struct Lattice<1> {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr int NP = 9;
    static constexpr int K = 15;
    static constexpr int NPAIR = 8;
    static constexpr int cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
    static constexpr int cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    static constexpr double w[Q] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                    1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr int T[Q][Q] = {
        {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
        {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0},
        {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1},
        {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
        {-1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
        {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
        {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
        {0, -2, 2, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0},
        {0, 0, 0, -2, 2, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1},
        {0, 0, 0, 0, 0, -2, 2, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
        {0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 0, 0, -1, 1, -1, 1, 0, 0, 0, 0, 1, 1, -1, -1},
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1},
        {1, -2, -2, -2, -2, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
        {0, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
        {0, 0, 0, -1, -1, 1, 1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    };
    static constexpr double N[Q] = {1.0,     1.0 / 3, 1.0 / 3, 1.0 / 3, 2.0 / 3,
                                    4.0 / 3, 4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    2.0 / 3, 2.0 / 3, 2.0 / 3, 2.0 / 9, 2.0 / 9,
                                    2.0 / 9, 2.0,     4.0 / 3, 4.0 / 9};
    static constexpr int cls[Q] = {CLS_RHO,   CLS_MOM,   CLS_MOM,   CLS_MOM,   CLS_BULK,
                                   CLS_SHEAR, CLS_SHEAR, CLS_SHEAR, CLS_SHEAR, CLS_SHEAR,
                                   CLS_GHOST, CLS_GHOST, CLS_GHOST, CLS_GHOST, CLS_GHOST,
                                   CLS_GHOST, CLS_GHOST, CLS_GHOST, CLS_GHOST};
    static constexpr int odd[Q] = {0, 1, 1, 1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 0, 0, 0};
    static constexpr int pair[NP][2] = {{1, 2},   {3, 4},   {5, 6},   {7, 10},  {8, 9},
                                        {11, 14}, {12, 13}, {15, 18}, {16, 17}};
    static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
};

// opp really maps every velocity to its negative
template <int LAT>
constexpr bool opp_ok() {
    using L = Lattice<LAT>;
    for (int i = 0; i < L::Q; ++i) {
        const int j = L::opp[i];
        if (L::cx[j] != -L::cx[i] || L::cy[j] != -L::cy[i] || L::cz[j] != -L::cz[i]) return false;
        if (L::opp[j] != i) return false;
    }
    return true;
}
static_assert(opp_ok<0>() && opp_ok<1>(), "opposite-velocity tables");

}  // namespace flb
