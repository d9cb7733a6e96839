// Modified-equilibrium (Swift) fluctuating LB, linearized about rest, D2Q9
// (Sec. IV.B, subsection on the modified-equilibrium model).
//
// State: the deviations delta f_i from the uniform rest state, stored
// f[i * V + x + nx y].  One step with index n:
//   pull       f_i(x) = S_i(x - c_i)
//   moments    m_a = sum_i T_ai f_i                        (App. B basis)
//   equilibrium (eq. meq-yeo, linearized)  m^eq = {rho, j_x, j_y, D, 0, 0, 0, 0, -D},
//              D = d(k) rho = 6 (cs2_0 - cs2) rho - 6 kappa rho0 lap_h rho,
//              i.e. d(k) = 6 (c_s^2(k) - cs2) with c_s^2(k) = cs2_0 + kappa rho0 Lambda(k),
//              Lambda(k) = (4/3)(2 - cos kx - cos ky) + (2/3)(1 - cos kx cos ky)
//              the symbol of -lap_h (9-point isotropic Laplacian)
//   relax      m*_a = m_a - lam_a (m_a - m^eq_a) + xi_a
//   back       S_{n+1,i} = w_i sum_a T_ai m*_a / N_a.
// Noise: the covariance Xi(k) = G - C G C^T that keeps the equal-time
// correlations of eq. f-correl-yeo stationary under the step.  p_xx, p_xy,
// q_x, q_y get white noise rho0 kT N_a lam (2 - lam) / cs2; the (e, eps) pair
// has the k-dependent block
//   Xi_ee = 12 rho0 kT lam_e (2 - lam_e)(2 - 3 c2),
//   Xi_eE = 12 rho0 kT (3 c2 - 1)(lam_e + lam_g - lam_e lam_g),
//   Xi_EE = 12 rho0 kT lam_g (2 - lam_g)(5 - 3 c2),      c2 = c_s^2(k),
// whose small-rate limit is eq. noise-yeo (the (e, eps) entry at half its
// printed value: the value for which Xi is a covariance wherever the
// equilibrium populations are non-negative).  That pair is drawn as white
// normals z_e, z_eps (the site's Philox normals 0 and 5), transformed, mixed
// by the lower Cholesky factor of the block at every k, and transformed back:
//   k_meq_noise_x      normals of one row, DFT along x         (one block per row)
//   k_meq_filter_cols  DFT along y, Cholesky mix, inverse DFT  (CB adjacent columns
//     / k_meq_filter_y                                          per block; one column
//                                                               when ny is not a power of 2)
//   k_meq_noise_ix     inverse DFT along x, real part / V      (one block per row)
// The noise does not depend on the state, so a launch of these three
// kernels draws and filters the noise of a batch of consecutive steps
// (blockIdx.y = step within the batch): at small lattices a single step's
// lines are far fewer blocks than the chip has CUs.
// Each line sits in LDS with its twiddles.  Power-of-two extents use an
// in-place radix-2 FFT, the butterfly stages taken three per pass through LDS
// and shared by all lines of a block: decimation in time from bit-reversed
// input for the rows, and for the columns decimation in frequency forward
// (bit-reversed output), the mix in that order, then decimation in time back.
// Other extents (at most 1024) use direct sums.  Then k_meq_step applies the
// step.  The transforms and the filtered fields are in the state's precision
// (R = float or double; twiddles and Cholesky factors formed in FP64 and
// rounded once).
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"
#include "philox.h"

namespace flb {

namespace {

constexpr int MQ_THREADS = 256;
constexpr int MQ_MAXK = SPECTRUM_MAX_N / MQ_THREADS;   // outputs per thread and line
constexpr int MQ_TX = 64, MQ_TY = 4;

// Complex values of precision R in LDS and in the work buffer.
template <typename R> struct Cx;
template <> struct Cx<double> {
    using T = double2;
    static __device__ __forceinline__ T make(double re, double im) { return make_double2(re, im); }
};
template <> struct Cx<float> {
    using T = float2;
    static __device__ __forceinline__ T make(float re, float im) { return make_float2(re, im); }
};
template <typename R> using cx_t = typename Cx<R>::T;

// X(k) = sum_j x(j) exp(-+ 2 pi i j k / n) (sign - forward, + inverse), from a
// line in LDS and the forward twiddles tw[j] = exp(-2 pi i j / n).
template <typename R>
__device__ __forceinline__ cx_t<R> dft_at(const cx_t<R>* __restrict__ buf,
                                          const cx_t<R>* __restrict__ tw, int n, int k,
                                          bool inverse) {
    R re = R(0), im = R(0);
    int idx = 0;   // j k mod n
    for (int j = 0; j < n; ++j) {
        const cx_t<R> x = buf[j];
        const cx_t<R> w = tw[idx];
        const R wi = inverse ? -w.y : w.y;
        re = fma(x.x, w.x, fma(-x.y, wi, re));
        im = fma(x.x, wi, fma(x.y, w.x, im));
        idx += k;
        if (idx >= n) idx -= n;
    }
    return Cx<R>::make(re, im);
}

// tw[j] = exp(-2 pi i j / n), evaluated in FP64 and rounded to R.
template <typename R>
__device__ __forceinline__ void twiddles(cx_t<R>* tw, int n) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)j / (double)n, &s, &c);
        tw[j] = Cx<R>::make((R)c, (R)-s);
    }
}

__device__ __forceinline__ bool pow2(int n) { return (n & (n - 1)) == 0; }

__device__ __forceinline__ int log2i(int n) { return 31 - __clz(n); }

// Position of element j in the bit-reversed order of a 2^logn line.
__device__ __forceinline__ int brev(int j, int logn) {
    return logn == 0 ? 0 : (int)(__brev((unsigned)j) >> (32 - logn));
}

// a + w x, a - w x for complex values, w's imaginary part negated for an
// inverse transform
template <typename R>
__device__ __forceinline__ void bfly(cx_t<R>& a, cx_t<R>& x, cx_t<R> w, bool inverse) {
    const R wi = inverse ? -w.y : w.y;
    const R vr = x.x * w.x - x.y * wi, vi = x.x * wi + x.y * w.x;
    x = Cx<R>::make(a.x - vr, a.y - vi);
    a = Cx<R>::make(a.x + vr, a.y + vi);
}

// In place, the NL lines b[L n .. (L + 1) n) (n = 2^logn), each loaded in
// bit-reversed order, become their transforms in natural order
// (exp(-+ 2 pi i j k / n), sign - forward, + inverse): decimation in time.
// Radix-2 stages are taken three at a time: stages s, s + 1, s + 2 (half
// h = 2^(s-1)) combine the eight elements a + k h (k = 0 .. 7) of a group, so
// a thread loads them once, applies the three stages in registers and stores
// them; the groups of a pass are disjoint.  The one or two stages left over
// take a pass of four-element groups or a plain radix-2 pass.  Every
// butterfly is the one of the stage-by-stage transform.  Ends with a barrier.
template <typename R>
__device__ __forceinline__ void fft_lines_dit(cx_t<R>* b, const cx_t<R>* __restrict__ tw, int NL,
                                              int n, int logn, bool inverse) {
    int s = 1;
    for (; s + 2 <= logn; s += 3) {
        const int h = 1 << (s - 1);
        const int st1 = n >> s, st2 = n >> (s + 1), st3 = n >> (s + 2);
        const int ng = n >> 3;
        for (int t = threadIdx.x; t < NL * ng; t += blockDim.x) {
            const int L = t >> (logn - 3);
            const int q = t - L * ng;
            const int pos = q & (h - 1);
            const int a = L * n + ((q >> (s - 1)) << (s + 2)) + pos;
            cx_t<R> x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = b[a + k * h];
            const cx_t<R> w1 = tw[pos * st1];
#pragma unroll
            for (int k = 0; k < 8; k += 2) bfly<R>(x[k], x[k + 1], w1, inverse);   // stage s
            const cx_t<R> w20 = tw[pos * st2], w21 = tw[(pos + h) * st2];
            bfly<R>(x[0], x[2], w20, inverse);                                    // stage s + 1
            bfly<R>(x[1], x[3], w21, inverse);
            bfly<R>(x[4], x[6], w20, inverse);
            bfly<R>(x[5], x[7], w21, inverse);
#pragma unroll
            for (int k = 0; k < 4; ++k) bfly<R>(x[k], x[k + 4], tw[(pos + k * h) * st3], inverse);   // stage s + 2
#pragma unroll
            for (int k = 0; k < 8; ++k) b[a + k * h] = x[k];
        }
        __syncthreads();
    }
    for (; s + 1 <= logn; s += 2) {
        const int h = 1 << (s - 1);
        const int st1 = n >> s, st2 = n >> (s + 1);
        const int nq = n >> 2;
        for (int t = threadIdx.x; t < NL * nq; t += blockDim.x) {
            const int L = t >> (logn - 2);
            const int q = t - L * nq;
            const int pos = q & (h - 1);
            const int a = L * n + ((q >> (s - 1)) << (s + 1)) + pos;
            cx_t<R> x0 = b[a], x1 = b[a + h], x2 = b[a + 2 * h], x3 = b[a + 3 * h];
            const cx_t<R> w1 = tw[pos * st1];
            bfly<R>(x0, x1, w1, inverse);   // stage s
            bfly<R>(x2, x3, w1, inverse);
            bfly<R>(x0, x2, tw[pos * st2], inverse);         // stage s + 1
            bfly<R>(x1, x3, tw[(pos + h) * st2], inverse);
            b[a] = x0;
            b[a + h] = x1;
            b[a + 2 * h] = x2;
            b[a + 3 * h] = x3;
        }
        __syncthreads();
    }
    if (s == logn) {
        const int h = 1 << (s - 1);
        const int st1 = n >> s;
        const int nh = n >> 1;
        for (int t = threadIdx.x; t < NL * nh; t += blockDim.x) {
            const int L = t >> (logn - 1);
            const int bt = t - L * nh;
            const int pos = bt & (h - 1);
            const int i0 = L * n + ((bt >> (s - 1)) << s) + pos;
            cx_t<R> u = b[i0], x = b[i0 + h];
            bfly<R>(u, x, tw[pos * st1], inverse);
            b[i0] = u;
            b[i0 + h] = x;
        }
        __syncthreads();
    }
}

template <typename R>
__device__ __forceinline__ void fft2_lines(cx_t<R>* b, const cx_t<R>* __restrict__ tw, int n,
                                           int logn, bool inverse) {
    fft_lines_dit<R>(b, tw, 2, n, logn, inverse);
}

// (u, v) -> (u + v, (u - v) w): the decimation-in-frequency butterfly
template <typename R>
__device__ __forceinline__ void bfly_dif(cx_t<R>& u, cx_t<R>& v, cx_t<R> w) {
    const R dr = u.x - v.x, di = u.y - v.y;
    u = Cx<R>::make(u.x + v.x, u.y + v.y);
    v = Cx<R>::make(dr * w.x - di * w.y, dr * w.y + di * w.x);
}

// In place, the NL lines of b (natural order) become their forward
// transforms in bit-reversed order: decimation in frequency, stages from
// half n/2 down to 1, three per pass (halves 4 q, 2 q and q combine the
// elements a + k q, k = 0 .. 7, of a group of 8 q); one or two stages left
// over take a pass of four-element groups (halves 2 q, q) or the last stage
// (half 1) alone.  Every butterfly is the one of the stage-by-stage
// transform.  Ends with a barrier.
template <typename R>
__device__ __forceinline__ void fft_lines_dif(cx_t<R>* b, const cx_t<R>* __restrict__ tw, int NL,
                                              int n, int logn) {
    int s = logn;
    for (; s >= 3; s -= 3) {
        const int q8 = 1 << (s - 3);
        const int stA = n >> s, stB = n >> (s - 1), stC = n >> (s - 2);
        const int ng = n >> 3;
        for (int t = threadIdx.x; t < NL * ng; t += blockDim.x) {
            const int L = t >> (logn - 3);
            const int qq = t - L * ng;
            const int pos = qq & (q8 - 1);
            const int a = L * n + ((qq >> (s - 3)) << s) + pos;
            cx_t<R> x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = b[a + k * q8];
#pragma unroll
            for (int k = 0; k < 4; ++k) bfly_dif<R>(x[k], x[k + 4], tw[(pos + k * q8) * stA]);   // half 4 q8
            const cx_t<R> wB0 = tw[pos * stB], wB1 = tw[(pos + q8) * stB];
            bfly_dif<R>(x[0], x[2], wB0);                                                      // half 2 q8
            bfly_dif<R>(x[1], x[3], wB1);
            bfly_dif<R>(x[4], x[6], wB0);
            bfly_dif<R>(x[5], x[7], wB1);
            const cx_t<R> wC = tw[pos * stC];                                                  // half q8
#pragma unroll
            for (int k = 0; k < 8; k += 2) bfly_dif<R>(x[k], x[k + 1], wC);
#pragma unroll
            for (int k = 0; k < 8; ++k) b[a + k * q8] = x[k];
        }
        __syncthreads();
    }
    for (; s >= 2; s -= 2) {
        const int q4 = 1 << (s - 2);
        const int stA = n >> s, stC = n >> (s - 1);
        const int nq = n >> 2;
        for (int t = threadIdx.x; t < NL * nq; t += blockDim.x) {
            const int L = t >> (logn - 2);
            const int qq = t - L * nq;
            const int pos = qq & (q4 - 1);
            const int a = L * n + ((qq >> (s - 2)) << s) + pos;
            cx_t<R> x0 = b[a], x1 = b[a + q4], x2 = b[a + 2 * q4], x3 = b[a + 3 * q4];
            bfly_dif<R>(x0, x2, tw[pos * stA]);          // half 2 q4
            bfly_dif<R>(x1, x3, tw[(pos + q4) * stA]);
            const cx_t<R> wC = tw[pos * stC];         // half q4
            bfly_dif<R>(x0, x1, wC);
            bfly_dif<R>(x2, x3, wC);
            b[a] = x0;
            b[a + q4] = x1;
            b[a + 2 * q4] = x2;
            b[a + 3 * q4] = x3;
        }
        __syncthreads();
    }
    if (s == 1) {
        const int nh = n >> 1;
        for (int t = threadIdx.x; t < NL * nh; t += blockDim.x) {
            const int L = t >> (logn - 1);
            const int i0 = L * n + 2 * (t - L * nh);
            cx_t<R> u = b[i0], v = b[i0 + 1];
            bfly_dif<R>(u, v, Cx<R>::make(R(1), R(0)));
            b[i0] = u;
            b[i0 + 1] = v;
        }
        __syncthreads();
    }
}

// Lower Cholesky factor of the (e, eps) noise block at wavenumber (kx, ky),
// given cos kx and cos ky, in FP64.
__device__ __forceinline__ void meq_chol(const ModEqArgs& a, double cx, double cy, double& l11,
                                         double& l21, double& l22) {
    const double pre = 12.0 * a.rho0 * a.kT;
    const double le = a.rate_bulk, lg = a.rate_ghost;
    const double lap = (4.0 / 3.0) * (2.0 - cx - cy) + (2.0 / 3.0) * (1.0 - cx * cy);
    const double c2 = a.cs2_0 + a.kappa * a.rho0 * lap;
    const double see = pre * le * (2.0 - le) * (2.0 - 3.0 * c2);
    const double sep = pre * (3.0 * c2 - 1.0) * (le + lg - le * lg);
    const double spp = pre * lg * (2.0 - lg) * (5.0 - 3.0 * c2);
    l11 = sqrt(fmax(see, 0.0));
    l21 = l11 > 0.0 ? sep / l11 : 0.0;
    l22 = sqrt(fmax(spp - l21 * l21, 0.0));
}

// Dynamic LDS of the noise kernels (lines and twiddles of either precision).
extern __shared__ __align__(16) unsigned char lds_mq[];

template <typename Real>
__global__ __launch_bounds__(MQ_THREADS) void k_meq_noise_x(ModEqArgs a, uint32_t step0,
                                                            cx_t<Real>* __restrict__ W) {
    using C = cx_t<Real>;
    const int n = a.nx, y = blockIdx.x;
    const size_t V = (size_t)a.nx * a.ny;
    const uint32_t step = step0 + blockIdx.y;
    W += (size_t)blockIdx.y * 2 * V;
    C* tw = (C*)lds_mq;
    C* be = tw + n;
    C* bp = tw + 2 * n;
    const bool fft = pow2(n);
    const int logn = log2i(n);
    twiddles<Real>(tw, n);
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        Real z[6];
        site_normals<3, Real>((uint32_t)(x + n * y), step, 0u, 0u, a.k0, a.k1, z);
        const int j = fft ? brev(x, logn) : x;
        be[j] = Cx<Real>::make(z[0], Real(0));
        bp[j] = Cx<Real>::make(z[5], Real(0));
    }
    __syncthreads();
    if (fft) {
        fft2_lines<Real>(be, tw, n, logn, false);
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            W[(size_t)y * n + k] = be[k];
            W[V + (size_t)y * n + k] = bp[k];
        }
        return;
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        W[(size_t)y * n + k] = dft_at<Real>(be, tw, n, k, false);
        W[V + (size_t)y * n + k] = dft_at<Real>(bp, tw, n, k, false);
    }
}

template <typename Real>
__global__ __launch_bounds__(MQ_THREADS) void k_meq_filter_y(ModEqArgs a,
                                                             cx_t<Real>* __restrict__ W) {
    using C = cx_t<Real>;
    // blocks of neighbouring columns (which share cache lines) go to the same
    // XCD, so one L2 serves the line to all of them
    const uint32_t lin = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int n = a.ny, nx = a.nx, kx = (int)(lin % gridDim.x);
    const size_t V = (size_t)a.nx * a.ny;
    W += (size_t)(lin / gridDim.x) * 2 * V;
    C* tw = (C*)lds_mq;
    C* be = tw + n;
    C* bp = tw + 2 * n;
    const bool fft = pow2(n);
    const int logn = log2i(n);
    twiddles<Real>(tw, n);
    for (int y = threadIdx.x; y < n; y += blockDim.x) {
        const int j = fft ? brev(y, logn) : y;
        be[j] = W[(size_t)y * nx + kx];
        bp[j] = W[V + (size_t)y * nx + kx];
    }
    __syncthreads();
    if (fft) fft2_lines<Real>(be, tw, n, logn, false);
    double sx, cx;
    sincospi(2.0 * (double)kx / (double)nx, &sx, &cx);
    C oe[MQ_MAXK], op[MQ_MAXK];
#pragma unroll
    for (int r = 0; r < MQ_MAXK; ++r) {
        const int ky = threadIdx.x + r * MQ_THREADS;
        if (ky < n) {
            const C ze = fft ? be[ky] : dft_at<Real>(be, tw, n, ky, false);
            const C zp = fft ? bp[ky] : dft_at<Real>(bp, tw, n, ky, false);
            double d11, d21, d22;
            meq_chol(a, cx, (double)tw[ky].x, d11, d21, d22);
            const Real l11 = (Real)d11, l21 = (Real)d21, l22 = (Real)d22;
            oe[r] = Cx<Real>::make(l11 * ze.x, l11 * ze.y);
            op[r] = Cx<Real>::make(l21 * ze.x + l22 * zp.x, l21 * ze.y + l22 * zp.y);
        }
    }
    __syncthreads();   // every forward value has been read from be, bp
#pragma unroll
    for (int r = 0; r < MQ_MAXK; ++r) {
        const int ky = threadIdx.x + r * MQ_THREADS;
        if (ky < n) {
            const int j = fft ? brev(ky, logn) : ky;
            be[j] = oe[r];
            bp[j] = op[r];
        }
    }
    __syncthreads();
    if (fft) {
        fft2_lines<Real>(be, tw, n, logn, true);
        for (int y = threadIdx.x; y < n; y += blockDim.x) {
            W[(size_t)y * nx + kx] = be[y];
            W[V + (size_t)y * nx + kx] = bp[y];
        }
        return;
    }
    for (int y = threadIdx.x; y < n; y += blockDim.x) {
        W[(size_t)y * nx + kx] = dft_at<Real>(be, tw, n, y, true);
        W[V + (size_t)y * nx + kx] = dft_at<Real>(bp, tw, n, y, true);
    }
}

// Power-of-two ny: CB adjacent columns per block (loads and stores of a row
// touch CB consecutive values).  The forward transforms leave the spectra in
// bit-reversed order (decimation in frequency), the Cholesky mix is
// pointwise there (position j holds wavenumber ky = brev(j)), and the inverse
// transforms take that order back to natural order (decimation in time), so
// no permutation step is needed.  Lines in LDS: e of columns 0 .. CB-1, then
// eps.  nx must be a multiple of CB.
template <typename Real, int CB>
__global__ __launch_bounds__(MQ_THREADS) void k_meq_filter_cols(ModEqArgs a,
                                                                cx_t<Real>* __restrict__ W) {
    using C = cx_t<Real>;
    // blocks of neighbouring column groups (which share cache lines) go to
    // the same XCD, so one L2 serves the line to all of them
    const uint32_t lin = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int n = a.ny, nx = a.nx, kx0 = (int)(lin % gridDim.x) * CB;
    const int logn = log2i(n);
    const size_t V = (size_t)a.nx * a.ny;
    W += (size_t)(lin / gridDim.x) * 2 * V;
    C* tw = (C*)lds_mq;
    C* b = tw + n;
    twiddles<Real>(tw, n);
    for (int idx = threadIdx.x; idx < CB * n; idx += blockDim.x) {
        const int y = idx / CB, c = idx - y * CB;
        b[c * n + y] = W[(size_t)y * nx + kx0 + c];
        b[(CB + c) * n + y] = W[V + (size_t)y * nx + kx0 + c];
    }
    __syncthreads();
    fft_lines_dif<Real>(b, tw, 2 * CB, n, logn);
    double cxs[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        double sx;
        sincospi(2.0 * (double)(kx0 + c) / (double)nx, &sx, &cxs[c]);
    }
    for (int idx = threadIdx.x; idx < CB * n; idx += blockDim.x) {
        const int c = idx >> logn, j = idx & (n - 1);
        double d11, d21, d22;
        meq_chol(a, cxs[c], (double)tw[brev(j, logn)].x, d11, d21, d22);
        const Real l11 = (Real)d11, l21 = (Real)d21, l22 = (Real)d22;
        const C ze = b[c * n + j], zp = b[(CB + c) * n + j];
        b[c * n + j] = Cx<Real>::make(l11 * ze.x, l11 * ze.y);
        b[(CB + c) * n + j] = Cx<Real>::make(l21 * ze.x + l22 * zp.x, l21 * ze.y + l22 * zp.y);
    }
    __syncthreads();
    fft_lines_dit<Real>(b, tw, 2 * CB, n, logn, true);
    for (int idx = threadIdx.x; idx < CB * n; idx += blockDim.x) {
        const int y = idx / CB, c = idx - y * CB;
        W[(size_t)y * nx + kx0 + c] = b[c * n + y];
        W[V + (size_t)y * nx + kx0 + c] = b[(CB + c) * n + y];
    }
}

template <typename Real>
__global__ __launch_bounds__(MQ_THREADS) void k_meq_noise_ix(ModEqArgs a,
                                                             const cx_t<Real>* __restrict__ W,
                                                             Real* __restrict__ xi) {
    using C = cx_t<Real>;
    const int n = a.nx, y = blockIdx.x;
    const size_t V = (size_t)a.nx * a.ny;
    const Real inv_v = (Real)(1.0 / (double)V);
    W += (size_t)blockIdx.y * 2 * V;
    xi += (size_t)blockIdx.y * 2 * V;
    C* tw = (C*)lds_mq;
    C* be = tw + n;
    C* bp = tw + 2 * n;
    const bool fft = pow2(n);
    const int logn = log2i(n);
    twiddles<Real>(tw, n);
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        const int j = fft ? brev(x, logn) : x;
        be[j] = W[(size_t)y * n + x];
        bp[j] = W[V + (size_t)y * n + x];
    }
    __syncthreads();
    if (fft) {
        fft2_lines<Real>(be, tw, n, logn, true);
        for (int x = threadIdx.x; x < n; x += blockDim.x) {
            xi[(size_t)y * n + x] = be[x].x * inv_v;
            xi[V + (size_t)y * n + x] = bp[x].x * inv_v;
        }
        return;
    }
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        xi[(size_t)y * n + x] = dft_at<Real>(be, tw, n, x, true).x * inv_v;
        xi[V + (size_t)y * n + x] = dft_at<Real>(bp, tw, n, x, true).x * inv_v;
    }
}

__device__ __forceinline__ int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

template <typename Real>
__global__ __launch_bounds__(MQ_TX * MQ_TY) void k_meq_step(ModEqArgs a, Geom g,
                                                            const Real* __restrict__ fin,
                                                            Real* __restrict__ fout,
                                                            uint32_t step,
                                                            const Real* __restrict__ xi) {
    using L = Lattice<0>;
    constexpr int SX = MQ_TX + 2, NS = SX * (MQ_TY + 2);
    constexpr int NRING = NS - MQ_TX * MQ_TY;   // halo sites: two rows of SX, two columns of TY
    static_assert(NRING <= MQ_TX * MQ_TY, "one halo site per thread at most");
    __shared__ Real rs[NS];
    const int x0 = blockIdx.x * MQ_TX, y0 = blockIdx.y * MQ_TY;
    const int tx = threadIdx.x % MQ_TX, ty = threadIdx.x / MQ_TX;
    const int x = x0 + tx, y = y0 + ty;
    // density of the pulled populations on the tile and a one-site halo: each
    // thread pulls its own site (periodic image for a ragged edge) and keeps
    // the populations, the first NRING threads pull the halo ring
    Real f[L::Q];
    pull<0, Real>(fin, wrap(x, g.nx), wrap(y, g.ny), 0, g, f);
    {
        Real s = Real(0);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) s += f[i];
        rs[(ty + 1) * SX + tx + 1] = s;
    }
    if (threadIdx.x < NRING) {
        const int r = threadIdx.x;
        int lx, ly;
        if (r < SX) {
            lx = r;
            ly = 0;
        } else if (r < 2 * SX) {
            lx = r - SX;
            ly = MQ_TY + 1;
        } else {
            const int c = r - 2 * SX;   // 0 .. 2 TY - 1
            lx = c < MQ_TY ? 0 : SX - 1;
            ly = 1 + (c < MQ_TY ? c : c - MQ_TY);
        }
        Real h[L::Q];
        pull<0, Real>(fin, wrap(x0 - 1 + lx, g.nx), wrap(y0 - 1 + ly, g.ny), 0, g, h);
        Real s = Real(0);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) s += h[i];
        rs[ly * SX + lx] = s;
    }
    __syncthreads();
    if (x >= g.nx || y >= g.ny) return;
    Real m[L::Q];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        Real s = Real(0);
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            if (L::T[q][i] != 0) s += Real(L::T[q][i]) * f[i];
        m[q] = s;
    }
    const int c = (ty + 1) * SX + tx + 1;
    Real lap = Real(0);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) lap += Real(L::w[i]) * (rs[c + L::cy[i] * SX + L::cx[i]] - rs[c]);
    lap *= Real(6);
    const Real D = Real(6.0 * (a.cs2_0 - 1.0 / 3.0)) * m[0] - Real(6.0 * a.kappa * a.rho0) * lap;
    const Real le = Real(a.rate_bulk), ls = Real(a.rate_shear), lg = Real(a.rate_ghost);
    m[3] -= le * (m[3] - D);
    m[4] -= ls * m[4];
    m[5] -= ls * m[5];
    m[6] -= lg * m[6];
    m[7] -= lg * m[7];
    m[8] -= lg * (m[8] + D);
    const uint32_t site = (uint32_t)(x + g.nx * y);
    if (xi) {
        Real z[6];
        site_normals<3, Real>(site, step, 0u, 0u, a.k0, a.k1, z);
        m[3] += xi[site];
        m[4] += Real(a.amp[0]) * z[1];
        m[5] += Real(a.amp[1]) * z[2];
        m[6] += Real(a.amp[2]) * z[3];
        m[7] += Real(a.amp[3]) * z[4];
        m[8] += xi[g.V + site];
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        Real s = Real(0);
#pragma unroll
        for (int q = 0; q < L::Q; ++q)
            if (L::T[q][i] != 0) s += Real(L::T[q][i] / L::N[q]) * m[q];
        plane_st(fout + (size_t)i * g.V, site, Real(L::w[i]) * s);
    }
}

// Analysis: the nine moment fields m_a(x) = sum_i T_ai f_i(x) of the pulled
// populations, in FP64, m[a * V + site].
template <typename Real>
__global__ __launch_bounds__(256) void k_meq_moments(Geom g, const Real* __restrict__ fin,
                                                     double* __restrict__ m) {
    using L = Lattice<0>;
    const uint32_t site = blockIdx.x * 256u + threadIdx.x;
    if (site >= g.V) return;
    const int x = (int)(site % (uint32_t)g.nx), y = (int)(site / (uint32_t)g.nx);
    Real f[L::Q];
    pull<0, Real>(fin, x, y, 0, g, f);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            if (L::T[q][i] != 0) s += (double)L::T[q][i] * (double)f[i];
        m[(size_t)q * g.V + site] = s;
    }
}

}  // namespace

hipError_t launch_modeq_moments(const ModEqArgs& a, int prec, const void* fin, double* m,
                                hipStream_t st) {
    Geom g{};
    g.nx = a.nx;
    g.ny = a.ny;
    g.nz = 1;
    g.V = (uint32_t)((size_t)a.nx * a.ny);
    const dim3 grid((g.V + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(k_meq_moments<float>, grid, dim3(256), 0, st, g, (const float*)fin, m);
    else
        hipLaunchKernelGGL(k_meq_moments<double>, grid, dim3(256), 0, st, g, (const double*)fin, m);
    return hipGetLastError();
}

size_t modeq_work_bytes(int nx, int ny, int prec) {
    const size_t V = (size_t)nx * ny;
    const size_t r = prec == 0 ? sizeof(float) : sizeof(double);
    return 2 * V * (2 * r) + 2 * V * r;
}

namespace {

// Choice of CB for k_meq_filter_cols: the widest of 4, 2 that divides nx and
// whose lines fit the block's LDS, else 1.
int filter_cols_cb(const ModEqArgs& a, size_t csize) {
    int dev = 0, lmax = 65536;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const size_t per = (size_t)a.ny * csize;
    // two columns per block measured fastest at 1024^2 (323 us per 16-step
    // launch against 385 for four and 337 for one): twice the resident
    // blocks of four for half the LDS
    for (int c : {2, 4})
        if (a.nx % c == 0 && (1 + 2 * (size_t)c) * per <= (size_t)lmax) return c;
    return 1;
}

template <typename Real, int CB>
hipError_t launch_filter_cols(const ModEqArgs& a, int nb, cx_t<Real>* W, hipStream_t st) {
    const size_t lc = (1 + 2 * (size_t)CB) * (size_t)a.ny * sizeof(cx_t<Real>);
    hipError_t e = hipFuncSetAttribute((const void*)k_meq_filter_cols<Real, CB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lc);
    if (e != hipSuccess) return e;
    const dim3 gc((unsigned)(a.nx / CB), (unsigned)nb);
    hipLaunchKernelGGL((k_meq_filter_cols<Real, CB>), gc, dim3(MQ_THREADS), lc, st, a, W);
    return hipSuccess;
}

template <typename Real>
hipError_t launch_noise_t(const ModEqArgs& a, uint32_t step0, int nb, void* Wv, Real* xi,
                          hipStream_t st) {
    using C = cx_t<Real>;
    C* W = (C*)Wv;
    const size_t lx = 3 * (size_t)a.nx * sizeof(C), ly = 3 * (size_t)a.ny * sizeof(C);
    const dim3 gx((unsigned)a.ny, (unsigned)nb), gy((unsigned)a.nx, (unsigned)nb);
    hipLaunchKernelGGL(k_meq_noise_x<Real>, gx, dim3(MQ_THREADS), lx, st, a, step0, W);
    if ((a.ny & (a.ny - 1)) == 0) {
        hipError_t e = hipSuccess;
        switch (filter_cols_cb(a, sizeof(C))) {
            case 4: e = launch_filter_cols<Real, 4>(a, nb, W, st); break;
            case 2: e = launch_filter_cols<Real, 2>(a, nb, W, st); break;
            default: e = launch_filter_cols<Real, 1>(a, nb, W, st); break;
        }
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_meq_filter_y<Real>, gy, dim3(MQ_THREADS), ly, st, a, W);
    }
    hipLaunchKernelGGL(k_meq_noise_ix<Real>, gx, dim3(MQ_THREADS), lx, st, a, (const C*)W, xi);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_modeq_noise(const ModEqArgs& a, int prec, uint32_t step0, int nb, void* W,
                              void* xi, hipStream_t st) {
    if (prec == 0) return launch_noise_t<float>(a, step0, nb, W, (float*)xi, st);
    return launch_noise_t<double>(a, step0, nb, W, (double*)xi, st);
}

hipError_t launch_modeq_step(const ModEqArgs& a, int prec, const void* fin, void* fout,
                             uint32_t step, const void* xi, hipStream_t st) {
    const size_t V = (size_t)a.nx * a.ny;
    Geom g{};
    g.nx = a.nx;
    g.ny = a.ny;
    g.nz = 1;
    g.nbx = (a.nx + MQ_TX - 1) / MQ_TX;
    g.nby = (a.ny + MQ_TY - 1) / MQ_TY;
    g.nbz = 1;
    g.nblocks = (uint32_t)(g.nbx * g.nby);
    g.V = (uint32_t)V;
    g.zc = 0;
    const dim3 grid((unsigned)g.nbx, (unsigned)g.nby);
    if (prec == 0)
        hipLaunchKernelGGL(k_meq_step<float>, grid, dim3(MQ_TX * MQ_TY), 0, st, a, g,
                           (const float*)fin, (float*)fout, step, (const float*)xi);
    else
        hipLaunchKernelGGL(k_meq_step<double>, grid, dim3(MQ_TX * MQ_TY), 0, st, a, g,
                           (const double*)fin, (double*)fout, step, (const double*)xi);
    return hipGetLastError();
}

}  // namespace flb
