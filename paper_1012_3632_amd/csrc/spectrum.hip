// Equal-time mode spectra of one state: the measurement behind the
// equilibration ratio of Sec. VI (the equal-time correlation |m_a(k)|^2 of
// every LB mode, averaged over snapshots and divided by its theoretical
// variance).
//
// Input: the q real mode fields of a periodic nx x ny x nz lattice (site
// s = x + nx (y + ny z)).  The three-dimensional DFT
//   m_a(k) = sum_x m_a(x) exp(-i k.x),  k = 2 pi (kx / nx, ky / ny, kz / nz)
// is taken one axis at a time: every line along x, then y, then z, is
// transformed by one block that holds the line and its twiddle factors in
// LDS (a direct sum, n complex multiply-adds per output; the extents of the
// equilibration runs are 128 to 400, and the snapshots are hundreds of steps
// apart, so this is not the time that matters).  The last pass leaves m_a(k)
// in the work array; k_spec_accumulate then adds |m_a(k)|^2 for every mode
// and Re(j_alpha(k) conj j_beta(k)) for the momentum pairs (x, y) [2-D] or
// (x, y), (y, z), (z, x) [3-D], the cross spectra that split the momentum
// into longitudinal and transverse parts.  The same passes give the spectra
// of any real fields (flb_field_spectrum), e.g. of interface heights.
//
// Interface heights (the capillary test of Sec. VI): for every column across
// a planar interface, the shift h of the mean-field profile (eq. denprof)
// that best fits the column's density (eq. height-def), by Gauss-Newton.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace flb {

namespace {

constexpr int DFT_THREADS = 256;

// One line per block: blockIdx.x = line, blockIdx.y = field.  Element j of
// the line is at  field * V + (line % inner) + (line / inner) * outer + j * stride.
// The line is read from `real_in` (imaginary part zero) when that is non-null,
// else from `work`, and its transform X(k) = sum_j x(j) exp(-2 pi i j k / n)
// is written to `work` at the same positions (in place: the whole line is in
// LDS before any thread writes).  With gridDim.z > 1 (only when reading
// real_in, so that no block overwrites what another still reads) block z
// computes the outputs k = z DFT_THREADS + t, t < DFT_THREADS, of every
// gridDim.z DFT_THREADS.
__global__ __launch_bounds__(DFT_THREADS) void k_dft_lines(const double* __restrict__ real_in,
                                                            double2* work, int n, long stride,
                                                            long inner, long outer, long V) {
    __shared__ double2 tw[SPECTRUM_MAX_N];
    __shared__ double2 buf[SPECTRUM_MAX_N];
    const long line = blockIdx.x;
    const long base = (long)blockIdx.y * V + (line % inner) + (line / inner) * outer;
    for (int j = threadIdx.x; j < n; j += DFT_THREADS) {
        double sn, cs;
        sincospi(2.0 * (double)j / (double)n, &sn, &cs);
        tw[j] = make_double2(cs, -sn);
        const long off = base + (long)j * stride;
        buf[j] = real_in ? make_double2(real_in[off], 0.0) : work[off];
    }
    __syncthreads();
    for (int k = blockIdx.z * DFT_THREADS + threadIdx.x; k < n; k += DFT_THREADS * gridDim.z) {
        double re = 0.0, im = 0.0;
        int idx = 0;   // j k mod n
        for (int j = 0; j < n; ++j) {
            const double2 x = buf[j];
            const double2 w = tw[idx];
            re = fma(x.x, w.x, fma(-x.y, w.y, re));
            im = fma(x.x, w.y, fma(x.y, w.x, im));
            idx += k;
            if (idx >= n) idx -= n;
        }
        work[base + (long)k * stride] = make_double2(re, im);
    }
}

// spec[a V + s] += |W_a(s)|^2 (a < q); spec[(q + p) V + s] += Re(W_{1+al} conj W_{1+be})
// for the momentum pair p = (al, be) = (p, (p + 1) mod 3), p < npairs.
__global__ __launch_bounds__(256) void k_spec_accumulate(const double2* __restrict__ W,
                                                         double* __restrict__ spec, int q,
                                                         int npairs, long V) {
    for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < V;
         s += (long)gridDim.x * blockDim.x) {
        for (int a = 0; a < q; ++a) {
            const double2 w = W[a * V + s];
            spec[a * V + s] += w.x * w.x + w.y * w.y;
        }
        for (int p = 0; p < npairs; ++p) {
            const int al = p, be = (p + 1) % 3;
            const double2 u = W[(1 + al) * V + s], v = W[(1 + be) * V + s];
            spec[(q + p) * V + s] += u.x * v.x + u.y * v.y;
        }
    }
}

// Interface heights (capillary test): one wavefront per column c and
// interface j (blockIdx.y), its lanes over the window.  The density of column
// c at profile coordinate y is rho0 + drho[c + y ncol].  The height h minimizes
//   E(h) = sum_{k=-W..W} (rho(y0 + k) - m(y0 + k - h))^2,
//   m(u) = rho_c + sign (rho_L - rho_V)/2 tanh(2 u / w),
// the mean-field profile; Gauss-Newton from h = y0, clamped to the window,
// until the update is below 1e-13 (at most 64 iterations).  The two sums of
// every iteration are reduced over the wavefront by a fixed butterfly, so
// all lanes hold the same h and leave the loop together.
constexpr int HEIGHT_WAVES = 4;
template <typename Real>
__global__ __launch_bounds__(64 * HEIGHT_WAVES) void k_interface_heights(
    const Real* __restrict__ drho, double rho0, int n, long ncol, InterfaceSet set, double rho_c,
    double half_jump, double two_over_w, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const long c = (long)blockIdx.x * HEIGHT_WAVES + (threadIdx.x >> 6);
    const int j = blockIdx.y;
    if (c >= ncol) return;   // whole wavefronts leave together
    const int y0 = set.y0[j], W = set.half_window[j];
    const double s = set.sign[j] * half_jump;
    double h = (double)y0;
    for (int it = 0; it < 64; ++it) {
        double num = 0.0, den = 0.0;
        for (int k = -W + lane; k <= W; k += 64) {
            int yy = y0 + k;
            if (yy < 0) yy += n;
            if (yy >= n) yy -= n;
            const double r = rho0 + (double)drho[c + (long)yy * ncol];
            const double t = tanh(two_over_w * ((double)(y0 + k) - h));
            const double mp = s * (1.0 - t * t) * two_over_w;
            num += (r - (rho_c + s * t)) * mp;
            den += mp * mp;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            num += __shfl_xor(num, off, 64);
            den += __shfl_xor(den, off, 64);
        }
        if (!(den > 0.0)) break;
        const double hn = fmin(fmax(h - num / den, (double)(y0 - W)), (double)(y0 + W));
        const double dh = hn - h;
        h = hn;
        if (fabs(dh) < 1e-13) break;
    }
    if (lane == 0) out[(long)j * ncol + c] = h;
}

}  // namespace

hipError_t launch_interface_heights(int prec, const void* drho, double rho0, int n, long ncol,
                                    const InterfaceSet& set, double rho_L, double rho_V,
                                    double width, double* out, hipStream_t st) {
    const dim3 grid((unsigned)((ncol + HEIGHT_WAVES - 1) / HEIGHT_WAVES), set.n);
    const dim3 block(64 * HEIGHT_WAVES);
    const double rc = 0.5 * (rho_L + rho_V), half = 0.5 * (rho_L - rho_V), tw = 2.0 / width;
    if (prec == 0)
        hipLaunchKernelGGL(k_interface_heights<float>, grid, block, 0, st, (const float*)drho,
                           rho0, n, ncol, set, rc, half, tw, out);
    else
        hipLaunchKernelGGL(k_interface_heights<double>, grid, block, 0, st, (const double*)drho,
                           rho0, n, ncol, set, rc, half, tw, out);
    return hipGetLastError();
}

hipError_t launch_spectrum(int q, int npairs, int nx, int ny, int nz, const double* fields,
                           void* work, double* spec, hipStream_t st) {
    const long V = (long)nx * ny * nz;
    double2* W = (double2*)work;
    // x: lines of contiguous sites, read from the real fields; few long lines
    // have their outputs split over blocks
    const long xlines = V / nx;
    int chunks = 1;
    while (chunks * DFT_THREADS < nx && xlines * q * chunks < 1024) chunks *= 2;
    hipLaunchKernelGGL(k_dft_lines, dim3((unsigned)xlines, q, chunks), dim3(DFT_THREADS), 0, st,
                       fields, W, nx, 1L, 1L, (long)nx, V);
    if (ny > 1)
        hipLaunchKernelGGL(k_dft_lines, dim3((unsigned)(V / ny), q), dim3(DFT_THREADS), 0, st,
                           nullptr, W, ny, (long)nx, (long)nx, (long)nx * ny, V);
    if (nz > 1)
        hipLaunchKernelGGL(k_dft_lines, dim3((unsigned)(V / nz), q), dim3(DFT_THREADS), 0, st,
                           nullptr, W, nz, (long)nx * ny, (long)nx * ny, V, V);
    const long blocks = (V + 255) / 256 < 4096 ? (V + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_spec_accumulate, dim3((unsigned)blocks), dim3(256), 0, st, W, spec, q,
                       npairs, V);
    return hipGetLastError();
}

}  // namespace flb
