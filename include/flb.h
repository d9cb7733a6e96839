/*
 * flb.h -- C ABI of the MI355X (gfx950) fluctuating lattice Boltzmann library.
 *
 * The library integrates the fluctuating lattice Boltzmann equation in moment
 * space (Gross, Cates, Varnik, Adhikari, "Langevin theory of fluctuations in
 * the discrete Boltzmann equation", Sec. V eq. lbe-mom) on periodic D2Q9 or
 * D3Q19 lattices, for the ideal gas (Sec. IV.A) and for the force-based
 * non-ideal fluid (Sec. IV.B.1) with the square-gradient force of App. A
 * (eq. he-force) and the Landau double well of Sec. VI (eq. f0-bulk); and,
 * handle-free (flb_modeq_*), the modified-equilibrium model of Sec. IV.B
 * linearized about rest on D2Q9, with its k-dependent noise.
 *
 * One time step with index n maps the post-collision populations S_n to S_{n+1}:
 *   pull      f_i(x) = S_{n,i}(x - c_i)                         (periodic)
 *   moments   m_a = sum_i T_ai f_i                              (Sec. III eq. moments)
 *   hydro     rho = m_0, rho u = j + F/2                        (Sec. V eq. lbe-moments)
 *   update    m*_a = m_a - lam_a (m_a - m^eq_a) + (1 - lam_a/2) m^F_a + xi_a
 *             lam_a = 0 for rho and j; <xi_a xi_b> = rho kT N_a lam_a (2 - lam_a)/cs2 delta_ab
 *                                                                (Sec. V eq. noise-lbe, Delta V = 1)
 *   back      S_{n+1,i}(x) = w_i sum_a T_ai m*_a / N_a          (Sec. III eq. moments-inv)
 * with cs2 = 1/3, the ideal-gas equilibrium moments of Sec. III eq. feq and the
 * second-order (Guo) forcing moments {0, F, uF + Fu, 0 on ghosts}.
 *
 * Non-ideal force (force_model = 1), evaluated on the density after streaming:
 *   mu = psi'(rho) - kappa lap_h rho,   psi = a (rho - rho_c)^2 + b (rho - rho_c)^4
 *   F  = -rho grad_h mu + eta cs2 grad_h rho
 *   grad_h phi = (1/cs2) sum_i w_i c_i phi(x + c_i),
 *   lap_h  phi = (2/cs2) sum_i w_i (phi(x + c_i) - phi(x))   (9- or 19-point)
 *
 * Noise: every non-conserved mode a (in basis order, k = a - d - 1) draws a
 * standard normal z_k from Philox4x32-10 (Salmon et al., SC'11) with counter
 * (site, step, block | tag << 16, replica) and key (seed mod 2^32, seed >> 32),
 * site = x + nx (y + ny z), tag = 0.  The words w_0, w_1, ... of blocks 0, 1, ...
 * feed P = ceil(K/2) Box-Muller pairs: pair p has radius
 * sqrt(-2 ln u), u = (w_p + 1) 2^-32 (in the run's precision), and angle
 * 2 pi (h + 1) 2^-16 with h the high (p even) or low (p odd) half of
 * w_{P + p/2}; z_{2p}, z_{2p+1} = radius (cos, sin) of the angle.  D3Q19 uses
 * 3 blocks per site-step, D2Q9 2.
 *
 * Storage: populations are stored shifted, delta f_i = f_i - w_i rho0, in
 * structure-of-arrays order f[i * V + site] (V = nx ny nz sites, x fastest),
 * in FP32 or FP64.  Statistics are accumulated in FP64.
 *
 * Conventions for every call:
 *  - Device buffers are allocated and owned by the caller; the library never
 *    allocates or frees device memory.  Pointers must be 256-byte aligned.
 *  - "stream" is a hipStream_t (NULL = the null stream).  Calls are
 *    stream-ordered and asynchronous unless stated otherwise.
 *  - Every call returns an flb_status; nothing throws across the ABI.
 *    flb_last_error() gives a text description of the last failure of the
 *    calling thread.
 *  - A handle is host-side state only; it is not thread-safe.
 */
#ifndef FLB_H
#define FLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FLB_OK = 0,
    FLB_ERR_INVALID_ARG = -1, /* a parameter, size or pointer was rejected     */
    FLB_ERR_HIP = -2,         /* a HIP runtime call failed                      */
    FLB_ERR_NONFINITE = -3,   /* a population or the statistics became NaN/Inf  */
    FLB_ERR_UNSUPPORTED = -4, /* combination not implemented                   */
    FLB_ERR_STATE = -5        /* call not valid in the handle's current state   */
} flb_status;

enum { FLB_D2Q9 = 0, FLB_D3Q19 = 1 };
enum { FLB_FP32 = 0, FLB_FP64 = 1 };
enum { FLB_IDEAL = 0, FLB_LANDAU = 1 };

/* Parameters of one run.  Rates are the lattice rates lam^LB in (0, 2)
 * (Sec. V: lam^LB = 2 lam / (2 + lam)), one per mode class of App. B:
 * bulk (trace of the stress), shear (traceless stress), ghost (all ghosts).
 * kT must satisfy 0 <= kT < rho0 cs2 (stability bound stated in Sec. VI.A). */
typedef struct flb_params {
    int32_t lattice;          /* FLB_D2Q9 or FLB_D3Q19                          */
    int32_t precision;        /* FLB_FP32 or FLB_FP64                           */
    int32_t nx, ny, nz;       /* periodic box; nz = 1 for D2Q9                  */
    int32_t force_model;      /* FLB_IDEAL or FLB_LANDAU                        */
    int32_t eta;              /* 0: F = -rho grad mu; 1: + cs2 grad rho         */
    int32_t noise_rho_local;  /* 1: noise variance uses local rho(x); 0: rho0   */
    double rho0;              /* reference density (> 0)                        */
    double kT;                /* fluctuation temperature                        */
    double rate_bulk, rate_shear, rate_ghost;
    double a, b, rho_c, kappa;/* Landau psi and square-gradient coefficient    */
    uint64_t seed;            /* Philox key                                     */
    uint64_t step0;           /* index of the first step (resume)               */
    uint32_t replica;         /* Philox counter word 3                          */
    uint32_t reserved;
} flb_params;

typedef struct flb_handle flb_handle;

/* Sizes (bytes) of the caller-allocated device buffers for parameters p:
 * pop_bytes for each of the two population buffers (Q V reals), scratch_bytes
 * for the work area (counters and, for the non-ideal fluid, the density and
 * adjoint fields; for the D3Q19 non-ideal fluid in FP32 also the next-step
 * density that the z-marching force step forms, V floats, and its x-segment
 * edge records, 64 B per 64 sites of a row), stats_bytes for the FP64
 * statistics partials.
 * Returns FLB_ERR_INVALID_ARG for invalid parameters (see flb_init). Host only. */
flb_status flb_query_sizes(const flb_params* p, size_t* pop_bytes, size_t* scratch_bytes,
                           size_t* stats_bytes);

/* Create a handle and write the initial state S_0,i(x) = w_i rho(x) (the u = 0
 * equilibrium of Sec. III eq. feq) into f_a, with rho = rho0 + drho_init[x]
 * (drho_init: device pointer to V doubles, or NULL for rho = rho0).  Clears the
 * statistics.  f_a, f_b, scratch and stats must have the sizes given by
 * flb_query_sizes and stay valid for the handle's life.
 * Rejects (FLB_ERR_INVALID_ARG): unknown lattice/precision/force model, sizes
 * < 1 or nz != 1 for D2Q9 or sites >= 2^31, rates outside (0, 2), kT < 0 or
 * kT >= rho0/3, rho0 <= 0, null or misaligned buffers. */
flb_status flb_init(const flb_params* p, void* f_a, void* f_b, void* scratch, void* stats,
                    const double* drho_init, void* stream, flb_handle** out);

/* Advance nsteps time steps of Sec. V eq. lbe-mom (each: pull, moments of
 * Sec. III eq. moments, relaxation with the forcing moments of Sec. V
 * eq. lbe-moments and the noise of eq. noise-lbe, back-transform of Sec. III
 * eq. moments-inv; the force of App. A eq. he-force for force_model 1).  If
 * stats_stride > 0, the pre-collision moments of every step k (0-based in
 * this call) with (k + 1) % stats_stride == 0 are accumulated into the FP64
 * statistics (sum and sum of squares per mode over sites, with m_0 taken as
 * rho - rho0): the equal-time mode variances that Sec. IV.A eq. G-ideal fixes.
 * Identical calls give identical bits.  With a launch shape that forms the
 * next step's density in the force step (flb_launch_shape shape[7] == 2), the
 * first step of a call (and of each flb_set_check chunk) takes its density
 * from a density pass and the later ones from the step's own sums, which
 * agree to FP32 rounding: splitting the same steps into other calls changes
 * the state at that level (every other shape gives the same bits however
 * the steps are split).
 * Returns FLB_ERR_INVALID_ARG for nsteps < 0 or stats_stride < 0 (nothing
 * queued), FLB_ERR_HIP if a launch fails.  Asynchronous. */
flb_status flb_step(flb_handle* h, int64_t nsteps, int32_t stats_stride, void* stream);

/* Failure detection.  Every step's collision sets a device flag of the
 * handle when the density it pulled at a site (the sum of the site's Q
 * populations after streaming, Sec. V eq. lbe-moments) is NaN or Inf, so a
 * non-finite population anywhere is seen within one step.  With every > 0,
 * flb_step runs its steps in chunks of `every`, reads the flag after each
 * chunk (synchronizing the stream) and returns FLB_ERR_NONFINITE as soon as
 * it is set, with the step counter at the end of that chunk; every = 0
 * (the default) turns the reads off, and flb_step stays asynchronous.  The
 * flag is sticky; this call clears it (asynchronously on `stream`).
 * FLB_ERR_INVALID_ARG for every < 0. */
flb_status flb_set_check(flb_handle* h, int64_t every, void* stream);

/* Current state: *cur receives the device buffer holding S_n, *other the
 * second buffer, *step the index n of the next step.  Host only. */
flb_status flb_state(const flb_handle* h, void** cur, void** other, uint64_t* step);

/* Set the index of the next step (e.g. after loading a checkpointed state
 * into the current buffer).  Asynchronous. */
flb_status flb_seek(flb_handle* h, uint64_t step, void* stream);

/* Finalize the statistics in a fixed order and copy them to the host:
 * mode_sum[Q], mode_sumsq[Q] (either may be NULL), *nsamples the number of
 * sampled steps.  Per mode a, sumsq / (nsamples V) - (sum / (nsamples V))^2
 * is the equal-time variance that the fluctuation-dissipation theorem fixes
 * at rho0 kT N_a / cs2 for the ideal gas (Sec. IV.A eq. G-ideal; the
 * per-mode equilibration ratio of Sec. VI.A).  Host arrays, caller-owned.
 * Synchronizes the stream.  Returns FLB_ERR_NONFINITE if a sum is not
 * finite (the outputs are still written). */
flb_status flb_moments(flb_handle* h, double* mode_sum, double* mode_sumsq, int64_t* nsamples,
                       void* stream);

/* Zero the statistics.  Asynchronous. */
flb_status flb_reset_stats(flb_handle* h, void* stream);

/* Hydrodynamic fields of the current state after streaming (Sec. V
 * eq. lbe-moments): out[0..V) = rho, out[(1 + a) V ..) = rho u_a for a < d,
 * rho u = sum_i c_i f_i + F/2, in the handle's precision (device pointer to
 * (1 + d) V reals).  Asynchronous. */
flb_status flb_fields(flb_handle* h, void* out, void* stream);

/* All Q mode densities of the current state after streaming, FP64 (Sec. III
 * eq. moments on the shifted populations): out[a V + s] = sum_i T_ai df_i(s),
 * so row 0 is rho - rho0, and the momentum rows 1..d are rho u = j + F/2
 * (Sec. V eq. lbe-moments).  out: device pointer to Q V doubles, caller-owned,
 * 8-byte aligned.  These are the fields whose equal-time correlations Sec. VI
 * compares with the theory.  Asynchronous. */
flb_status flb_mode_fields(flb_handle* h, double* out, void* stream);

/* Bytes of the device work buffer flb_mode_spectrum needs: 24 Q V. */
flb_status flb_spectrum_work_bytes(const flb_handle* h, size_t* bytes);

/* Equal-time mode spectra of the current state (the measurement of the
 * equilibration ratio of Sec. VI): with m_a(k) = sum_x m_a(x) exp(-i k.x) the
 * DFT of the flb_mode_fields rows, k = 2 pi (kx/nx, ky/ny, kz/nz),
 *   spec[a V + k]       += |m_a(k)|^2                      (a < Q)
 *   spec[(Q + p) V + k] += Re(m_{1+al}(k) conj m_{1+be}(k))  (momentum pairs)
 * with k = kx + nx (ky + ny kz) and the pairs p = (al, be) = (x, y) for D2Q9,
 * (x, y), (y, z), (z, x) for D3Q19.  spec: device, (Q + 1) V doubles (D2Q9) or
 * (Q + 3) V (D3Q19), caller-owned and caller-zeroed; calls add to it, so a
 * sum over snapshots is one buffer.  work: device, flb_spectrum_work_bytes,
 * 256-byte aligned, contents not kept.  FLB_ERR_UNSUPPORTED if an extent
 * exceeds 1024.  Asynchronous. */
flb_status flb_mode_spectrum(flb_handle* h, void* work, double* spec, void* stream);

/* Power spectra of real fields: for f = 0 .. nfields - 1,
 *   spec[f V + k] += |sum_x fields[f V + x] exp(-i k.x)|^2,
 * x and k laid out as sites (x fastest), V = nx ny nz, periodic, direct DFT
 * along each axis.  Used for interface-height spectra (Sec. VI capillary
 * fluctuations, eq. capill-static).  fields, spec: device doubles, 8-byte
 * aligned, caller-owned (spec caller-zeroed; calls add to it).  work: device,
 * 16 nfields V bytes, 256-byte aligned.  FLB_ERR_UNSUPPORTED if an extent
 * exceeds 1024.  Asynchronous. */
flb_status flb_field_spectrum(const double* fields, int32_t nfields, int32_t nx, int32_t ny,
                              int32_t nz, void* work, double* spec, void* stream);

/* One planar interface across the profile axis (y for D2Q9, z for D3Q19). */
typedef struct {
    double y_ref;        /* approximate position along the profile axis, in [0, n) */
    int32_t sign;        /* +1: the density rises from rho_V to rho_L as y grows; -1: falls */
    int32_t half_window; /* the fit uses the 2 W + 1 sites y0 - W .. y0 + W, y0 =
                            floor(y_ref + 1/2), read periodically; 1 <= W, 2 W + 1 <= n */
} flb_interface;

/* Local interface heights of the current state (Sec. VI, capillary
 * fluctuations; eq. height-def): for every column (x for D2Q9, x + nx y for
 * D3Q19) and interface j, the h that minimizes
 *   sum_{y in window} (rho(y) - rho_MF(y - h))^2,
 *   rho_MF(u) = (rho_L + rho_V)/2 + sign (rho_L - rho_V)/2 tanh(2 u / width)
 * (the mean-field profile of eq. denprof), rho the density after streaming;
 * Gauss-Newton from y0, clamped to the window.  h is in the window's unwrapped
 * coordinate.  heights: device, n_if x ncol doubles (interface-major),
 * caller-owned.  Needs force_model = 1 (FLB_ERR_UNSUPPORTED otherwise); at most
 * 8 interfaces.  Uses the handle's density scratch.  Asynchronous. */
flb_status flb_interface_heights(flb_handle* h, const flb_interface* ifs, int32_t n_if,
                                 double rho_L, double rho_V, double width, double* heights,
                                 void* stream);

/* ----------------------------------------------------------------------
 * Modified-equilibrium (Swift) model, linearized about rest, D2Q9
 * (Sec. IV.B, subsection on the modified-equilibrium model).
 *
 * State: deviations delta f_i from the uniform rest state, f[i * V + x + nx y]
 * (V = nx ny), reals of `precision`.  One step with index n:
 *   pull f_i(x) = S_i(x - c_i); m = T f (App. B basis: rho, j_x, j_y, e, p_xx,
 *   p_xy, q_x, q_y, eps); linearized equilibrium of eq. meq-yeo
 *     m^eq = {rho, j_x, j_y, D, 0, 0, 0, 0, -D},
 *     D = 6 (cs2_0 - 1/3) rho - 6 kappa rho0 lap_h rho   (= d(k) rho,
 *     d(k) = 6 (c_s^2(k) - 1/3), c_s^2(k) = cs2_0 + kappa rho0 Lambda(k),
 *     Lambda the symbol of -lap_h; S(k) = rho0 kT / c_s^2(k), eq. s-nonideal);
 *   m*_a = m_a - lam_a (m_a - m^eq_a) + xi_a;  S_{n+1} = w_i sum_a T_ai m*_a / N_a.
 * Noise: covariance Xi(k) = G - C G C^T, G the equal-time correlations of
 * eq. f-correl-yeo, C the collision matrix: white on p_xx, p_xy, q_x, q_y
 * (rho0 kT N_a lam (2 - lam) / cs2, normals z_1..z_4 of the site), and for
 * (e, eps), with c2 = c_s^2(k), lam_e = rate_bulk, lam_g = rate_ghost,
 *   Xi_ee = 12 rho0 kT lam_e (2 - lam_e)(2 - 3 c2),
 *   Xi_eE = 12 rho0 kT (3 c2 - 1)(lam_e + lam_g - lam_e lam_g),
 *   Xi_EE = 12 rho0 kT lam_g (2 - lam_g)(5 - 3 c2),
 * drawn as xi = IDFT[L(k) DFT[z_0, z_5]], L the lower Cholesky factor, z the
 * site normals of the force-based step (Philox counter (site, n, block, 0),
 * tag 0, replica 0).  Its small-rate limit is eq. noise-yeo with the (e, eps)
 * entry at half its printed value (the value for which Xi is a covariance
 * wherever the equilibrium populations are non-negative).
 * --------------------------------------------------------------------- */
typedef struct flb_modeq_params {
    int32_t nx, ny;       /* periodic lattice, each in [1, 1024]                        */
    int32_t precision;    /* FLB_FP32 or FLB_FP64: state, step arithmetic and the noise
                             transforms and fields                                       */
    int32_t reserved;     /* 0                                                          */
    double rho0;          /* > 0                                                        */
    double kT;            /* >= 0; 0 runs the deterministic step and needs no work      */
    double cs2_0;         /* c_s^2 at k = 0, > 0                                        */
    double kappa;         /* >= 0, with cs2_0 + kappa rho0 16/3 <= 0.6                  */
    double rate_bulk, rate_shear, rate_ghost;   /* lam^LB in (0, 2); ghost = q and eps  */
    uint64_t seed;        /* Philox key                                                 */
} flb_modeq_params;

/* Minimum device work bytes of flb_modeq_step / _run / _noise: per step of
 * a noise batch the two complex noise spectra and the two filtered fields,
 * 24 V bytes in FP32 and 48 V in FP64.  Rejects invalid parameters
 * (FLB_ERR_INVALID_ARG), including rates for which the (e, eps) covariance
 * is not positive semidefinite somewhere on [cs2_0, cs2_0 + kappa rho0 16/3]. */
flb_status flb_modeq_work_bytes(const flb_modeq_params* p, size_t* bytes);

/* One step with index `step` from fin to fout (distinct, device, 256-byte
 * aligned, 9 V reals each).  `work` (device, 256-byte aligned, at least
 * flb_modeq_work_bytes) is overwritten; it may be NULL when kT = 0.
 * Asynchronous on `stream`. */
flb_status flb_modeq_step(const flb_modeq_params* p, const void* fin, void* fout, uint64_t step,
                          void* work, size_t work_bytes, void* stream);

/* nsteps steps with indices step0 .. step0 + nsteps - 1; the result is in f,
 * tmp (device, 9 V reals) is overwritten.  The noise of consecutive steps is
 * drawn and filtered in batches of b = min(16, work_bytes / w) steps, w the
 * per-step bytes of flb_modeq_work_bytes
 * (one launch set per batch; a larger work buffer fills more of the chip at
 * small lattices).  The result does not depend on b. */
flb_status flb_modeq_run(const flb_modeq_params* p, void* f, void* tmp, uint64_t step0,
                         int32_t nsteps, void* work, size_t work_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step as flb_modeq_step, bit for bit, with the noise work taken from a fixed
 * device array inside the library instead of a caller buffer.  The array
 * holds flb_modeq_static_work_bytes() bytes (16 MiB) on each GPU the library
 * runs on, from its first use there until the process ends, so the step
 * needs 24 V <= 16 MiB in FP32 (V <= 699050 sites, e.g. 1024 x 512) and
 * 48 V <= 16 MiB in FP64 (V <= 349525, e.g. 512 x 512); kT = 0 needs no
 * work and has no limit; larger lattices are rejected with
 * FLB_ERR_INVALID_ARG before anything is queued.  fin, fout as for
 * flb_modeq_step.  Calls no allocator.  Every call on a GPU uses that GPU's
 * one array: calls that overlap on one GPU (other streams, other threads)
 * race and must be ordered by the caller.  Asynchronous on `stream`. */
flb_status flb_modeq_step_noalloc(const flb_modeq_params* p, const void* fin, void* fout,
                                  uint64_t step, void* stream);
/* Size in bytes of that fixed array.  Host only. */
flb_status flb_modeq_static_work_bytes(size_t* bytes);

/* Analysis: the moment fields of the pulled populations of state f,
 * m[a * V + site] = sum_i T_ai f_i(x - c_i) (device, FP64, 9 V), the modes
 * whose equal-time spectra eq. f-correl-yeo fixes.  Asynchronous. */
flb_status flb_modeq_moments(const flb_modeq_params* p, const void* f, double* m, void* stream);

/* Verification: the filtered (e, eps) noise of step `step`, xi[0 .. V) = xi_e,
 * xi[V .. 2V) = xi_eps (device, reals of p->precision). */
flb_status flb_modeq_noise(const flb_modeq_params* p, uint64_t step, void* xi, void* work,
                           size_t work_bytes, void* stream);

/* Verification: the raw Philox4x32-10 words the step draws for noise block
 * `block` (tag `tag`) at step `step` for sites site0 .. site0 + nsites - 1,
 * written to out_dev[4 * s + k] (device, uint32).  Uses p->seed and
 * p->replica.  Asynchronous. */
flb_status flb_noise_words(const flb_params* p, uint64_t step, uint32_t block, uint32_t tag,
                           uint64_t site0, uint64_t nsites, uint32_t* out_dev, void* stream);

/* Verification: the standard normals the collision of step `step` draws at
 * sites site0 .. site0 + nsites - 1 (Sec. V eq. noise-lbe: the xi_a are these
 * normals times the per-mode amplitudes), written to out_dev[2 P s + k]
 * (device, reals of p->precision), P = 8 Box-Muller pairs for D3Q19 and 3 for
 * D2Q9: z[2j], z[2j+1] = R (cos theta, sin theta) of pair j, with R from word
 * j and theta from half of word P + j/2 of the site's Philox blocks (the
 * layout flb_noise_words exposes); the collision uses the first 15 (D3Q19) or
 * 6 (D2Q9).  Uses p->seed and p->replica.  Asynchronous. */
flb_status flb_noise_normals(const flb_params* p, uint64_t step, uint64_t site0, uint64_t nsites,
                             void* out_dev, void* stream);

/* Verification: the library's constant tables for a lattice, written to host
 * arrays: c[3 Q] (int, z = 0 in 2-D), w[Q], T[Q Q] (row-major, rows = modes),
 * N[Q], cls[Q] (0 rho, 1 momentum, 2 bulk, 3 shear, 4 ghost); *q receives Q.
 * Any output may be NULL.  Host only. */
flb_status flb_lattice_tables(int32_t lattice, int32_t* q, int32_t* c, double* w, double* T,
                              double* N, int32_t* cls);

/* Record nsteps steps (same meaning as flb_step; nsteps even, stream not
 * NULL) into HIP graphs owned by the handle, replacing any previous ones: one
 * recording for each of the two population buffers the state can start
 * from, so a replay continues the state after any number of ordinary steps.
 * The step index is read from device memory, so every replay continues the
 * noise sequence.  Nothing runs. */
flb_status flb_graph_capture(flb_handle* h, int64_t nsteps, int32_t stats_stride, void* stream);

/* Replay the captured steps once from the current buffer (advances the
 * state by their nsteps).  FLB_ERR_STATE if nothing was captured. */
flb_status flb_graph_launch(flb_handle* h, void* stream);

/* Adjoint of one time step (reverse mode), for the gradient of a scalar loss.
 * Given S_n = s_n (device, Q V reals, shifted populations: the state the step
 * with index n starts from) and abar_np1 = dL/dS_{n+1} (device, Q V reals),
 * writes abar_n = dL/dS_n (device, Q V reals; must not alias the inputs) and
 * accumulates the parameter derivatives of this step, with the same noise
 * (regenerated from Philox), into FP64 device accumulators.  If grad is not
 * NULL the accumulators are finalized and ADDED to grad[4] on the host
 * (order: d/d rate_shear, d/d kT, d/d rate_bulk, d/d rate_ghost) and cleared;
 * that form synchronizes the stream.  FP32 and FP64, ideal and Landau force
 * (eta = 0 or 1).  Returns FLB_ERR_INVALID_ARG if kT > 0 is required for the
 * kT derivative and kT == 0 (the derivative is then reported as 0). */
flb_status flb_adjoint_step(flb_handle* h, const void* s_n, const void* abar_np1, void* abar_n,
                            double* grad, uint64_t n, void* stream);

/* Reverse pass over one checkpoint segment [k0, k1) in a single call: the
 * states S_{k0+1} .. S_{k1-1} are recomputed from s_k0 (device, the state the
 * step with index k0 starts from) with the forward kernels and kept in `work`
 * (device, flb_adjoint_segment_bytes(h, k1 - k0) bytes, 256-byte aligned),
 * together with their densities for the force model; then the adjoint step is
 * applied for n = k1 - 1 down to k0.  abar (device, Q V reals) holds
 * dL/dS_{k1} on entry and dL/dS_{k0} on return.  Parameter derivatives are
 * accumulated as in flb_adjoint_step; grad (host, nullable) behaves the same.
 * Does not touch the handle's state buffers or step counter. */
flb_status flb_adjoint_segment(flb_handle* h, const void* s_k0, void* abar, void* work,
                               uint64_t k0, uint64_t k1, double* grad, void* stream);
flb_status flb_adjoint_segment_bytes(const flb_handle* h, int64_t nsteps, size_t* bytes);

/* Reverse pass over a whole checkpointed run in one call: steps 0 .. nsteps-1
 * in nseg segments of seg_len steps (the last may be shorter), ckpts[s]
 * (host array of device pointers, Q V reals each) holding the state the step
 * with index s * seg_len starts from.  abar (device, Q V reals) holds
 * dL/dS_{nsteps} on entry and dL/dS_0 on return; parameter derivatives as in
 * flb_adjoint_segment, grad (host, nullable) added to at the end.  The
 * results equal those of flb_adjoint_segment called for the segments from
 * last to first; the difference is scheduling: the recompute of segment
 * s - 1 runs on a helper stream of the handle (created on first use, default
 * priority) while the reverse sweep of segment s runs on `stream`, the two
 * halves of `work` (device, flb_adjoint_run_bytes(h, seg_len) bytes, 256-byte
 * aligned) alternating under events.  Work the caller queued on `stream`
 * before the call is complete before anything of it starts; when it returns
 * (without grad: asynchronously) everything it queued is ordered before later
 * work on `stream`. */
flb_status flb_adjoint_run(flb_handle* h, const void* const* ckpts, int32_t nseg,
                           int64_t seg_len, int64_t nsteps, void* abar, void* work,
                           double* grad, void* stream);
flb_status flb_adjoint_run_bytes(const flb_handle* h, int64_t seg_len, size_t* bytes);

/* Adjoint seed of the loss of the final density: given S_N (device) and
 * rhobar[V] = dL/drho_N (device, handle precision), where
 * rho_N(x) = rho0 + sum_i delta S_{N,i}(x - c_i), writes abar_N = dL/dS_N
 * (device, Q V reals): abar_{N,i}(y) = rhobar(y + c_i).  Asynchronous. */
flb_status flb_adjoint_density_seed(flb_handle* h, const void* rhobar, void* abar_N,
                                    void* stream);

/* Density after streaming of an arbitrary state s (device, Q V reals):
 * out[x] = sum_i delta s_i(x - c_i) (= rho(x) - rho0), handle precision. */
flb_status flb_density(flb_handle* h, const void* s, void* out, void* stream);

/* Release the handle (host memory and any captured graph). */
flb_status flb_destroy(flb_handle* h);

/* ---------------------------------------------------------------------------
 * Batched replicas: R independent lattices (same lattice type, precision and
 * physical parameters, each with its own box and seed) advanced by one
 * persistent launch per step over a flattened tile table.  Replica r uses
 * Philox key seeds[r] and counter word 3 = r; its populations occupy
 * Q V_r consecutive reals starting at element offset Q * sum_{s<r} V_s of
 * each population buffer (replica-major, then SoA within the replica).
 * Statistics buffer: a table of per-chunk sums (2Q x chunks FP64, a chunk
 * being up to 8 tiles of 256 sites of one replica; each sampled step of a
 * call adds to it) followed by the per-replica FP64 accumulators (R x 2Q), to
 * which the end of each call (flb_batch_step, a graph replay) adds the sums
 * over the replica's chunks, clearing the table.
 * -------------------------------------------------------------------------*/
typedef struct flb_batch flb_batch;

/* dims[3 r + 0..2] = (nx, ny, nz) of replica r.  Host only. */
flb_status flb_batch_query_sizes(const flb_params* base, int32_t nrep, const int32_t* dims,
                                 size_t* pop_bytes, size_t* scratch_bytes, size_t* stats_bytes);

/* Initial state w_i rho0 in every replica; ideal gas only (force_model 0). */
flb_status flb_batch_init(const flb_params* base, int32_t nrep, const int32_t* dims,
                          const uint64_t* seeds, void* f_a, void* f_b, void* scratch,
                          void* stats, void* stream, flb_batch** out);

flb_status flb_batch_step(flb_batch* b, int64_t nsteps, int32_t stats_stride, void* stream);

/* Per-replica statistics: mode_sum[r Q + a], mode_sumsq[r Q + a]; synchronizes. */
flb_status flb_batch_moments(flb_batch* b, double* mode_sum, double* mode_sumsq,
                             int64_t* nsamples, void* stream);

/* Zero the per-replica statistics and the sample count.  Asynchronous. */
flb_status flb_batch_reset_stats(flb_batch* b, void* stream);

flb_status flb_batch_state(const flb_batch* b, void** cur, void** other, uint64_t* step);
/* As flb_graph_capture / flb_graph_launch, for the batch (one recording per
 * current buffer; the schedule in force at capture is kept). */
flb_status flb_batch_graph_capture(flb_batch* b, int64_t nsteps, int32_t stats_stride,
                                   void* stream);
flb_status flb_batch_graph_launch(flb_batch* b, void* stream);
flb_status flb_batch_destroy(flb_batch* b);

/* Launch shapes in use and autotuning.  A handle keeps a launch shape for
 * steps without statistics, one for steps that accumulate them and, for the
 * ideal gas, optionally an in-place shape: consecutive pairs of steps then
 * run in place on the current population buffer (the first step of a pair
 * pulls and stores each result in the opposite-velocity plane at x + c_i, the
 * second reads that plane locally and restores the ordinary layout), which
 * halves the working set; populations, statistics and noise are bit-identical
 * to ordinary steps, and a lone last step of a call runs the ordinary kernel.
 * flb_autotune times every candidate launch shape of the handle's step kernel
 * (block size, sites per thread, store hints, in-place pairs; tile or
 * z-marching shape for the force kernel, and for the D3Q19 force step in FP32
 * z-marching shapes that form the next step's density themselves (the
 * populations of Sec. V eq. lbe-mom after collision, summed over c_i as
 * streaming delivers them: in-tile sources through LDS and wavefront shifts,
 * the rest added by a completion pass), so that only the first step of a
 * call runs a density pass; the trials time steady steps, so for calls of a
 * few steps the plain march of the same tile, which needs no such first
 * pass, can be the faster choice) the way a run uses it (ordinary
 * steps alternate the two buffers over `repeats` steps; in-place pairs are
 * timed after about 4 ms of settling steps, round-robin over at least three
 * rounds of about 2 ms each, best round kept) and afterwards
 * restores the state and the accumulated statistics from a host copy (host
 * memory of one population buffer plus the statistics slots); it writes
 * best[4]: the fastest shape for plain steps, for steps with statistics, the
 * fastest in-place shape (-1 if none) and the in-place shape now in use (-1:
 * pairs are used only if they beat ordinary steps with statistics); and
 * best_ms[3]: ms per step of the first three (either pointer may be NULL).
 * The statistics trials run on the handle's own slots, saved to host memory
 * before and restored after; the call synchronizes the stream.
 * Until then a handle uses shape 0, except D2Q9 force steps, which use
 * shape 4 (32 x 8, forming its own density tile).
 * flb_set_launch sets every shape to `config` (an in-place shape then serves
 * pairs and, as an ordinary kernel of its tile, lone steps);
 * flb_launch_configs writes the number of shapes and current[3] (plain, with
 * statistics, in-place or -1). */
flb_status flb_autotune(flb_handle* h, int32_t repeats, int32_t* best, double* best_ms,
                        void* stream);
flb_status flb_set_launch(flb_handle* h, int32_t config);
flb_status flb_launch_configs(const flb_handle* h, int32_t* count, int32_t* current);
/* shape[8] = threads per block in x, y, z, sites per thread (stacked in y),
 * 1 if populations are stored with non-temporal hints, the number of z planes
 * a block sweeps (z-marching force step; 0 otherwise), 1 for an in-place
 * shape, and 1 for a force step that forms its density tile from the
 * populations itself (no density pass before it; D2Q9), 2 for a z-marching
 * force step that forms the next step's density (D3Q19, FP32; in FP64 such a
 * shape runs the plain march of its tile). */
flb_status flb_launch_shape(const flb_handle* h, int32_t config, int32_t* shape);
/* The same for a batch: the candidates are persistent grids of 8, 4, 16 or 2
 * blocks per compute unit; best[2] / best_ms[2] as for flb_autotune.  It then
 * times in-place pairs group by group (flb_batch_set_pairs) with groups of up
 * to 64, 128, 160, 192, 224, 256 and 320 MiB on each of the four grids, with statistics, and keeps
 * the fastest (budget and grid) if it beats
 * the ordinary step with statistics (else turns pairs off).  The statistics
 * trials add only to the per-chunk table, which is clear between calls and
 * cleared again afterwards, so the accumulated statistics are unchanged;
 * the pair trials run on a copy
 * of the state in the other buffer, so the state is unchanged.
 * Synchronizes. */
flb_status flb_batch_autotune(flb_batch* b, int32_t repeats, int32_t* best, double* best_ms,
                              void* stream);

/* Schedule of the batch's steps.  pair_bytes = 0: every step advances all
 * replicas, alternating the two buffers.  pair_bytes > 0: consecutive
 * replicas are grouped up to pair_bytes of populations (a larger replica is a
 * group of its own) and each group is taken through all the steps of a call
 * (flb_batch_step, or the steps recorded by flb_batch_graph_capture) before
 * the next, pairs of steps in place in one buffer (the layout of
 * flb_step's in-place pairs), a last odd step in the ordinary way; a group
 * small enough to stay in the last-level cache runs faster.  The noise counters
 * are global, so states and statistics are bitwise the same in either
 * schedule.  A graph captured earlier keeps the schedule it was captured
 * with.  Host only. */
flb_status flb_batch_set_pairs(flb_batch* b, uint64_t pair_bytes);
/* The current pair_bytes and number of groups (0 when off).  Host only. */
flb_status flb_batch_pairs(const flb_batch* b, uint64_t* pair_bytes, int32_t* ngroups);

/* Calibration of the HBM roofline of the step kernels: `repeats` launches
 * that each read q FP32 planes of V elements (plane stride V, the population
 * layout) and write them back scaled by 1, one thread per site, to b (b = a:
 * in place, the pattern of an in-place pair; b != a: the two-buffer
 * pattern).  Moves 8 q V bytes per launch and does no arithmetic of the
 * method.  a, b: device, 4 q V bytes each.  FLB_ERR_INVALID_ARG unless q is 9
 * or 19, 0 < V < 2^31 and repeats >= 1.  Asynchronous. */
flb_status flb_plane_stream_probe(const void* a, void* b, int32_t q, uint64_t V, int32_t repeats,
                                  void* stream);

/* Text of a status code; last error text (thread-local) with HIP details. */
const char* flb_strerror(flb_status s);
const char* flb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FLB_H */
