// Host-side interface between the C ABI (api.hip) and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flb {

// Launch shapes of the step kernels: tile TX x TY x TZ sites, one site per thread.
struct TileShape {
    int tx, ty, tz;   // threads per block in x, y, z
    int spt;          // sites per thread, stacked in y: the site tile is tx x (ty spt) x tz
    int nt;           // 1: populations are stored with non-temporal hints
    int zc;           // > 0: the block sweeps zc planes in z (D3Q19 force step), tz = 1
    int ip;           // 1: in-place step pairs in one buffer (ideal gas); a lone
                      //    step runs the ordinary kernel of the same tile
    int fd;           // 1: the force step forms the staged density tile from the
                      //    populations itself (no density pass; D2Q9)
    int pd;           // 1: the z-marching force step also forms the next step's
                      //    density from its own sources (FP32), completed by
                      //    launch_density_fix (no density pass between steps)
};

// Candidate tiles (the autotuner picks one per handle).
constexpr int N_IDEAL_CFG = 15;
constexpr TileShape IDEAL_CFG[N_IDEAL_CFG] = {
    {64, 4, 1, 1, 0},  {128, 2, 1, 1, 0}, {256, 1, 1, 1, 0}, {32, 8, 1, 1, 0},
    {128, 2, 1, 2, 0}, {64, 4, 1, 2, 0},  {128, 2, 1, 4, 0}, {256, 1, 1, 2, 0},
    {128, 2, 1, 1, 1}, {256, 1, 1, 1, 1}, {128, 2, 1, 1, 0, 0, 1}, {64, 4, 1, 1, 0, 0, 1},
    {256, 1, 1, 1, 0, 0, 1}, {128, 2, 1, 2, 0, 0, 1}, {64, 4, 1, 2, 0, 0, 1}};
constexpr int N_FORCE3_CFG = 12;
constexpr TileShape FORCE3_CFG[N_FORCE3_CFG] = {
    {32, 4, 2, 1, 0},     {16, 4, 4, 1, 0},     {64, 2, 2, 1, 0},
    {64, 4, 1, 1, 0, 16}, {64, 4, 1, 1, 0, 32}, {32, 8, 1, 1, 0, 16},
    {64, 8, 1, 1, 0, 16}, {128, 2, 1, 1, 0, 16}, {128, 2, 1, 1, 1, 16},
    {128, 2, 1, 1, 1, 16, 0, 0, 1}, {64, 4, 1, 1, 0, 16, 0, 0, 1},
    {64, 8, 1, 1, 0, 16, 0, 0, 1}};
constexpr int N_FORCE2_CFG = 6;
constexpr TileShape FORCE2_CFG[N_FORCE2_CFG] = {
    {64, 4, 1, 1, 0},          {32, 8, 1, 1, 0},          {128, 2, 1, 1, 0},
    {64, 4, 1, 1, 0, 0, 0, 1}, {32, 8, 1, 1, 0, 0, 0, 1}, {128, 2, 1, 1, 0, 0, 0, 1}};

// Everything a forward launch needs, in FP64 on the host (converted per precision).
struct StepSpec {
    int lat;           // 0 D2Q9, 1 D3Q19
    int prec;          // 0 FP32, 1 FP64
    int force;         // 0 ideal, 1 Landau
    int nx, ny, nz;
    double rho0, kT, lam_bulk, lam_shear, lam_ghost;
    double amp_cls[3];   // sqrt(kT lam (2 - lam) / cs2) for the bulk, shear and ghost rates
    int noise_on, noise_local;
    uint32_t key0, key1, replica;
    double a, b, rho_c, kappa, eta;
    uint32_t* nonfinite;   // device flag the collision sets on a non-finite density, or null
};

// Record the text returned by flb_last_error() (api.hip).
void set_last_error(const char* msg);

int n_configs(int lat, int force);
TileShape config_shape(int lat, int force, int cfg);
uint32_t config_blocks(const StepSpec& s, int cfg);

hipError_t launch_init(const StepSpec& s, void* f, const double* drho, hipStream_t st);
hipError_t launch_density(const StepSpec& s, const void* fin, void* drho_out, hipStream_t st);
// One step fin -> fout.  drho: density field of fin after streaming (force only).
// step_dev/step_host: step index (device counter + offset).  partial: stats slots or null.
// rho_out: for the force shapes that form their own density tile
// (config_fused), if non-null, receives fin's density field, the bits
// launch_density would write; ignored otherwise.
// rho_part: for the partial-density shapes (config_partial_density), if
// non-null, receives the part of fout's density that the march forms; null
// runs the plain march of the same shape.
hipError_t launch_step(const StepSpec& s, int cfg, const void* fin, void* fout, const void* drho,
                       const unsigned long long* step_dev, unsigned long long step_host,
                       double* partial, hipStream_t st, void* rho_out = nullptr,
                       void* rho_part = nullptr);
// Partial-density shapes: the density of fin after streaming from the
// march's rho_part (the step fin was written by, same shape) and the
// populations of fin whose sources lie outside the forming block.
bool config_partial_density(const StepSpec& s, int cfg);
// Bytes of the partial-density work area (the partial density and the
// march's edge records; 0 where no shape forms a partial density).
size_t partial_density_bytes(const StepSpec& s);
hipError_t launch_density_fix(const StepSpec& s, int cfg, const void* fin, const void* rho_part,
                              void* out, hipStream_t st);
// In-place shapes: one step of a pair on the single buffer f (phase 0 then 1;
// see push_rows_opp).  The state is in the ordinary layout after phase 1.
bool config_in_place(const StepSpec& s, int cfg);
// Force shapes whose step needs no density pass before it.
bool config_fused(const StepSpec& s, int cfg);
hipError_t launch_step_in_place(const StepSpec& s, int cfg, int phase, void* f,
                                const unsigned long long* step_dev, unsigned long long step_host,
                                double* partial, hipStream_t st);
hipError_t launch_fields(const StepSpec& s, const void* fin, const void* drho, void* out,
                         hipStream_t st);
// All Q mode densities of fin after streaming (FP64, out[a V + s]); momentum
// rows are j + F/2.  drho as for launch_fields.
hipError_t launch_mode_fields(const StepSpec& s, const void* fin, const void* drho, double* out,
                              hipStream_t st);
hipError_t launch_stats_finalize(const double* partial, uint32_t nslots, int nvals, double* out,
                                 hipStream_t st);
hipError_t launch_noise_words(const StepSpec& s, unsigned long long step, uint32_t block,
                              uint32_t tag, unsigned long long site0, unsigned long long nsites,
                              uint32_t* out, hipStream_t st);
hipError_t launch_noise_normals(const StepSpec& s, unsigned long long step,
                                unsigned long long site0, unsigned long long nsites, void* out,
                                hipStream_t st);
hipError_t launch_add_u64(unsigned long long* ctr, unsigned long long inc, hipStream_t st);
hipError_t launch_set_u64(unsigned long long* ctr, unsigned long long v, hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);

// Mode spectra (spectrum.hip).  fields: q real fields of nx ny nz sites;
// work: q V complex; spec: (q + npairs) V doubles, added to; npairs momentum
// cross spectra (rows 1..3 of fields), 0 for plain power spectra.
constexpr int SPECTRUM_MAX_N = 1024;
hipError_t launch_spectrum(int q, int npairs, int nx, int ny, int nz, const double* fields,
                           void* work, double* spec, hipStream_t st);
// Interface heights: up to 8 interfaces, window centre y0 = floor(y_ref + 1/2).
constexpr int MAX_INTERFACES = 8;
struct InterfaceSet {
    int n;
    int y0[MAX_INTERFACES];
    int sign[MAX_INTERFACES];
    int half_window[MAX_INTERFACES];
};
hipError_t launch_interface_heights(int prec, const void* drho, double rho0, int n, long ncol,
                                    const InterfaceSet& set, double rho_L, double rho_V,
                                    double width, double* out, hipStream_t st);

// Linearized modified-equilibrium model (modeq.hip), D2Q9.
struct ModEqArgs {
    int nx, ny;
    int prec;            // 0 FP32, 1 FP64: the state, the noise transforms and fields
    double rho0, kT, cs2_0, kappa;
    double rate_bulk, rate_shear, rate_ghost;
    uint32_t k0, k1;     // Philox key
    double amp[4];       // white-noise amplitudes of p_xx, p_xy, q_x, q_y
};
// Work per step of a noise batch, in the state's precision (prec 0 FP32,
// 1 FP64): the two complex noise spectra (2 V complex values) and the
// filtered noise fields xi_e, xi_eps (2 V reals): 24 V bytes in FP32, 48 V
// in FP64.
constexpr int MODEQ_MAX_BATCH = 16;
size_t modeq_work_bytes(int nx, int ny, int prec);
// The noise of steps step0 .. step0 + nb - 1: spectra of step b at
// W + 2 V b (complex), filtered fields at xi + 2 V b (reals of prec).
hipError_t launch_modeq_noise(const ModEqArgs& a, int prec, uint32_t step0, int nb, void* W,
                              void* xi, hipStream_t st);
// Moment fields of the pulled populations, FP64, m[a * V + site].
hipError_t launch_modeq_moments(const ModEqArgs& a, int prec, const void* fin, double* m,
                                hipStream_t st);
// One step; xi = that step's filtered fields, or null for kT = 0.
hipError_t launch_modeq_step(const ModEqArgs& a, int prec, const void* fin, void* fout,
                             uint32_t step, const void* xi, hipStream_t st);

// Adjoint launchers (adjoint.hip).
hipError_t launch_adjoint_seed(const StepSpec& s, const void* rhobar, void* abar, hipStream_t st);
struct AdjointStepArgs {
    const void* s_n;         // state S_n
    const void* drho;        // density of S_n after streaming (force model)
    const void* abar_np1;    // dL/dS_{n+1}, less the pending spread of rb_in
    void* abar_n;            // out: dL/dS_n, less the spread of rb_out unless spread
    void* work;              // adjoint_work_bytes: Fbar planes, two rhobar planes
    int rb_in;               // rhobar plane (0/1) still to be spread into abar_np1, or -1
    int rb_out;              // rhobar plane (0/1) this step writes
    bool spread;             // spread rb_out into abar_n now
    unsigned long long step;
    double* gpartial;        // per-block parameter-derivative slots (added to)
    const void* drho_next;   // D2Q9 force: density of S_{n+1} when rb_in >= 0 (the
                             //   pending rhobar is formed from its Fbar set rb_in)
};
hipError_t launch_adjoint_step(const StepSpec& s, const AdjointStepArgs& a, hipStream_t st);
// abar_i(y) += rhobar(y + c_i) from rhobar plane rb of the work space (D2Q9
// force: rhobar formed first from Fbar set rb and the density drho).
hipError_t launch_adjoint_spread(const StepSpec& s, void* work, int rb, const void* drho,
                                 void* abar, hipStream_t st);
size_t adjoint_work_bytes(const StepSpec& s);
uint32_t adjoint_slots(const StepSpec& s);

}  // namespace flb
