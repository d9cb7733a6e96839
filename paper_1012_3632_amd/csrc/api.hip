// C ABI of the fluctuating LB library (declarations and contracts in
// include/flb.h).  Host-side state only: the caller owns every device buffer.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <string>
#include <algorithm>
#include <vector>

#include "../../include/flb.h"
#include "internal.h"
#include "lattice.h"

using namespace flb;

namespace {

thread_local std::string g_last_error;

flb_status fail(flb_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(FLB_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

constexpr double CS2 = 1.0 / 3.0;
constexpr size_t ALIGN = 256;
constexpr size_t SCRATCH_HEADER = 256;   // step counter for graph replays, non-finite flag
constexpr size_t NONFINITE_OFF = 64;     // byte offset of the non-finite flag in the header

int lattice_q(int lat) { return lat == FLB_D2Q9 ? 9 : 19; }
int lattice_d(int lat) { return lat == FLB_D2Q9 ? 2 : 3; }

flb_status validate(const flb_params* p) {
    if (!p) return fail(FLB_ERR_INVALID_ARG, "params is NULL");
    if (p->lattice != FLB_D2Q9 && p->lattice != FLB_D3Q19)
        return fail(FLB_ERR_INVALID_ARG, "unknown lattice %d", p->lattice);
    if (p->precision != FLB_FP32 && p->precision != FLB_FP64)
        return fail(FLB_ERR_INVALID_ARG, "unknown precision %d", p->precision);
    if (p->force_model != FLB_IDEAL && p->force_model != FLB_LANDAU)
        return fail(FLB_ERR_INVALID_ARG, "unknown force model %d", p->force_model);
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(FLB_ERR_INVALID_ARG, "box %d x %d x %d", p->nx, p->ny, p->nz);
    if (p->lattice == FLB_D2Q9 && p->nz != 1)
        return fail(FLB_ERR_INVALID_ARG, "D2Q9 needs nz = 1 (got %d)", p->nz);
    const double V = (double)p->nx * p->ny * p->nz;
    if (V >= 2147483648.0) return fail(FLB_ERR_INVALID_ARG, "too many sites (%.0f)", V);
    if (V * (p->precision ? 8.0 : 4.0) >= 4294967296.0)
        return fail(FLB_ERR_INVALID_ARG, "a population plane must stay below 4 GiB");
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0))
        return fail(FLB_ERR_INVALID_ARG, "rho0 = %g must be positive", p->rho0);
    if (!(p->kT >= 0.0) || !(p->kT < p->rho0 * CS2))
        return fail(FLB_ERR_INVALID_ARG, "kT = %g outside [0, rho0 cs2 = %g)", p->kT,
                    p->rho0 * CS2);
    const double r[3] = {p->rate_bulk, p->rate_shear, p->rate_ghost};
    for (double x : r)
        if (!(x > 0.0 && x < 2.0)) return fail(FLB_ERR_INVALID_ARG, "rate %g outside (0, 2)", x);
    if (p->force_model == FLB_LANDAU) {
        const double f[4] = {p->a, p->b, p->rho_c, p->kappa};
        for (double x : f)
            if (!std::isfinite(x)) return fail(FLB_ERR_INVALID_ARG, "non-finite force parameter");
        if (p->kappa < 0.0) return fail(FLB_ERR_INVALID_ARG, "kappa = %g < 0", p->kappa);
        if (p->eta != 0 && p->eta != 1) return fail(FLB_ERR_INVALID_ARG, "eta = %d", p->eta);
    }
    return FLB_OK;
}

StepSpec spec_of(const flb_params& p) {
    StepSpec s{};
    s.lat = p.lattice;
    s.prec = p.precision;
    s.force = p.force_model;
    s.nx = p.nx;
    s.ny = p.ny;
    s.nz = p.nz;
    s.rho0 = p.rho0;
    s.kT = p.kT;
    s.lam_bulk = p.rate_bulk;
    s.lam_shear = p.rate_shear;
    s.lam_ghost = p.rate_ghost;
    const double lam[3] = {p.rate_bulk, p.rate_shear, p.rate_ghost};
    for (int c = 0; c < 3; ++c) s.amp_cls[c] = std::sqrt(p.kT * lam[c] * (2.0 - lam[c]) / CS2);
    s.noise_on = p.kT > 0.0;
    s.noise_local = p.noise_rho_local ? 1 : 0;
    s.key0 = (uint32_t)(p.seed & 0xffffffffu);
    s.key1 = (uint32_t)(p.seed >> 32);
    s.replica = p.replica;
    s.a = p.a;
    s.b = p.b;
    s.rho_c = p.rho_c;
    s.kappa = p.kappa;
    s.eta = p.eta;
    return s;
}

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

uint32_t max_slots(const StepSpec& s) {
    uint32_t m = 0;
    for (int c = 0; c < n_configs(s.lat, s.force); ++c) m = std::max(m, config_blocks(s, c));
    return m;
}

bool aligned(const void* p) { return p && ((uintptr_t)p % ALIGN) == 0; }

}  // namespace

void flb::set_last_error(const char* msg) { g_last_error = msg; }

struct flb_handle {
    flb_params p;
    StepSpec spec;
    int q, d;
    size_t V, real_bytes;
    void* fa;
    void* fb;
    bool cur_a;
    char* scratch;
    double* stats;          // [slots][2q] partials, then [2q] finalized
    uint32_t slots;
    uint64_t step;
    int64_t nsamples;
    int cfg;                // launch shape of steps without statistics
    int cfg_stats;          // launch shape of steps that accumulate statistics
    int pair_cfg;           // in-place shape for pairs of steps, or -1
    int64_t check_every;    // > 0: flb_step reads the non-finite flag every this many steps
    // captured steps, one graph per current buffer (index cur_a): kernel
    // arguments hold the buffer pointers, so a replay must start from the
    // buffer its graph was recorded for
    hipGraph_t graph[2];
    hipGraphExec_t gexec[2];
    int64_t graph_steps, graph_samples;
    hipStream_t aux;        // helper stream of flb_adjoint_run (created on first use)
    // scratch regions
    unsigned long long* step_dev;
    void* drho;             // V reals (force model)
    void* rho_part;         // V reals: the march's partial next density (D3Q19 force, FP32)
    void* adj_work;
    double* gpartial;       // adjoint gradient partials
    uint32_t gslots;

    void* cur() const { return cur_a ? fa : fb; }
    void* other() const { return cur_a ? fb : fa; }
};

namespace {

void release_graphs(flb_handle* h) {
    for (int k = 0; k < 2; ++k) {
        if (h->gexec[k]) (void)hipGraphExecDestroy(h->gexec[k]);
        if (h->graph[k]) (void)hipGraphDestroy(h->graph[k]);
        h->gexec[k] = nullptr;
        h->graph[k] = nullptr;
    }
}

void scratch_layout(const StepSpec& s, size_t V, size_t rb, size_t* drho_off, size_t* part_off,
                    size_t* adj_off, size_t* gpart_off, size_t* total) {
    size_t off = SCRATCH_HEADER;
    *drho_off = off;
    off += align_up(V * rb);
    // the partial-density march's output (D3Q19 force steps in FP32)
    *part_off = off;
    off += align_up(partial_density_bytes(s));
    *adj_off = off;
    off += align_up(adjoint_work_bytes(s));
    *gpart_off = off;
    off += align_up(((size_t)adjoint_slots(s) + 1) * 4 * sizeof(double));
    *total = off;
}

// One forward step of the handle: cur -> other, then swap.  drho_ready: the
// density scratch already holds cur's density (the previous step of this
// call was a partial-density march and its completion); updated on return.
flb_status do_step(flb_handle* h, bool sample, const unsigned long long* step_dev,
                   unsigned long long step_host, hipStream_t st, bool* drho_ready) {
    const int cfg = sample ? h->cfg_stats : h->cfg;
    const bool pd = config_partial_density(h->spec, cfg);
    if (h->spec.force && !config_fused(h->spec, cfg) && !(pd && *drho_ready))
        HIP_TRY(launch_density(h->spec, h->cur(), h->drho, st));
    HIP_TRY(launch_step(h->spec, cfg, h->cur(), h->other(), h->drho, step_dev, step_host,
                        sample ? h->stats : nullptr, st, nullptr, pd ? h->rho_part : nullptr));
    if (pd) HIP_TRY(launch_density_fix(h->spec, cfg, h->other(), h->rho_part, h->drho, st));
    *drho_ready = pd;
    h->cur_a = !h->cur_a;
    return FLB_OK;
}

// Steps k = 0 .. nsteps - 1 of a call whose first k0 steps already ran; a
// step is sampled when (k0 + k + 1) % stride == 0.
flb_status run_steps(flb_handle* h, int64_t nsteps, int32_t stride, bool graph_mode,
                     hipStream_t st, int64_t* samples, int64_t k0 = 0) {
    int64_t ns = 0;
    bool drho_ready = false;   // a call starts with a density pass
    const unsigned long long* dev = graph_mode ? h->step_dev : nullptr;
    const unsigned long long base = graph_mode ? 0ull : (unsigned long long)h->step;
    for (int64_t k = 0; k < nsteps;) {
        const bool sample = stride > 0 && ((k0 + k + 1) % stride) == 0;
        if (h->pair_cfg >= 0 && k + 1 < nsteps) {
            // two steps in place on the current buffer (no swap)
            const bool sample1 = stride > 0 && ((k0 + k + 2) % stride) == 0;
            HIP_TRY(launch_step_in_place(h->spec, h->pair_cfg, 0, h->cur(), dev,
                                         base + (unsigned long long)k,
                                         sample ? h->stats : nullptr, st));
            HIP_TRY(launch_step_in_place(h->spec, h->pair_cfg, 1, h->cur(), dev,
                                         base + (unsigned long long)(k + 1),
                                         sample1 ? h->stats : nullptr, st));
            ns += (int64_t)sample + (int64_t)sample1;
            k += 2;
            continue;
        }
        flb_status r = do_step(h, sample, dev, base + (unsigned long long)k, st, &drho_ready);
        if (r != FLB_OK) return r;
        ns += sample;
        ++k;
    }
    if (graph_mode) HIP_TRY(launch_add_u64(h->step_dev, (unsigned long long)nsteps, st));
    *samples = ns;
    return FLB_OK;
}

}  // namespace

extern "C" {

const char* flb_strerror(flb_status s) {
    switch (s) {
        case FLB_OK: return "ok";
        case FLB_ERR_INVALID_ARG: return "invalid argument";
        case FLB_ERR_HIP: return "HIP runtime error";
        case FLB_ERR_NONFINITE: return "non-finite statistics";
        case FLB_ERR_UNSUPPORTED: return "unsupported";
        case FLB_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

const char* flb_last_error(void) { return g_last_error.c_str(); }

flb_status flb_lattice_tables(int32_t lattice, int32_t* q, int32_t* c, double* w, double* T,
                              double* N, int32_t* cls) {
    auto emit = [&](auto L) {
        using LL = decltype(L);
        if (q) *q = LL::Q;
        for (int i = 0; i < LL::Q; ++i) {
            if (c) {
                c[3 * i + 0] = LL::cx[i];
                c[3 * i + 1] = LL::cy[i];
                c[3 * i + 2] = LL::cz[i];
            }
            if (w) w[i] = LL::w[i];
            if (N) N[i] = LL::N[i];
            if (cls) cls[i] = LL::cls[i];
            if (T)
                for (int j = 0; j < LL::Q; ++j) T[i * LL::Q + j] = LL::T[i][j];
        }
    };
    if (lattice == FLB_D2Q9) emit(Lattice<0>{});
    else if (lattice == FLB_D3Q19) emit(Lattice<1>{});
    else return fail(FLB_ERR_INVALID_ARG, "unknown lattice %d", lattice);
    return FLB_OK;
}

flb_status flb_query_sizes(const flb_params* p, size_t* pop_bytes, size_t* scratch_bytes,
                           size_t* stats_bytes) {
    flb_status r = validate(p);
    if (r != FLB_OK) return r;
    const StepSpec s = spec_of(*p);
    const size_t V = (size_t)p->nx * p->ny * p->nz;
    const size_t rb = p->precision == FLB_FP64 ? 8 : 4;
    const int q = lattice_q(p->lattice);
    size_t a, b, c, d, total;
    scratch_layout(s, V, rb, &a, &b, &c, &d, &total);
    if (pop_bytes) *pop_bytes = align_up((size_t)q * V * rb);
    if (scratch_bytes) *scratch_bytes = total;
    if (stats_bytes) *stats_bytes = align_up(((size_t)max_slots(s) + 1) * 2 * q * sizeof(double));
    return FLB_OK;
}

flb_status flb_init(const flb_params* p, void* f_a, void* f_b, void* scratch, void* stats,
                    const double* drho_init, void* stream, flb_handle** out) {
    if (!out) return fail(FLB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    flb_status r = validate(p);
    if (r != FLB_OK) return r;
    if (!aligned(f_a) || !aligned(f_b) || !aligned(scratch) || !aligned(stats))
        return fail(FLB_ERR_INVALID_ARG, "buffers must be non-NULL and 256-byte aligned");
    if (f_a == f_b) return fail(FLB_ERR_INVALID_ARG, "f_a and f_b must differ");
    hipStream_t st = (hipStream_t)stream;
    flb_handle* h = new (std::nothrow) flb_handle();
    if (!h) return fail(FLB_ERR_INVALID_ARG, "out of host memory");
    h->p = *p;
    h->spec = spec_of(*p);
    h->q = lattice_q(p->lattice);
    h->d = lattice_d(p->lattice);
    h->V = (size_t)p->nx * p->ny * p->nz;
    h->real_bytes = p->precision == FLB_FP64 ? 8 : 4;
    h->fa = f_a;
    h->fb = f_b;
    h->cur_a = true;
    h->scratch = (char*)scratch;
    h->stats = (double*)stats;
    h->slots = max_slots(h->spec);
    h->step = p->step0;
    h->nsamples = 0;
    // D2Q9 force steps default to the 32 x 8 tile that forms its own density
    // tile (no density pass); every other kind to shape 0
    h->cfg = h->cfg_stats = (h->spec.force && h->spec.lat == 0) ? 4 : 0;
    h->pair_cfg = -1;
    h->graph[0] = h->graph[1] = nullptr;
    h->gexec[0] = h->gexec[1] = nullptr;
    size_t drho_off, part_off, adj_off, gp_off, total;
    scratch_layout(h->spec, h->V, h->real_bytes, &drho_off, &part_off, &adj_off, &gp_off, &total);
    h->step_dev = (unsigned long long*)h->scratch;
    h->spec.nonfinite = (uint32_t*)(h->scratch + NONFINITE_OFF);
    h->check_every = 0;
    h->drho = h->scratch + drho_off;
    h->rho_part = h->scratch + part_off;
    h->adj_work = h->scratch + adj_off;
    h->gpartial = (double*)(h->scratch + gp_off);
    h->gslots = adjoint_slots(h->spec);
    const size_t stats_bytes = ((size_t)h->slots + 1) * 2 * h->q * sizeof(double);
    hipError_t e = launch_init(h->spec, f_a, drho_init, st);
    if (e == hipSuccess) e = launch_fill_zero(stats, stats_bytes, st);
    if (e == hipSuccess) e = launch_fill_zero(h->scratch, total, st);
    if (e == hipSuccess) e = launch_set_u64(h->step_dev, h->step, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete h;
        return fail(FLB_ERR_HIP, "flb_init: %s", hipGetErrorString(e));
    }
    *out = h;
    return FLB_OK;
}

flb_status flb_step(flb_handle* h, int64_t nsteps, int32_t stats_stride, void* stream) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    if (nsteps < 0 || stats_stride < 0)
        return fail(FLB_ERR_INVALID_ARG, "nsteps %lld, stats_stride %d", (long long)nsteps,
                    stats_stride);
    hipStream_t st = (hipStream_t)stream;
    // without checks one chunk; with checks, chunks of check_every steps, the
    // device flag read (and the stream synchronized) after each
    const int64_t chunk = h->check_every > 0 ? h->check_every : (nsteps > 0 ? nsteps : 1);
    for (int64_t k0 = 0; k0 < nsteps; k0 += chunk) {
        const int64_t n = nsteps - k0 < chunk ? nsteps - k0 : chunk;
        int64_t ns = 0;
        flb_status r = run_steps(h, n, stats_stride, false, st, &ns, k0);
        if (r != FLB_OK) return r;
        h->step += (uint64_t)n;
        h->nsamples += ns;
        if (h->check_every > 0) {
            uint32_t flag = 0;
            HIP_TRY(hipMemcpyAsync(&flag, h->spec.nonfinite, sizeof flag, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (flag) {
                HIP_TRY(launch_set_u64(h->step_dev, h->step, st));
                return fail(FLB_ERR_NONFINITE,
                            "a non-finite density was pulled by a step before step %llu",
                            (unsigned long long)h->step);
            }
        }
    }
    // keep the device step counter in step with the host (graph replays read it)
    HIP_TRY(launch_set_u64(h->step_dev, h->step, st));
    return FLB_OK;
}

flb_status flb_set_check(flb_handle* h, int64_t every, void* stream) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    if (every < 0) return fail(FLB_ERR_INVALID_ARG, "every = %lld < 0", (long long)every);
    h->check_every = every;
    HIP_TRY(launch_fill_zero(h->spec.nonfinite, sizeof(uint32_t), (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_seek(flb_handle* h, uint64_t step, void* stream) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    h->step = step;
    HIP_TRY(launch_set_u64(h->step_dev, h->step, (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_state(const flb_handle* h, void** cur, void** other, uint64_t* step) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    if (cur) *cur = h->cur();
    if (other) *other = h->other();
    if (step) *step = h->step;
    return FLB_OK;
}

flb_status flb_moments(flb_handle* h, double* mode_sum, double* mode_sumsq, int64_t* nsamples,
                       void* stream) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    hipStream_t st = (hipStream_t)stream;
    const int nv = 2 * h->q;
    double* out = h->stats + (size_t)h->slots * nv;
    HIP_TRY(launch_stats_finalize(h->stats, h->slots, nv, out, st));
    std::vector<double> host(nv);
    HIP_TRY(hipMemcpyAsync(host.data(), out, nv * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (mode_sum) std::memcpy(mode_sum, host.data(), h->q * sizeof(double));
    if (mode_sumsq) std::memcpy(mode_sumsq, host.data() + h->q, h->q * sizeof(double));
    if (nsamples) *nsamples = h->nsamples;
    for (double v : host)
        if (!std::isfinite(v)) return fail(FLB_ERR_NONFINITE, "statistics are not finite");
    return FLB_OK;
}

flb_status flb_reset_stats(flb_handle* h, void* stream) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    HIP_TRY(launch_fill_zero(h->stats, ((size_t)h->slots + 1) * 2 * h->q * sizeof(double),
                             (hipStream_t)stream));
    h->nsamples = 0;
    return FLB_OK;
}

flb_status flb_fields(flb_handle* h, void* out, void* stream) {
    if (!h || !out) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    if (h->spec.force) HIP_TRY(launch_density(h->spec, h->cur(), h->drho, st));
    HIP_TRY(launch_fields(h->spec, h->cur(), h->drho, out, st));
    return FLB_OK;
}

flb_status flb_mode_fields(flb_handle* h, double* out, void* stream) {
    if (!h || !out) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if ((uintptr_t)out % sizeof(double)) return fail(FLB_ERR_INVALID_ARG, "out must be 8-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    if (h->spec.force) HIP_TRY(launch_density(h->spec, h->cur(), h->drho, st));
    HIP_TRY(launch_mode_fields(h->spec, h->cur(), h->drho, out, st));
    return FLB_OK;
}

flb_status flb_spectrum_work_bytes(const flb_handle* h, size_t* bytes) {
    if (!h || !bytes) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    *bytes = (size_t)h->q * h->V * (2 * sizeof(double) + sizeof(double));
    return FLB_OK;
}

flb_status flb_mode_spectrum(flb_handle* h, void* work, double* spec, void* stream) {
    if (!h || !work || !spec) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (!aligned(work)) return fail(FLB_ERR_INVALID_ARG, "work must be 256-byte aligned");
    if ((uintptr_t)spec % sizeof(double)) return fail(FLB_ERR_INVALID_ARG, "spec must be 8-byte aligned");
    const StepSpec& s = h->spec;
    if (s.nx > SPECTRUM_MAX_N || s.ny > SPECTRUM_MAX_N || s.nz > SPECTRUM_MAX_N)
        return fail(FLB_ERR_UNSUPPORTED, "mode spectra need every extent <= 1024");
    hipStream_t st = (hipStream_t)stream;
    // work: q V complex transforms, then the q V real mode fields
    double* fields = (double*)((char*)work + (size_t)h->q * h->V * 2 * sizeof(double));
    if (s.force) HIP_TRY(launch_density(s, h->cur(), h->drho, st));
    HIP_TRY(launch_mode_fields(s, h->cur(), h->drho, fields, st));
    HIP_TRY(launch_spectrum(h->q, h->d == 2 ? 1 : 3, s.nx, s.ny, s.nz, fields, work, spec, st));
    return FLB_OK;
}

flb_status flb_field_spectrum(const double* fields, int32_t nfields, int32_t nx, int32_t ny,
                              int32_t nz, void* work, double* spec, void* stream) {
    if (!fields || !work || !spec) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (nfields < 1 || nx < 1 || ny < 1 || nz < 1)
        return fail(FLB_ERR_INVALID_ARG, "nfields and extents must be positive");
    if (nx > SPECTRUM_MAX_N || ny > SPECTRUM_MAX_N || nz > SPECTRUM_MAX_N)
        return fail(FLB_ERR_UNSUPPORTED, "field spectra need every extent <= 1024");
    if (!aligned(work)) return fail(FLB_ERR_INVALID_ARG, "work must be 256-byte aligned");
    if ((uintptr_t)fields % sizeof(double) || (uintptr_t)spec % sizeof(double))
        return fail(FLB_ERR_INVALID_ARG, "fields and spec must be 8-byte aligned");
    HIP_TRY(launch_spectrum(nfields, 0, nx, ny, nz, fields, work, spec, (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_interface_heights(flb_handle* h, const flb_interface* ifs, int32_t n_if,
                                 double rho_L, double rho_V, double width, double* heights,
                                 void* stream) {
    if (!h || !ifs || !heights) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (!h->spec.force)
        return fail(FLB_ERR_UNSUPPORTED, "interface heights need the non-ideal fluid");
    if (n_if < 1 || n_if > MAX_INTERFACES)
        return fail(FLB_ERR_INVALID_ARG, "n_if must be in [1, 8]");
    if (!(width > 0.0) || !(rho_L != rho_V) || !std::isfinite(rho_L) || !std::isfinite(rho_V))
        return fail(FLB_ERR_INVALID_ARG, "width must be positive and rho_L != rho_V");
    if ((uintptr_t)heights % sizeof(double))
        return fail(FLB_ERR_INVALID_ARG, "heights must be 8-byte aligned");
    const StepSpec& s = h->spec;
    const int n = h->d == 2 ? s.ny : s.nz;           // profile axis: y (2-D) or z (3-D)
    const long ncol = (long)(h->V / (size_t)n);
    InterfaceSet set{};
    set.n = n_if;
    for (int j = 0; j < n_if; ++j) {
        const flb_interface& f = ifs[j];
        if (!(f.y_ref >= 0.0 && f.y_ref < n) || (f.sign != 1 && f.sign != -1) ||
            f.half_window < 1 || 2 * f.half_window + 1 > n)
            return fail(FLB_ERR_INVALID_ARG,
                        "interface: y_ref in [0, n), sign +-1, 1 <= half_window, 2 W + 1 <= n");
        set.y0[j] = (int)std::floor(f.y_ref + 0.5);
        set.sign[j] = f.sign;
        set.half_window[j] = f.half_window;
    }
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_density(s, h->cur(), h->drho, st));
    HIP_TRY(launch_interface_heights(s.prec, h->drho, s.rho0, n, ncol, set, rho_L, rho_V, width,
                                     heights, st));
    return FLB_OK;
}

flb_status flb_density(flb_handle* h, const void* s, void* out, void* stream) {
    if (!h || !s || !out) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    HIP_TRY(launch_density(h->spec, s, out, (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_noise_words(const flb_params* p, uint64_t step, uint32_t block, uint32_t tag,
                           uint64_t site0, uint64_t nsites, uint32_t* out_dev, void* stream) {
    flb_status r = validate(p);
    if (r != FLB_OK) return r;
    if (!out_dev && nsites) return fail(FLB_ERR_INVALID_ARG, "out_dev is NULL");
    if (block > 0xffffu || tag > 0xffffu) return fail(FLB_ERR_INVALID_ARG, "block/tag > 16 bit");
    HIP_TRY(launch_noise_words(spec_of(*p), step, block, tag, site0, nsites, out_dev,
                               (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_noise_normals(const flb_params* p, uint64_t step, uint64_t site0, uint64_t nsites,
                             void* out_dev, void* stream) {
    flb_status r = validate(p);
    if (r != FLB_OK) return r;
    if (!out_dev && nsites) return fail(FLB_ERR_INVALID_ARG, "out_dev is NULL");
    HIP_TRY(launch_noise_normals(spec_of(*p), step, site0, nsites, out_dev, (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_graph_capture(flb_handle* h, int64_t nsteps, int32_t stats_stride, void* stream) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    if (nsteps <= 0 || stats_stride < 0)
        return fail(FLB_ERR_INVALID_ARG, "nsteps %lld", (long long)nsteps);
    if (nsteps % 2 != 0)
        return fail(FLB_ERR_INVALID_ARG, "graph step count must be even (buffers alternate)");
    hipStream_t st = (hipStream_t)stream;
    if (!st) return fail(FLB_ERR_INVALID_ARG, "graph capture needs a non-null stream");
    release_graphs(h);
    // record the steps once for each buffer the state can be in, so that a
    // replay after an odd number of ordinary steps still continues the state
    const bool cur_a = h->cur_a;
    int64_t ns = 0;
    flb_status r = FLB_OK;
    for (int k = 0; k < 2 && r == FLB_OK; ++k) {
        h->cur_a = k == 1;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            r = fail(FLB_ERR_HIP, "begin capture: %s", hipGetErrorString(e));
            break;
        }
        r = run_steps(h, nsteps, stats_stride, true, st, &ns);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(st, &g);
        if (r == FLB_OK && e != hipSuccess)
            r = fail(FLB_ERR_HIP, "capture: %s", hipGetErrorString(e));
        if (r != FLB_OK) {
            if (g) (void)hipGraphDestroy(g);
            break;
        }
        h->graph[k] = g;
        e = hipGraphInstantiate(&h->gexec[k], g, nullptr, nullptr, 0);
        if (e != hipSuccess) r = fail(FLB_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    h->cur_a = cur_a;   // nothing ran
    if (r != FLB_OK) {
        release_graphs(h);
        return r;
    }
    h->graph_steps = nsteps;
    h->graph_samples = ns;
    return FLB_OK;
}

flb_status flb_graph_launch(flb_handle* h, void* stream) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    hipGraphExec_t ex = h->gexec[h->cur_a ? 1 : 0];
    if (!ex) return fail(FLB_ERR_STATE, "no graph captured");
    HIP_TRY(hipGraphLaunch(ex, (hipStream_t)stream));
    h->step += (uint64_t)h->graph_steps;
    h->nsamples += h->graph_samples;
    // graph_steps is even, so the current buffer is unchanged
    return FLB_OK;
}

flb_status flb_autotune(flb_handle* h, int32_t repeats, int32_t* best, double* best_ms,
                        void* stream) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    if (repeats < 1) repeats = 1;
    hipStream_t st = (hipStream_t)stream;
    // Trials run as real stepping does (ordinary steps alternate the two
    // buffers, pairs update one buffer in place), so cache residency is the
    // same as in a run.  The state and the statistics slots are saved to host
    // memory first and put back afterwards.
    const size_t pbytes = ((size_t)h->slots + 1) * 2 * h->q * sizeof(double);
    const size_t sbytes = (size_t)h->q * h->V * h->real_bytes;
    std::vector<double> saved_stats(pbytes / sizeof(double));
    std::vector<unsigned char> saved_state;
    try {
        saved_state.resize(sbytes);
    } catch (...) {
        return fail(FLB_ERR_INVALID_ARG, "autotune: no host memory for a copy of the state");
    }
    void* const A = h->cur();
    void* const B = h->other();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMemcpyAsync(saved_stats.data(), h->stats, pbytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(saved_state.data(), A, sbytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int ncfg = n_configs(h->spec.lat, h->spec.force);
    int bi[2] = {h->cfg, h->cfg_stats};
    float bt[2] = {1e30f, 1e30f};
    if (e == hipSuccess && h->spec.force) e = launch_density(h->spec, A, h->drho, st);
    auto timed = [&](auto&& launch, int per_call, float* ms_out) {
        hipError_t r = launch(0);   // warm-up
        if (r == hipSuccess) r = hipEventRecord(e0, st);
        for (int k = 1; k <= repeats && r == hipSuccess; ++k) r = launch(k);
        if (r == hipSuccess) r = hipEventRecord(e1, st);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        float ms = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        *ms_out = ms / (float)(repeats * per_call);
        return r;
    };
    for (int mode = 0; mode < 2 && e == hipSuccess; ++mode) {
        double* part = mode ? h->stats : nullptr;
        for (int c = 0; c < ncfg && e == hipSuccess; ++c) {
            if (config_in_place(h->spec, c)) continue;   // timed as pairs below
            float ms = 0.f;
            // a force step that reads a density field pays for its pass; a
            // partial-density march for the completion of the next density
            const bool pd = config_partial_density(h->spec, c);
            const bool pass = h->spec.force && !config_fused(h->spec, c) && !pd;
            e = timed([&](int k) {
                void* in = (k & 1) ? B : A;
                void* out = (k & 1) ? A : B;
                if (pass) {
                    hipError_t r = launch_density(h->spec, in, h->drho, st);
                    if (r != hipSuccess) return r;
                }
                hipError_t r = launch_step(h->spec, c, in, out, h->drho, nullptr, h->step, part, st,
                                           nullptr, pd ? h->rho_part : nullptr);
                if (r == hipSuccess && pd)
                    r = launch_density_fix(h->spec, c, out, h->rho_part, h->drho, st);
                return r;
            }, 1, &ms);
            if (e == hipSuccess && ms < bt[mode]) {
                bt[mode] = ms;
                bi[mode] = c;
            }
        }
    }
    // In-place pairs: their point is cache residency, which a run reaches
    // only after its buffer has settled, and the candidates differ by a few
    // percent.  So the state is first stepped for about 4 ms with the first
    // candidate, then every candidate is timed for about 2 ms per trial,
    // round-robin, and each keeps its best round.
    int best_pair = -1;
    float pair_ms = 1e30f;
    std::vector<int> cands;
    for (int c = 0; c < ncfg; ++c)
        if (config_in_place(h->spec, c)) cands.push_back(c);
    auto pair = [&](int c) {
        hipError_t r = launch_step_in_place(h->spec, c, 0, A, nullptr, h->step, h->stats, st);
        if (r == hipSuccess)
            r = launch_step_in_place(h->spec, c, 1, A, nullptr, h->step + 1, h->stats, st);
        return r;
    };
    auto time_pairs = [&](int c, int n, float* ms_per_step) {
        hipError_t r = hipEventRecord(e0, st);
        for (int k = 0; k < n && r == hipSuccess; ++k) r = pair(c);
        if (r == hipSuccess) r = hipEventRecord(e1, st);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        float ms = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        *ms_per_step = ms / (float)(2 * n);
        return r;
    };
    if (!cands.empty() && e == hipSuccess) {
        float t1 = 0.f;
        e = pair(cands[0]);
        if (e == hipSuccess) e = time_pairs(cands[0], 1, &t1);
        const float pair_est = std::max(2.f * t1, 1e-3f);   // ms per pair
        const int settle = std::min(400, std::max(2, (int)(4.f / pair_est)));
        const int per = std::min(200, std::max(repeats, (int)(2.f / pair_est)));
        for (int k = 0; k < settle && e == hipSuccess; ++k) e = pair(cands[0]);
        std::vector<float> bt_c(cands.size(), 1e30f);
        for (int round = 0; round < std::max(3, repeats) && e == hipSuccess; ++round)
            for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i) {
                float ms = 0.f;
                e = time_pairs(cands[i], per, &ms);
                if (e == hipSuccess) bt_c[i] = std::min(bt_c[i], ms);
            }
        for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i)
            if (bt_c[i] < pair_ms) {
                pair_ms = bt_c[i];
                best_pair = cands[i];
            }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // restore the state and the sums even after a failed trial
    hipError_t er = hipMemcpyAsync(A, saved_state.data(), sbytes, hipMemcpyHostToDevice, st);
    if (er == hipSuccess)
        er = hipMemcpyAsync(h->stats, saved_stats.data(), pbytes, hipMemcpyHostToDevice, st);
    if (er == hipSuccess) er = hipStreamSynchronize(st);
    if (e == hipSuccess) e = er;
    if (e != hipSuccess) return fail(FLB_ERR_HIP, "autotune: %s", hipGetErrorString(e));
    h->cfg = bi[0];
    h->cfg_stats = bi[1];
    // pairs are used when they beat ordinary steps with statistics
    h->pair_cfg = (best_pair >= 0 && pair_ms < bt[1]) ? best_pair : -1;
    for (int m = 0; m < 2; ++m) {
        if (best) best[m] = bi[m];
        if (best_ms) best_ms[m] = bt[m];
    }
    if (best) best[2] = best_pair;
    if (best_ms) best_ms[2] = best_pair >= 0 ? pair_ms : 0.0;
    if (best) best[3] = h->pair_cfg;
    return FLB_OK;
}

flb_status flb_set_launch(flb_handle* h, int32_t config) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    if (config < 0 || config >= n_configs(h->spec.lat, h->spec.force))
        return fail(FLB_ERR_INVALID_ARG, "launch config %d out of range", config);
    if (config_in_place(h->spec, config)) {
        h->pair_cfg = config;
        h->cfg = h->cfg_stats = config;   // a lone step runs the ordinary kernel of this tile
    } else {
        h->pair_cfg = -1;
        h->cfg = h->cfg_stats = config;
    }
    return FLB_OK;
}

flb_status flb_launch_configs(const flb_handle* h, int32_t* count, int32_t* current) {
    if (!h) return fail(FLB_ERR_INVALID_ARG, "handle is NULL");
    if (count) *count = n_configs(h->spec.lat, h->spec.force);
    if (current) {
        current[0] = h->cfg;
        current[1] = h->cfg_stats;
        current[2] = h->pair_cfg;
    }
    return FLB_OK;
}

flb_status flb_launch_shape(const flb_handle* h, int32_t config, int32_t* shape) {
    if (!h || !shape) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (config < 0 || config >= n_configs(h->spec.lat, h->spec.force))
        return fail(FLB_ERR_INVALID_ARG, "launch config %d out of range", config);
    const TileShape t = config_shape(h->spec.lat, h->spec.force, config);
    shape[0] = t.tx;
    shape[1] = t.ty;
    shape[2] = t.tz;
    shape[3] = t.spt;
    shape[4] = t.nt;
    shape[5] = t.zc;
    shape[6] = t.ip;
    shape[7] = t.fd ? 1 : (t.pd ? 2 : 0);
    return FLB_OK;
}

flb_status flb_adjoint_density_seed(flb_handle* h, const void* rhobar, void* abar_N,
                                    void* stream) {
    if (!h || !rhobar || !abar_N) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    HIP_TRY(launch_adjoint_seed(h->spec, rhobar, abar_N, (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_adjoint_step(flb_handle* h, const void* s_n, const void* abar_np1, void* abar_n,
                            double* grad, uint64_t n, void* stream) {
    if (!h || !s_n || !abar_np1 || !abar_n) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (abar_n == abar_np1 || abar_n == s_n)
        return fail(FLB_ERR_INVALID_ARG, "abar_n must not alias the inputs");
    hipStream_t st = (hipStream_t)stream;
    if (h->spec.force) HIP_TRY(launch_density(h->spec, s_n, h->drho, st));
    AdjointStepArgs a{s_n, h->drho, abar_np1, abar_n, h->adj_work, -1, 0, true,
                      (unsigned long long)n, h->gpartial, nullptr};
    HIP_TRY(launch_adjoint_step(h->spec, a, st));
    if (grad) {
        double* out = h->gpartial + (size_t)h->gslots * 4;
        HIP_TRY(launch_stats_finalize(h->gpartial, h->gslots, 4, out, st));
        double host[4];
        HIP_TRY(hipMemcpyAsync(host, out, sizeof host, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int k = 0; k < 4; ++k) grad[k] += host[k];
        HIP_TRY(launch_fill_zero(h->gpartial, (size_t)h->gslots * 4 * sizeof(double), st));
    }
    return FLB_OK;
}

flb_status flb_adjoint_segment_bytes(const flb_handle* h, int64_t nsteps, size_t* bytes) {
    if (!h || !bytes || nsteps < 1) return fail(FLB_ERR_INVALID_ARG, "bad argument");
    const size_t plane = align_up((size_t)h->q * h->V * h->real_bytes);
    const size_t dens = align_up(h->V * h->real_bytes);
    // nsteps - 1 recomputed states, one spare adjoint buffer, nsteps densities
    *bytes = (size_t)nsteps * plane + (h->spec.force ? (size_t)nsteps * dens : 0);
    return FLB_OK;
}

}  // extern "C"

namespace {

// Work layout of one segment [k0, k0 + k): states S_{k0+1} .. S_{k0+k-1},
// one spare adjoint buffer, then k densities (force model).
struct SegWork {
    flb_handle* h;
    const void* s_k0;
    char* w;
    size_t k, plane, dens;
    SegWork(flb_handle* h_, const void* s0, void* work, size_t k_)
        : h(h_), s_k0(s0), w((char*)work), k(k_),
          plane(align_up((size_t)h_->q * h_->V * h_->real_bytes)),
          dens(align_up(h_->V * h_->real_bytes)) {}
    const void* state(size_t j) const { return j == 0 ? s_k0 : (const void*)(w + (j - 1) * plane); }
    void* spare() const { return w + (k - 1) * plane; }
    void* density(size_t j) const { return h->spec.force ? w + k * plane + j * dens : nullptr; }
};

// Recompute S_{k0+1} .. S_{k0+k-1} (and every state's density) with the forward kernels.
flb_status seg_recompute(const SegWork& sw, uint64_t k0, hipStream_t st) {
    flb_handle* h = sw.h;
    if (h->spec.force && config_fused(h->spec, h->cfg)) {
        // the step forms its input's density itself and writes it out, so a
        // recomputed step is one launch; the last state's density is a pass
        for (size_t j = 1; j < sw.k; ++j)
            HIP_TRY(launch_step(h->spec, h->cfg, sw.state(j - 1), (void*)sw.state(j), nullptr,
                                nullptr, (unsigned long long)(k0 + j - 1), nullptr, st,
                                (void*)sw.density(j - 1)));
        HIP_TRY(launch_density(h->spec, sw.state(sw.k - 1), sw.density(sw.k - 1), st));
        return FLB_OK;
    }
    if (h->spec.force) HIP_TRY(launch_density(h->spec, sw.state(0), sw.density(0), st));
    for (size_t j = 1; j < sw.k; ++j) {
        HIP_TRY(launch_step(h->spec, h->cfg, sw.state(j - 1), (void*)sw.state(j),
                            sw.density(j - 1), nullptr, (unsigned long long)(k0 + j - 1), nullptr,
                            st));
        if (h->spec.force) HIP_TRY(launch_density(h->spec, sw.state(j), sw.density(j), st));
    }
    return FLB_OK;
}

// Reverse sweep n = k0 + k - 1 .. k0: abar holds dL/dS_{k0+k} on entry and
// dL/dS_{k0} on return.  abar and the spare buffer alternate; each step's
// density adjoint is spread into the populations by the next (earlier) step,
// the last one's at the end.
flb_status seg_reverse(const SegWork& sw, void* abar, uint64_t k0, hipStream_t st) {
    flb_handle* h = sw.h;
    void* cur = abar;
    void* nxt = sw.spare();
    int rb_in = -1;
    for (size_t j = sw.k; j-- > 0;) {
        const int rb_out = (int)(j & 1);
        AdjointStepArgs a{sw.state(j), sw.density(j), cur, nxt, h->adj_work, rb_in, rb_out, false,
                          (unsigned long long)(k0 + j), h->gpartial,
                          j + 1 < sw.k ? sw.density(j + 1) : nullptr};
        HIP_TRY(launch_adjoint_step(h->spec, a, st));
        rb_in = rb_out;
        std::swap(cur, nxt);
    }
    if (h->spec.force)
        HIP_TRY(launch_adjoint_spread(h->spec, h->adj_work, rb_in, sw.density(0), cur, st));
    if (cur != abar)
        HIP_TRY(hipMemcpyAsync(abar, cur, (size_t)h->q * h->V * h->real_bytes,
                               hipMemcpyDeviceToDevice, st));
    return FLB_OK;
}

// Finalize the parameter-derivative accumulators, add them to grad[4], clear.
flb_status grad_finalize(flb_handle* h, double* grad, hipStream_t st) {
    double* out = h->gpartial + (size_t)h->gslots * 4;
    HIP_TRY(launch_stats_finalize(h->gpartial, h->gslots, 4, out, st));
    double host[4];
    HIP_TRY(hipMemcpyAsync(host, out, sizeof host, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int q = 0; q < 4; ++q) grad[q] += host[q];
    HIP_TRY(launch_fill_zero(h->gpartial, (size_t)h->gslots * 4 * sizeof(double), st));
    return FLB_OK;
}

}  // namespace

extern "C" {

flb_status flb_adjoint_segment(flb_handle* h, const void* s_k0, void* abar, void* work,
                               uint64_t k0, uint64_t k1, double* grad, void* stream) {
    if (!h || !s_k0 || !abar || !work) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (k1 <= k0) return fail(FLB_ERR_INVALID_ARG, "empty segment [%llu, %llu)",
                              (unsigned long long)k0, (unsigned long long)k1);
    if (!aligned(work)) return fail(FLB_ERR_INVALID_ARG, "work must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const SegWork sw(h, s_k0, work, (size_t)(k1 - k0));
    flb_status r = seg_recompute(sw, k0, st);
    if (r == FLB_OK) r = seg_reverse(sw, abar, k0, st);
    if (r == FLB_OK && grad) r = grad_finalize(h, grad, st);
    return r;
}

flb_status flb_adjoint_run_bytes(const flb_handle* h, int64_t seg_len, size_t* bytes) {
    size_t one = 0;
    flb_status r = flb_adjoint_segment_bytes(h, seg_len, &one);
    if (r != FLB_OK) return r;
    *bytes = 2 * align_up(one);
    return FLB_OK;
}

flb_status flb_adjoint_run(flb_handle* h, const void* const* ckpts, int32_t nseg,
                           int64_t seg_len, int64_t nsteps, void* abar, void* work,
                           double* grad, void* stream) {
    if (!h || !ckpts || !abar || !work) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (nseg < 1 || seg_len < 1 || nsteps <= (int64_t)(nseg - 1) * seg_len ||
        nsteps > (int64_t)nseg * seg_len)
        return fail(FLB_ERR_INVALID_ARG, "%d segments of %lld steps do not cover %lld steps",
                    nseg, (long long)seg_len, (long long)nsteps);
    for (int s = 0; s < nseg; ++s)
        if (!ckpts[s]) return fail(FLB_ERR_INVALID_ARG, "checkpoint %d is NULL", s);
    if (!aligned(work)) return fail(FLB_ERR_INVALID_ARG, "work must be 256-byte aligned");
    size_t one = 0;
    flb_status r = flb_adjoint_segment_bytes(h, seg_len, &one);
    if (r != FLB_OK) return r;
    one = align_up(one);
    hipStream_t A = (hipStream_t)stream;
    if (!h->aux) HIP_TRY(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    hipStream_t B = h->aux;
    hipEvent_t start = nullptr, ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&ready[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&freed[i], hipEventDisableTiming);
    }
    auto seg = [&](int s) {
        const uint64_t k0 = (uint64_t)s * (uint64_t)seg_len;
        const uint64_t k1 = std::min<uint64_t>(k0 + (uint64_t)seg_len, (uint64_t)nsteps);
        return SegWork(h, ckpts[s], (char*)work + (size_t)(s & 1) * one, (size_t)(k1 - k0));
    };
    // The recompute of segment s - 1 (helper stream) overlaps the reverse
    // sweep of segment s (caller's stream); the two halves of `work`
    // alternate, guarded by events.
    if (e == hipSuccess) e = hipEventRecord(start, A);
    if (e == hipSuccess) e = hipStreamWaitEvent(B, start, 0);
    if (e != hipSuccess) r = fail(FLB_ERR_HIP, "adjoint run: %s", hipGetErrorString(e));
    const int last = nseg - 1;
    if (r == FLB_OK) r = seg_recompute(seg(last), (uint64_t)last * seg_len, B);
    if (r == FLB_OK && hipEventRecord(ready[last & 1], B) != hipSuccess)
        r = fail(FLB_ERR_HIP, "adjoint run: event record failed");
    for (int s = last; s >= 0 && r == FLB_OK; --s) {
        if (s >= 1) {
            const int hb = (s - 1) & 1;
            if (s + 1 <= last && hipStreamWaitEvent(B, freed[hb], 0) != hipSuccess)
                r = fail(FLB_ERR_HIP, "adjoint run: wait failed");
            if (r == FLB_OK) r = seg_recompute(seg(s - 1), (uint64_t)(s - 1) * seg_len, B);
            if (r == FLB_OK && hipEventRecord(ready[hb], B) != hipSuccess)
                r = fail(FLB_ERR_HIP, "adjoint run: event record failed");
        }
        if (r == FLB_OK && hipStreamWaitEvent(A, ready[s & 1], 0) != hipSuccess)
            r = fail(FLB_ERR_HIP, "adjoint run: wait failed");
        if (r == FLB_OK) r = seg_reverse(seg(s), abar, (uint64_t)s * seg_len, A);
        if (r == FLB_OK && hipEventRecord(freed[s & 1], A) != hipSuccess)
            r = fail(FLB_ERR_HIP, "adjoint run: event record failed");
    }
    if (r != FLB_OK) (void)hipStreamSynchronize(B);   // nothing of ours left running
    if (r == FLB_OK && grad) r = grad_finalize(h, grad, A);
    if (start) (void)hipEventDestroy(start);
    for (int i = 0; i < 2; ++i) {
        if (ready[i]) (void)hipEventDestroy(ready[i]);
        if (freed[i]) (void)hipEventDestroy(freed[i]);
    }
    return r;
}

// ------------------------------------------------ modified-equilibrium model

namespace {

// Xi_(e,eps) block at c_s^2 = c2 (per rho0 kT); see modeq.hip.
void modeq_block(double c2, double le, double lg, double& see, double& sep, double& spp) {
    see = 12.0 * le * (2.0 - le) * (2.0 - 3.0 * c2);
    sep = 12.0 * (3.0 * c2 - 1.0) * (le + lg - le * lg);
    spp = 12.0 * lg * (2.0 - lg) * (5.0 - 3.0 * c2);
}

flb_status modeq_args(const flb_modeq_params* p, ModEqArgs* a) {
    if (!p) return fail(FLB_ERR_INVALID_ARG, "NULL params");
    if (p->nx < 1 || p->ny < 1 || p->nx > SPECTRUM_MAX_N || p->ny > SPECTRUM_MAX_N)
        return fail(FLB_ERR_INVALID_ARG, "modified-equilibrium extents must be in [1, 1024]");
    if (p->precision != FLB_FP32 && p->precision != FLB_FP64)
        return fail(FLB_ERR_INVALID_ARG, "precision must be FLB_FP32 or FLB_FP64");
    a->prec = p->precision == FLB_FP64 ? 1 : 0;
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0) || !(p->kT >= 0.0) || !std::isfinite(p->kT))
        return fail(FLB_ERR_INVALID_ARG, "rho0 must be positive and kT >= 0");
    const double rates[3] = {p->rate_bulk, p->rate_shear, p->rate_ghost};
    for (double r : rates)
        if (!(r > 0.0 && r < 2.0)) return fail(FLB_ERR_INVALID_ARG, "rates must lie in (0, 2)");
    if (!(p->cs2_0 > 0.0) || !(p->kappa >= 0.0) || !std::isfinite(p->kappa))
        return fail(FLB_ERR_INVALID_ARG, "cs2_0 must be positive and kappa >= 0");
    // c_s^2(k) spans [cs2_0, cs2_0 + kappa rho0 16/3]; the equilibrium
    // populations stay non-negative up to 0.6
    const double c2max = p->cs2_0 + p->kappa * p->rho0 * 16.0 / 3.0;
    if (!(c2max <= 0.6))
        return fail(FLB_ERR_INVALID_ARG,
                    "c_s^2(k) = cs2_0 + kappa rho0 Lambda(k) must stay <= 0.6 (max %g)", c2max);
    for (int s = 0; s <= 256; ++s) {
        const double c2 = p->cs2_0 + (c2max - p->cs2_0) * s / 256.0;
        double see, sep, spp;
        modeq_block(c2, p->rate_bulk, p->rate_ghost, see, sep, spp);
        if (see < 0.0 || spp < 0.0 || see * spp - sep * sep < -1e-12 * (see * spp + 1e-300))
            return fail(FLB_ERR_INVALID_ARG,
                        "the (e, eps) noise covariance is not positive semidefinite at c_s^2 = %g "
                        "for these rates",
                        c2);
    }
    a->nx = p->nx;
    a->ny = p->ny;
    a->rho0 = p->rho0;
    a->kT = p->kT;
    a->cs2_0 = p->cs2_0;
    a->kappa = p->kappa;
    a->rate_bulk = p->rate_bulk;
    a->rate_shear = p->rate_shear;
    a->rate_ghost = p->rate_ghost;
    a->k0 = (uint32_t)(p->seed & 0xffffffffu);
    a->k1 = (uint32_t)(p->seed >> 32);
    using L = Lattice<0>;
    const double lam[4] = {p->rate_shear, p->rate_shear, p->rate_ghost, p->rate_ghost};
    for (int k = 0; k < 4; ++k)
        a->amp[k] = std::sqrt(p->rho0 * p->kT * L::N[4 + k] * lam[k] * (2.0 - lam[k]) / CS2);
    return FLB_OK;
}

// The filtered noise fields of a batch of nb steps follow its nb complex
// spectrum pairs in the work buffer.
void* modeq_fields(const ModEqArgs& a, void* work, int nb) {
    const size_t V = (size_t)a.nx * a.ny;
    const size_t csize = a.prec == 0 ? 2 * sizeof(float) : 2 * sizeof(double);
    return (char*)work + (size_t)nb * 2 * V * csize;
}

flb_status modeq_work_ok(const ModEqArgs& a, const void* work, size_t work_bytes) {
    if (a.kT == 0.0) return FLB_OK;
    if (!work) return fail(FLB_ERR_INVALID_ARG, "work is NULL");
    if (!aligned(work)) return fail(FLB_ERR_INVALID_ARG, "work must be 256-byte aligned");
    if (work_bytes < modeq_work_bytes(a.nx, a.ny, a.prec))
        return fail(FLB_ERR_INVALID_ARG, "work holds %zu bytes, %zu needed", work_bytes,
                    modeq_work_bytes(a.nx, a.ny, a.prec));
    return FLB_OK;
}

}  // namespace

flb_status flb_modeq_work_bytes(const flb_modeq_params* p, size_t* bytes) {
    ModEqArgs a{};
    if (!bytes) return fail(FLB_ERR_INVALID_ARG, "NULL bytes");
    const flb_status r = modeq_args(p, &a);
    if (r != FLB_OK) return r;
    *bytes = modeq_work_bytes(a.nx, a.ny, a.prec);
    return FLB_OK;
}

flb_status flb_modeq_noise(const flb_modeq_params* p, uint64_t step, void* xi, void* work,
                           size_t work_bytes, void* stream) {
    ModEqArgs a{};
    flb_status r = modeq_args(p, &a);
    if (r != FLB_OK) return r;
    if (!xi || !work) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (!aligned(work)) return fail(FLB_ERR_INVALID_ARG, "work must be 256-byte aligned");
    const size_t rsize = a.prec == 0 ? sizeof(float) : sizeof(double);
    if ((uintptr_t)xi % rsize)
        return fail(FLB_ERR_INVALID_ARG, "xi must be aligned to its %zu-byte reals", rsize);
    if (work_bytes < modeq_work_bytes(a.nx, a.ny, a.prec))
        return fail(FLB_ERR_INVALID_ARG, "work too small");
    HIP_TRY(launch_modeq_noise(a, p->precision, (uint32_t)step, 1, work, xi, (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_modeq_moments(const flb_modeq_params* p, const void* f, double* m, void* stream) {
    ModEqArgs a{};
    flb_status r = modeq_args(p, &a);
    if (r != FLB_OK) return r;
    if (!f || !m) return fail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (!aligned(f)) return fail(FLB_ERR_INVALID_ARG, "populations must be 256-byte aligned");
    if ((uintptr_t)m % sizeof(double)) return fail(FLB_ERR_INVALID_ARG, "m must be 8-byte aligned");
    HIP_TRY(launch_modeq_moments(a, p->precision, f, m, (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_modeq_step(const flb_modeq_params* p, const void* fin, void* fout, uint64_t step,
                          void* work, size_t work_bytes, void* stream) {
    ModEqArgs a{};
    flb_status r = modeq_args(p, &a);
    if (r != FLB_OK) return r;
    if (!fin || !fout) return fail(FLB_ERR_INVALID_ARG, "NULL populations");
    if (fin == fout) return fail(FLB_ERR_INVALID_ARG, "fin and fout must differ");
    if (!aligned(fin) || !aligned(fout))
        return fail(FLB_ERR_INVALID_ARG, "populations must be 256-byte aligned");
    if ((r = modeq_work_ok(a, work, work_bytes)) != FLB_OK) return r;
    const hipStream_t st = (hipStream_t)stream;
    void* xi = nullptr;
    if (a.kT > 0.0) {
        xi = modeq_fields(a, work, 1);
        HIP_TRY(launch_modeq_noise(a, p->precision, (uint32_t)step, 1, work, xi, st));
    }
    HIP_TRY(launch_modeq_step(a, p->precision, fin, fout, (uint32_t)step, xi, st));
    return FLB_OK;
}

}  // extern "C"

// ----------------------------------------- modified-equilibrium step without allocation
//
// The noise work of flb_modeq_step (the two complex noise spectra and the
// filtered fields, 48 V bytes) lives in a fixed device array of this file
// instead of a caller buffer.  Each GPU holds its own copy of the array from
// the library's first use on it until the process ends.  In host code the
// array's name is only a stand-in: its device address is looked up once per
// device with hipGetSymbolAddress and that address is what the kernels get.

namespace {

constexpr size_t MODEQ_STATIC_BYTES = (size_t)16 << 20;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[MODEQ_STATIC_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the current device (looked up on the first
// call there, with that device current).
flb_status static_scratch(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(FLB_ERR_UNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                    MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(FLB_ERR_HIP, "hipGetSymbolAddress returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FLB_OK;
}

}  // namespace

extern "C" {

flb_status flb_modeq_static_work_bytes(size_t* bytes) {
    if (!bytes) return fail(FLB_ERR_INVALID_ARG, "NULL bytes");
    *bytes = MODEQ_STATIC_BYTES;
    return FLB_OK;
}

flb_status flb_modeq_step_noalloc(const flb_modeq_params* p, const void* fin, void* fout,
                                  uint64_t step, void* stream) {
    ModEqArgs a{};
    flb_status r = modeq_args(p, &a);
    if (r != FLB_OK) return r;
    if (!fin || !fout) return fail(FLB_ERR_INVALID_ARG, "NULL populations");
    if (fin == fout) return fail(FLB_ERR_INVALID_ARG, "fin and fout must differ");
    if (!aligned(fin) || !aligned(fout))
        return fail(FLB_ERR_INVALID_ARG, "populations must be 256-byte aligned");
    const size_t need = a.kT > 0.0 ? modeq_work_bytes(a.nx, a.ny, a.prec) : 0;
    if (need > MODEQ_STATIC_BYTES)
        return fail(FLB_ERR_INVALID_ARG,
                    "the step needs %zu bytes of noise work, the fixed device array holds %zu "
                    "(%d x %d sites is more than %d V <= %zu allows)",
                    need, MODEQ_STATIC_BYTES, a.nx, a.ny, a.prec == 0 ? 24 : 48,
                    MODEQ_STATIC_BYTES);
    const hipStream_t st = (hipStream_t)stream;
    void* xi = nullptr;
    if (a.kT > 0.0) {
        void* work = nullptr;
        if ((r = static_scratch(&work)) != FLB_OK) return r;
        // every byte the noise kernels read is written first in the same call
        // (spectra by the row transform, fields by the inverse), so nothing
        // has to be cleared
        xi = modeq_fields(a, work, 1);
        HIP_TRY(launch_modeq_noise(a, p->precision, (uint32_t)step, 1, work, xi, st));
    }
    HIP_TRY(launch_modeq_step(a, p->precision, fin, fout, (uint32_t)step, xi, st));
    return FLB_OK;
}

flb_status flb_modeq_run(const flb_modeq_params* p, void* f, void* tmp, uint64_t step0,
                         int32_t nsteps, void* work, size_t work_bytes, void* stream) {
    ModEqArgs a{};
    flb_status r = modeq_args(p, &a);
    if (r != FLB_OK) return r;
    if (!f || !tmp || f == tmp) return fail(FLB_ERR_INVALID_ARG, "f and tmp must be distinct");
    if (!aligned(f) || !aligned(tmp))
        return fail(FLB_ERR_INVALID_ARG, "populations must be 256-byte aligned");
    if (nsteps < 0) return fail(FLB_ERR_INVALID_ARG, "nsteps must be >= 0");
    if ((r = modeq_work_ok(a, work, work_bytes)) != FLB_OK) return r;
    const hipStream_t st = (hipStream_t)stream;
    const size_t V = (size_t)a.nx * a.ny;
    const size_t rsize = a.prec == 0 ? sizeof(float) : sizeof(double);
    // noise batches of up to MODEQ_MAX_BATCH steps, as many as work holds
    size_t fit = a.kT > 0.0 ? work_bytes / modeq_work_bytes(a.nx, a.ny, a.prec) : 1;
    const int nb_max = (int)(fit < (size_t)MODEQ_MAX_BATCH ? fit : MODEQ_MAX_BATCH);
    for (int32_t k0 = 0; k0 < nsteps; k0 += nb_max) {
        const int nb = nsteps - k0 < nb_max ? nsteps - k0 : nb_max;
        char* xi = nullptr;
        if (a.kT > 0.0) {
            xi = (char*)modeq_fields(a, work, nb);
            HIP_TRY(launch_modeq_noise(a, p->precision, (uint32_t)(step0 + k0), nb, work, xi, st));
        }
        for (int b = 0; b < nb; ++b) {
            const int32_t k = k0 + b;
            const void* in = (k % 2 == 0) ? f : tmp;
            void* out = (k % 2 == 0) ? tmp : f;
            HIP_TRY(launch_modeq_step(a, p->precision, in, out, (uint32_t)(step0 + k),
                                      xi ? xi + (size_t)b * 2 * V * rsize : nullptr, st));
        }
    }
    if (nsteps % 2) {
        const size_t bytes = (size_t)9 * a.nx * a.ny * (p->precision == FLB_FP64 ? 8 : 4);
        HIP_TRY(hipMemcpyAsync(f, tmp, bytes, hipMemcpyDeviceToDevice, st));
    }
    return FLB_OK;
}

flb_status flb_destroy(flb_handle* h) {
    if (!h) return FLB_OK;
    release_graphs(h);
    if (h->aux) {
        (void)hipStreamSynchronize(h->aux);
        (void)hipStreamDestroy(h->aux);
    }
    delete h;
    return FLB_OK;
}

}  // extern "C"
