// Batched replicas: many independent ideal-gas lattices of uneven size
// advanced by one persistent launch per step.
//
// Every replica's sites are cut into tiles of BT = 256 consecutive sites
// (x fastest), and its n tiles are dealt to c = ceil(n / CH) chunks (CH = 8):
// chunk j holds tiles j, j + c, j + 2c, ... (at most CH, all of one
// replica).  The chunks of all replicas form one flat table.  Blocks working
// on neighbouring chunks at the same time therefore touch neighbouring tiles.  A grid of (compute units x blocks per CU) workgroups walks the
// table with a grid stride, one chunk at a time, so uneven replica sizes cost
// nothing beyond the last partial wave.  Replica r has its own box, Philox
// key seeds[r] and counter word 3 = r, and its populations start at element
// Q * sum_{s<r} V_s of each buffer.
// In-place pairs (optional, flb_batch_set_pairs): consecutive replicas are
// grouped up to a byte budget and each group is taken through all the steps of
// a call before the next, pairs of steps in one buffer (the first step of a
// pair stores S*_i(x) in plane opp(i) at x + c_i, the second reads plane
// opp(i) at x and stores plane i at x; every location a thread writes is one
// only it reads, just before), so that a group's working set can stay in the
// last-level cache.  The noise counters hold the global step, so the result
// is the same bits in either schedule.
// Statistics: a thread sums the moments of its CH sites in registers; a
// sampled step adds each chunk's 2Q FP64 block sums to a value-major table
// partial[k][chunk] (one block reduction per chunk, the chunk's own slots),
// and at the end of a call k_batch_fold adds, per replica and value, the sum
// over the replica's chunks (fixed order) to an FP64 accumulator and clears
// the slots.  Either schedule adds the same chunk sums in the same step
// order, so the statistics are bitwise the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/flb.h"
#include "device.h"
#include "internal.h"

namespace flb {

constexpr int BT = 256;   // sites per tile (one per thread)
constexpr int CH = 8;     // tiles per chunk

struct RepInfo {
    int32_t nx, ny, nz;
    uint32_t V;
    uint64_t off;          // element offset of the replica in a population buffer
    uint32_t key0, key1;
    uint32_t chunk0, nchunks;
    uint32_t inv_nx, inv_ny;   // ceil(2^32 / n): exact division for n < 256, s < 2^24
};

__device__ __forceinline__ uint32_t div_small(uint32_t s, uint32_t inv) { return __umulhi(s, inv); }

// Periodic neighbourhood of site s = x + nx (y + ny z) of one replica, in
// bytes: s4 = s sizeof(Real) and the wrapped byte steps to x -+ 1, y -+ 1 and
// z -+ 1 (modulo 2^32), each a selection between two uniform values, so that
// the byte offset of x + c is s4 plus up to three of them (no multiplies;
// the partial sums are shared between directions).
template <typename Real>
struct Nbr {
    uint32_t s4, dx[2], dy[2], dz[2];
    __device__ __forceinline__ Nbr(uint32_t s, int x, int y, int z, const struct RepInfo& R);
    __device__ __forceinline__ uint32_t at(int cx, int cy, int cz) const {
        uint32_t o = s4;
        if (cz) o += dz[cz > 0];
        if (cy) o += dy[cy > 0];
        if (cx) o += dx[cx > 0];
        return o;
    }
};
template <typename Real>
__device__ __forceinline__ Nbr<Real>::Nbr(uint32_t s, int x, int y, int z, const RepInfo& R) {
    constexpr uint32_t E = sizeof(Real);
    const uint32_t ex = E, ey = E * (uint32_t)R.nx, ez = ey * (uint32_t)R.ny;
    const uint32_t wx = ey - ex, wy = ez - ey, wz = E * R.V - ez;   // a wrap: period minus a step
    s4 = s * E;
    dx[0] = x == 0 ? wx : 0u - ex;
    dx[1] = x == R.nx - 1 ? 0u - wx : ex;
    dy[0] = y == 0 ? wy : 0u - ey;
    dy[1] = y == R.ny - 1 ? 0u - wy : ey;
    dz[0] = z == 0 ? wz : 0u - ez;
    dz[1] = z == R.nz - 1 ? 0u - wz : ez;
}

// The populations of one replica (Q planes of V sites from rep) as a buffer
// resource: an access is the resource plus a uniform byte offset (plane i:
// i V sizeof(Real), an SGPR) plus the lane's 32-bit byte offset, so no lane
// forms a 64-bit address.  The record count is the replica's population
// bytes (a replica has V < 2^24 sites).  V is made opaque to the compiler by
// the caller once per tile (an empty asm on an SGPR), so that the plane
// offsets are formed next to their accesses instead of being hoisted out of
// the tile loop and held.  Word 3 of the resource is the CDNA raw-buffer
// format (32-bit data format, no swizzle, no stride).
// The record count and the scalar offsets are unsigned 32-bit fields of the
// hardware (V < 2^24 sites, so Q V sizeof(Real) < 2^32); the builtins take
// them as int, so values above 2^31 pass through the cast bit for bit.
template <int LAT, typename Real>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rep_rsrc(const Real* rep, uint32_t V) {
    const uint32_t bytes = (uint32_t)Lattice<LAT>::Q * V * (uint32_t)sizeof(Real);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<Real*>(rep), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ uint32_t plane_soff(uint32_t Vr, int i, uint32_t esize) {
    return (uint32_t)i * Vr * esize;
}
__device__ __forceinline__ float rep_ld(__amdgpu_buffer_rsrc_t r, uint32_t Vr, int i, uint32_t boff,
                                        float) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)boff, (int)plane_soff(Vr, i, 4), 0));
}
__device__ __forceinline__ double rep_ld(__amdgpu_buffer_rsrc_t r, uint32_t Vr, int i,
                                         uint32_t boff, double) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 w = __builtin_amdgcn_raw_buffer_load_b64(r, (int)boff, (int)plane_soff(Vr, i, 8), 0);
    return __longlong_as_double((long long)(((unsigned long long)w.y << 32) | w.x));
}
__device__ __forceinline__ void rep_st(__amdgpu_buffer_rsrc_t r, uint32_t Vr, int i, uint32_t boff,
                                       float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)boff, (int)plane_soff(Vr, i, 4), 0);
}
__device__ __forceinline__ void rep_st(__amdgpu_buffer_rsrc_t r, uint32_t Vr, int i, uint32_t boff,
                                       double v) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    u2 w;
    w.x = (unsigned int)b;
    w.y = (unsigned int)(b >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)boff, (int)plane_soff(Vr, i, 8), 0);
}

template <int LAT, typename Real>
__device__ __forceinline__ void rep_pull(__amdgpu_buffer_rsrc_t rep, uint32_t Vr,
                                         const Nbr<Real>& nb, Real (&f)[Lattice<LAT>::Q]) {
    using L = Lattice<LAT>;
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        f[i] = rep_ld(rep, Vr, i, nb.at(-L::cx[i], -L::cy[i], -L::cz[i]), Real(0));
}

template <int LAT, typename Real, bool STATS>
__global__ __launch_bounds__(BT) void k_batch_step(const Real* __restrict__ fin,
                                                   Real* __restrict__ fout,
                                                   const RepInfo* __restrict__ reps,
                                                   const uint32_t* __restrict__ chunk_rep,
                                                   uint32_t nchunks, CollideParams<Real> P,
                                                   StepIndex st, double* __restrict__ partial) {
    using L = Lattice<LAT>;
    using M = Moments<LAT, Real>;
    constexpr int Q = L::Q, D = L::D;
    constexpr int LDS1 = 4 * (BT / 64) * 2 * Q;
    __shared__ double lds_stats[STATS ? 2 * LDS1 : 1];
    const uint32_t step = st.get();
    uint32_t it = 0;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x, ++it) {
        const uint32_t r = chunk_rep[c];
        const RepInfo R = reps[r];
        const uint32_t s0 = (c - R.chunk0) * (uint32_t)BT;
        const uint32_t ds = R.nchunks * (uint32_t)BT;
        Real v[STATS ? 2 * Q : 1];
        if constexpr (STATS) {
#pragma unroll
            for (int k = 0; k < 2 * Q; ++k) v[k] = Real(0);
        }
#pragma unroll 1
        for (int tt = 0; tt < CH; ++tt) {
            if (s0 + (uint32_t)tt * ds >= R.V) break;   // chunk with fewer tiles (uniform)
            uint32_t Vr = R.V;
            asm volatile("" : "+s"(Vr));
            const uint32_t s = s0 + (uint32_t)tt * ds + threadIdx.x;
            if (s < R.V) {
                const uint32_t yz = div_small(s, R.inv_nx);
                const int x = (int)(s - yz * (uint32_t)R.nx);
                const uint32_t z = div_small(yz, R.inv_ny);
                const int y = (int)(yz - z * (uint32_t)R.ny);
                Real f[Q], m[Q];
                rep_pull<LAT, Real>(rep_rsrc<LAT, Real>(fin + R.off, R.V), Vr,
                                    Nbr<Real>(s, x, y, (int)z, R), f);
                M::forward(f, m);
                if constexpr (STATS) {
#pragma unroll
                    for (int a = 0; a < Q; ++a) {
                        v[a] += m[a];
                        v[Q + a] += m[a] * m[a];
                    }
                }
                Real zn[2 * L::NPAIR];
                if (P.noise_on) site_normals<L::NPAIR, Real>(s, step, 0u, r, R.key0, R.key1, zn);
                const Real F[D] = {};
                collide_moments<LAT, Real, false>(m, F, zn, P);
                M::inverse(m, f);
                const __amdgpu_buffer_rsrc_t out = rep_rsrc<LAT, Real>(fout + R.off, R.V);
                const uint32_t s4 = s * (uint32_t)sizeof(Real);
                uint32_t Vs = Vr;   // the store offsets are not those of the loads
                asm volatile("" : "+s"(Vs));
#pragma unroll
                for (int i = 0; i < Q; ++i) rep_st(out, Vs, i, s4, f[i]);
            }
        }
        // the two LDS buffers alternate: the barrier inside the finish of
        // chunk j + 1 orders the reads of chunk j before the writes of j + 2
        if constexpr (STATS) {
            double* lds = lds_stats + (it & 1) * LDS1;
            rows_to_lds<2 * Q>(v, lds);
            lds_rows_finish<2 * Q, BT, true>(lds, partial + c, nchunks);
        }
    }
}

// One step of an in-place pair on the chunks [c0, c1) of the single buffer f
// (not restrict: a thread's stores alias its own earlier loads).  PH 0 pulls
// from the ordinary layout and stores S*_i(x) in plane opp(i) at x + c_i; PH 1
// reads plane opp(i) at x and stores plane i at x.  The per-site arithmetic
// and the statistics are those of k_batch_step.
template <int LAT, typename Real, bool STATS, int PH>
__global__ __launch_bounds__(BT) void k_batch_step_ip(Real* f, const RepInfo* __restrict__ reps,
                                                      const uint32_t* __restrict__ chunk_rep,
                                                      uint32_t c0, uint32_t c1, uint32_t nchunks,
                                                      CollideParams<Real> P, StepIndex st,
                                                      double* __restrict__ partial) {
    using L = Lattice<LAT>;
    using M = Moments<LAT, Real>;
    constexpr int Q = L::Q, D = L::D;
    constexpr int LDS1 = 4 * (BT / 64) * 2 * Q;
    __shared__ double lds_stats[STATS ? 2 * LDS1 : 1];
    const uint32_t step = st.get();
    uint32_t it = 0;
    for (uint32_t c = c0 + blockIdx.x; c < c1; c += gridDim.x, ++it) {
        const uint32_t r = chunk_rep[c];
        const RepInfo R = reps[r];
        const uint32_t s0 = (c - R.chunk0) * (uint32_t)BT;
        const uint32_t ds = R.nchunks * (uint32_t)BT;
        const __amdgpu_buffer_rsrc_t rb = rep_rsrc<LAT, Real>(f + R.off, R.V);
        Real v[STATS ? 2 * Q : 1];
        if constexpr (STATS) {
#pragma unroll
            for (int k = 0; k < 2 * Q; ++k) v[k] = Real(0);
        }
#pragma unroll 1
        for (int tt = 0; tt < CH; ++tt) {
            if (s0 + (uint32_t)tt * ds >= R.V) break;   // chunk with fewer tiles (uniform)
            uint32_t Vr = R.V;
            asm volatile("" : "+s"(Vr));
            const uint32_t s = s0 + (uint32_t)tt * ds + threadIdx.x;
            if (s < R.V) {
                const uint32_t yz = div_small(s, R.inv_nx);
                const int x = (int)(s - yz * (uint32_t)R.nx);
                const uint32_t z = div_small(yz, R.inv_ny);
                const int y = (int)(yz - z * (uint32_t)R.ny);
                Real fl[Q], m[Q];
                if constexpr (PH == 0) {
                    rep_pull<LAT, Real>(rb, Vr, Nbr<Real>(s, x, y, (int)z, R), fl);
                } else {
                    // local accesses: one lane offset for every plane
                    const uint32_t s4 = s * (uint32_t)sizeof(Real);
#pragma unroll
                    for (int i = 0; i < Q; ++i) fl[i] = rep_ld(rb, Vr, L::opp[i], s4, Real(0));
                }
                M::forward(fl, m);
                if constexpr (STATS) {
#pragma unroll
                    for (int a = 0; a < Q; ++a) {
                        v[a] += m[a];
                        v[Q + a] += m[a] * m[a];
                    }
                }
                Real zn[2 * L::NPAIR];
                if (P.noise_on) site_normals<L::NPAIR, Real>(s, step, 0u, r, R.key0, R.key1, zn);
                const Real F[D] = {};
                collide_moments<LAT, Real, false>(m, F, zn, P);
                M::inverse(m, fl);
                if constexpr (PH == 0) {
                    // neighbourhood formed again after the collision (not held
                    // in registers through it)
                    int xs = x;
                    asm volatile("" : "+v"(xs));
                    const Nbr<Real> nb(s, xs, y, (int)z, R);
                    uint32_t Vs = Vr;   // the store offsets are not those of the loads
                    asm volatile("" : "+s"(Vs));
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        rep_st(rb, Vs, L::opp[i], nb.at(L::cx[i], L::cy[i], L::cz[i]), fl[i]);
                } else {
                    const uint32_t s4 = s * (uint32_t)sizeof(Real);
                    uint32_t Vs = Vr;
                    asm volatile("" : "+s"(Vs));
#pragma unroll
                    for (int i = 0; i < Q; ++i) rep_st(rb, Vs, i, s4, fl[i]);
                }
            }
        }
        if constexpr (STATS) {
            double* lds = lds_stats + (it & 1) * LDS1;
            rows_to_lds<2 * Q>(v, lds);
            lds_rows_finish<2 * Q, BT, true>(lds, partial + c, nchunks);
        }
    }
}

// acc[r][k] += sum over replica r's chunks (fixed order) of partial[k][chunk],
// then those slots are cleared.  One block per (value k, replica r).
__global__ void k_batch_fold(double* __restrict__ partial, const RepInfo* __restrict__ reps,
                             uint32_t nchunks, int nvals, double* __restrict__ acc_out) {
    __shared__ double red[256];
    const int k = blockIdx.x, r = blockIdx.y;
    const RepInfo R = reps[r];
    double* col = partial + (size_t)k * nchunks + R.chunk0;
    double acc = 0.0;
    for (uint32_t t = threadIdx.x; t < R.nchunks; t += 256) {
        acc += col[t];
        col[t] = 0.0;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc_out[(size_t)r * nvals + k] += red[0];
}

template <int LAT, typename Real>
__global__ void k_batch_init(Real* __restrict__ f, const RepInfo* __restrict__ reps,
                             const uint32_t* __restrict__ chunk_rep, uint32_t nchunks) {
    using L = Lattice<LAT>;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const RepInfo R = reps[chunk_rep[c]];
        const uint32_t s0 = (c - R.chunk0) * (uint32_t)BT;
        for (int tt = 0; tt < CH; ++tt) {
            const uint32_t s = s0 + (uint32_t)tt * R.nchunks * (uint32_t)BT + threadIdx.x;
            if (s < R.V) {
#pragma unroll
                for (int i = 0; i < L::Q; ++i) f[R.off + (size_t)i * R.V + s] = Real(0);
            }
        }
    }
}

}  // namespace flb

using namespace flb;

namespace {

flb_status bfail(flb_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_last_error(buf);
    return s;
}

#define BHIP(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return bfail(FLB_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
constexpr double CS2 = 1.0 / 3.0;

struct Layout {
    std::vector<RepInfo> reps;
    std::vector<uint32_t> chunk_rep;
    size_t elems;          // reals per population buffer
    size_t reps_off, tiles_off, ctr_off, scratch_bytes, stats_bytes;
};

flb_status batch_layout(const flb_params* p, int32_t nrep, const int32_t* dims,
                        const uint64_t* seeds, Layout* L) {
    if (!p || !dims) return bfail(FLB_ERR_INVALID_ARG, "NULL argument");
    if (nrep < 1 || nrep > 4096) return bfail(FLB_ERR_INVALID_ARG, "nrep = %d", nrep);
    if (p->force_model != FLB_IDEAL)
        return bfail(FLB_ERR_UNSUPPORTED, "batched replicas are ideal-gas only");
    flb_params q = *p;
    const int Q = p->lattice == FLB_D2Q9 ? 9 : 19;
    L->reps.clear();
    L->chunk_rep.clear();
    size_t off = 0;
    uint32_t chunk = 0;
    for (int r = 0; r < nrep; ++r) {
        q.nx = dims[3 * r];
        q.ny = dims[3 * r + 1];
        q.nz = dims[3 * r + 2];
        size_t a, b, c;
        flb_status st = flb_query_sizes(&q, &a, &b, &c);
        if (st != FLB_OK) {
            const std::string why = flb_last_error();
            return bfail(st, "replica %d: %s", r, why.c_str());
        }
        if (q.nx >= 256 || q.ny >= 256 || q.nz >= 65536)
            return bfail(FLB_ERR_INVALID_ARG, "replica %d: batched boxes need nx, ny < 256", r);
        RepInfo R{};
        R.nx = q.nx;
        R.ny = q.ny;
        R.nz = q.nz;
        R.V = (uint32_t)q.nx * q.ny * q.nz;
        if (R.V >= (1u << 24)) return bfail(FLB_ERR_INVALID_ARG, "replica %d too large", r);
        R.off = off;
        const uint64_t seed = seeds ? seeds[r] : (uint64_t)r;
        R.key0 = (uint32_t)(seed & 0xffffffffu);
        R.key1 = (uint32_t)(seed >> 32);
        R.chunk0 = chunk;
        R.nchunks = (R.V + CH * BT - 1) / (CH * BT);
        R.inv_nx = (uint32_t)(((1ull << 32) + R.nx - 1) / R.nx);
        R.inv_ny = (uint32_t)(((1ull << 32) + R.ny - 1) / R.ny);
        for (uint32_t c = 0; c < R.nchunks; ++c) L->chunk_rep.push_back((uint32_t)r);
        chunk += R.nchunks;
        off += (size_t)Q * R.V;
        L->reps.push_back(R);
    }
    L->elems = off;
    size_t s = 0;
    L->ctr_off = s;
    s += ALIGN;
    L->reps_off = s;
    s += align_up(L->reps.size() * sizeof(RepInfo));
    L->tiles_off = s;
    s += align_up(L->chunk_rep.size() * sizeof(uint32_t));
    L->scratch_bytes = s;
    L->stats_bytes = align_up(((size_t)chunk * 2 * Q + (size_t)nrep * 2 * Q) * sizeof(double));
    return FLB_OK;
}

}  // namespace

// Consecutive replicas [r0, r1), whose chunks are [c0, c1).
struct BatchGroup {
    uint32_t r0, r1, c0, c1;
};

struct flb_batch {
    flb_params p;
    int q, nrep;
    size_t rb;
    Layout L;
    void* fa;
    void* fb;
    bool cur_a;
    char* scratch;
    double* stats;
    RepInfo* reps_dev;
    uint32_t* tiles_dev;
    unsigned long long* ctr_dev;
    uint32_t nchunks;
    uint64_t step;
    int64_t nsamples;
    int grid_cfg;          // persistent grid of plain steps
    int grid_cfg_stats;    // persistent grid of steps with statistics
    int ncu;
    uint64_t pair_bytes;   // > 0: in-place pairs, groups of replicas up to this many bytes
    int pair_cfg;          // persistent grid of the in-place steps
    std::vector<BatchGroup> groups;
    // captured steps, one graph per current buffer (index cur_a): kernel
    // arguments hold the buffer pointers
    hipGraph_t graph[2];
    hipGraphExec_t gexec[2];
    int64_t graph_steps, graph_samples;
    void* cur() const { return cur_a ? fa : fb; }
    void* other() const { return cur_a ? fb : fa; }
};

namespace {

void release_batch_graphs(flb_batch* b) {
    for (int k = 0; k < 2; ++k) {
        if (b->gexec[k]) (void)hipGraphExecDestroy(b->gexec[k]);
        if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
        b->gexec[k] = nullptr;
        b->graph[k] = nullptr;
    }
}

constexpr int N_GRID_CFG = 4;
constexpr int GRID_PER_CU[N_GRID_CFG] = {8, 4, 16, 2};

template <int LAT, typename Real>
CollideParams<Real> batch_collide_params(const flb_batch* b) {
    CollideParams<Real> P;
    const flb_params& p = b->p;
    P.rho0 = (Real)p.rho0;
    P.lam_bulk = (Real)p.rate_bulk;
    P.lam_shear = (Real)p.rate_shear;
    P.lam_ghost = (Real)p.rate_ghost;
    const double lam[3] = {p.rate_bulk, p.rate_shear, p.rate_ghost};
    for (int c = 0; c < 3; ++c)
        P.amp_cls[c] = (Real)std::sqrt(p.kT * lam[c] * (2.0 - lam[c]) / CS2);
    P.noise_on = p.kT > 0.0;
    P.noise_local = p.noise_rho_local ? 1 : 0;
    P.key0 = P.key1 = 0;   // per replica
    P.replica = 0;
    P.nonfinite = nullptr;
    return P;
}

template <int LAT, typename Real>
void batch_launch(flb_batch* b, int cfg, const void* fin, void* fout,
                  const unsigned long long* step_dev, unsigned long long step_host,
                  double* partial, hipStream_t st) {
    const CollideParams<Real> P = batch_collide_params<LAT, Real>(b);
    StepIndex si{step_dev, step_host};
    const uint32_t grid = std::min<uint32_t>(b->nchunks, (uint32_t)(b->ncu * GRID_PER_CU[cfg]));
    if (partial)
        hipLaunchKernelGGL((k_batch_step<LAT, Real, true>), dim3(grid), dim3(BT), 0, st,
                           (const Real*)fin, (Real*)fout, b->reps_dev, b->tiles_dev, b->nchunks, P,
                           si, partial);
    else
        hipLaunchKernelGGL((k_batch_step<LAT, Real, false>), dim3(grid), dim3(BT), 0, st,
                           (const Real*)fin, (Real*)fout, b->reps_dev, b->tiles_dev, b->nchunks, P,
                           si, partial);
}

template <int LAT, typename Real>
void batch_ip_launch(flb_batch* b, int cfg, int phase, const BatchGroup& G, void* f,
                     const unsigned long long* step_dev, unsigned long long step_host,
                     double* partial, hipStream_t st) {
    const CollideParams<Real> P = batch_collide_params<LAT, Real>(b);
    StepIndex si{step_dev, step_host};
    const uint32_t n = G.c1 - G.c0;
    const uint32_t grid = std::min<uint32_t>(n, (uint32_t)(b->ncu * GRID_PER_CU[cfg]));
    Real* fr = (Real*)f;
#define FLB_BATCH_IP(S, PH)                                                                   \
    hipLaunchKernelGGL((k_batch_step_ip<LAT, Real, S, PH>), dim3(grid), dim3(BT), 0, st, fr,  \
                       b->reps_dev, b->tiles_dev, G.c0, G.c1, b->nchunks, P, si, partial)
    if (partial) {
        if (phase == 0) FLB_BATCH_IP(true, 0);
        else FLB_BATCH_IP(true, 1);
    } else {
        if (phase == 0) FLB_BATCH_IP(false, 0);
        else FLB_BATCH_IP(false, 1);
    }
#undef FLB_BATCH_IP
}

hipError_t batch_ip_one(flb_batch* b, int cfg, int phase, const BatchGroup& G, void* f,
                        const unsigned long long* step_dev, unsigned long long step_host,
                        double* partial, hipStream_t st) {
    const int lat = b->p.lattice, prec = b->p.precision;
    if (lat == 0 && prec == 0) batch_ip_launch<0, float>(b, cfg, phase, G, f, step_dev, step_host, partial, st);
    else if (lat == 0) batch_ip_launch<0, double>(b, cfg, phase, G, f, step_dev, step_host, partial, st);
    else if (prec == 0) batch_ip_launch<1, float>(b, cfg, phase, G, f, step_dev, step_host, partial, st);
    else batch_ip_launch<1, double>(b, cfg, phase, G, f, step_dev, step_host, partial, st);
    return hipGetLastError();
}

// Consecutive replicas up to `bytes` of populations per group (a replica
// larger than that forms a group of its own).
std::vector<BatchGroup> batch_groups(const flb_batch* b, uint64_t bytes) {
    std::vector<BatchGroup> out;
    const std::vector<RepInfo>& R = b->L.reps;
    uint32_t r0 = 0;
    uint64_t acc = 0;
    for (uint32_t r = 0; r < (uint32_t)R.size(); ++r) {
        const uint64_t rb = (uint64_t)b->q * R[r].V * b->rb;
        if (r > r0 && acc + rb > bytes) {
            out.push_back({r0, r, R[r0].chunk0, R[r].chunk0});
            r0 = r;
            acc = 0;
        }
        acc += rb;
    }
    out.push_back({r0, (uint32_t)R.size(), R[r0].chunk0, b->nchunks});
    return out;
}

hipError_t batch_one(flb_batch* b, int cfg, const void* fin, void* fout,
                     const unsigned long long* step_dev, unsigned long long step_host,
                     double* partial, hipStream_t st) {
    const int lat = b->p.lattice, prec = b->p.precision;
    if (lat == 0 && prec == 0) batch_launch<0, float>(b, cfg, fin, fout, step_dev, step_host, partial, st);
    else if (lat == 0) batch_launch<0, double>(b, cfg, fin, fout, step_dev, step_host, partial, st);
    else if (prec == 0) batch_launch<1, float>(b, cfg, fin, fout, step_dev, step_host, partial, st);
    else batch_launch<1, double>(b, cfg, fin, fout, step_dev, step_host, partial, st);
    return hipGetLastError();
}

double* batch_acc(flb_batch* b) { return b->stats + (size_t)b->nchunks * 2 * b->q; }

flb_status batch_run(flb_batch* b, int64_t nsteps, int32_t stride, bool graph_mode,
                     hipStream_t st, int64_t* samples) {
    int64_t ns = 0;
    const int nv = 2 * b->q;
    auto sampled = [stride](int64_t k) { return stride > 0 && ((k + 1) % stride) == 0; };
    auto index = [&](int64_t k) {
        return graph_mode ? (unsigned long long)k : (unsigned long long)(b->step + k);
    };
    const unsigned long long* sd = graph_mode ? b->ctr_dev : nullptr;
    int64_t k = 0;
    if (b->pair_bytes > 0 && nsteps >= 2) {
        // group by group, pairs of steps in place in the current buffer
        const int64_t np = nsteps & ~(int64_t)1;
        for (const BatchGroup& G : b->groups) {
            for (int64_t j = 0; j < np; ++j) {
                const bool sample = sampled(j);
                BHIP(batch_ip_one(b, b->pair_cfg, (int)(j & 1), G, b->cur(), sd, index(j),
                                  sample ? b->stats : nullptr, st));
            }
        }
        for (int64_t j = 0; j < np; ++j) ns += sampled(j);
        k = np;
    }
    for (; k < nsteps; ++k) {
        const bool sample = sampled(k);
        BHIP(batch_one(b, sample ? b->grid_cfg_stats : b->grid_cfg, b->cur(), b->other(), sd,
                       index(k), sample ? b->stats : nullptr, st));
        b->cur_a = !b->cur_a;
        ns += sample;
    }
    if (ns > 0) {
        hipLaunchKernelGGL(k_batch_fold, dim3(nv, b->nrep), dim3(256), 0, st, b->stats,
                           b->reps_dev, b->nchunks, nv, batch_acc(b));
        BHIP(hipGetLastError());
    }
    if (graph_mode) BHIP(launch_add_u64(b->ctr_dev, (unsigned long long)nsteps, st));
    *samples = ns;
    return FLB_OK;
}

}  // namespace

extern "C" {

flb_status flb_batch_query_sizes(const flb_params* base, int32_t nrep, const int32_t* dims,
                                 size_t* pop_bytes, size_t* scratch_bytes, size_t* stats_bytes) {
    Layout L;
    flb_status s = batch_layout(base, nrep, dims, nullptr, &L);
    if (s != FLB_OK) return s;
    const size_t rb = base->precision == FLB_FP64 ? 8 : 4;
    if (pop_bytes) *pop_bytes = align_up(L.elems * rb);
    if (scratch_bytes) *scratch_bytes = L.scratch_bytes;
    if (stats_bytes) *stats_bytes = L.stats_bytes;
    return FLB_OK;
}

flb_status flb_batch_init(const flb_params* base, int32_t nrep, const int32_t* dims,
                          const uint64_t* seeds, void* f_a, void* f_b, void* scratch,
                          void* stats, void* stream, flb_batch** out) {
    if (!out) return bfail(FLB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    auto al = [](const void* q) { return q && ((uintptr_t)q % ALIGN) == 0; };
    if (!al(f_a) || !al(f_b) || !al(scratch) || !al(stats) || f_a == f_b)
        return bfail(FLB_ERR_INVALID_ARG, "buffers must be distinct, non-NULL, 256-byte aligned");
    flb_batch* b = new (std::nothrow) flb_batch();
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "out of host memory");
    flb_status s = batch_layout(base, nrep, dims, seeds, &b->L);
    if (s != FLB_OK) {
        delete b;
        return s;
    }
    hipStream_t st = (hipStream_t)stream;
    b->p = *base;
    b->q = base->lattice == FLB_D2Q9 ? 9 : 19;
    b->nrep = nrep;
    b->rb = base->precision == FLB_FP64 ? 8 : 4;
    b->fa = f_a;
    b->fb = f_b;
    b->cur_a = true;
    b->scratch = (char*)scratch;
    b->stats = (double*)stats;
    b->reps_dev = (RepInfo*)(b->scratch + b->L.reps_off);
    b->tiles_dev = (uint32_t*)(b->scratch + b->L.tiles_off);
    b->ctr_dev = (unsigned long long*)(b->scratch + b->L.ctr_off);
    b->nchunks = (uint32_t)b->L.chunk_rep.size();
    b->step = base->step0;
    b->nsamples = 0;
    b->grid_cfg = 0;
    b->grid_cfg_stats = 0;
    b->pair_bytes = 0;
    b->pair_cfg = 2;
    b->graph[0] = b->graph[1] = nullptr;
    b->gexec[0] = b->gexec[1] = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->reps_dev, b->L.reps.data(), b->L.reps.size() * sizeof(RepInfo),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->tiles_dev, b->L.chunk_rep.data(), b->nchunks * sizeof(uint32_t),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_set_u64(b->ctr_dev, b->step, st);
    if (e == hipSuccess) e = launch_fill_zero(stats, b->L.stats_bytes, st);
    if (e == hipSuccess) {
        const uint32_t grid = std::min<uint32_t>(b->nchunks, 2048);
        if (b->p.lattice == 0 && b->p.precision == 0)
            hipLaunchKernelGGL((k_batch_init<0, float>), dim3(grid), dim3(BT), 0, st, (float*)f_a, b->reps_dev, b->tiles_dev, b->nchunks);
        else if (b->p.lattice == 0)
            hipLaunchKernelGGL((k_batch_init<0, double>), dim3(grid), dim3(BT), 0, st, (double*)f_a, b->reps_dev, b->tiles_dev, b->nchunks);
        else if (b->p.precision == 0)
            hipLaunchKernelGGL((k_batch_init<1, float>), dim3(grid), dim3(BT), 0, st, (float*)f_a, b->reps_dev, b->tiles_dev, b->nchunks);
        else
            hipLaunchKernelGGL((k_batch_init<1, double>), dim3(grid), dim3(BT), 0, st, (double*)f_a, b->reps_dev, b->tiles_dev, b->nchunks);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete b;
        return bfail(FLB_ERR_HIP, "flb_batch_init: %s", hipGetErrorString(e));
    }
    *out = b;
    return FLB_OK;
}

flb_status flb_batch_step(flb_batch* b, int64_t nsteps, int32_t stats_stride, void* stream) {
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "batch is NULL");
    if (nsteps < 0 || stats_stride < 0) return bfail(FLB_ERR_INVALID_ARG, "bad step count");
    int64_t ns = 0;
    flb_status s = batch_run(b, nsteps, stats_stride, false, (hipStream_t)stream, &ns);
    if (s != FLB_OK) return s;
    b->step += (uint64_t)nsteps;
    b->nsamples += ns;
    BHIP(launch_set_u64(b->ctr_dev, b->step, (hipStream_t)stream));
    return FLB_OK;
}

flb_status flb_batch_moments(flb_batch* b, double* mode_sum, double* mode_sumsq,
                             int64_t* nsamples, void* stream) {
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "batch is NULL");
    hipStream_t st = (hipStream_t)stream;
    const int nv = 2 * b->q;
    const double* out = batch_acc(b);
    std::vector<double> host((size_t)b->nrep * nv);
    BHIP(hipMemcpyAsync(host.data(), out, host.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    BHIP(hipStreamSynchronize(st));
    for (int r = 0; r < b->nrep; ++r)
        for (int a = 0; a < b->q; ++a) {
            if (mode_sum) mode_sum[r * b->q + a] = host[(size_t)r * nv + a];
            if (mode_sumsq) mode_sumsq[r * b->q + a] = host[(size_t)r * nv + b->q + a];
        }
    if (nsamples) *nsamples = b->nsamples;
    for (double v : host)
        if (!std::isfinite(v)) return bfail(FLB_ERR_NONFINITE, "statistics are not finite");
    return FLB_OK;
}

flb_status flb_batch_reset_stats(flb_batch* b, void* stream) {
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "batch is NULL");
    // the per-chunk table is clear between calls; the accumulators follow it
    BHIP(launch_fill_zero(batch_acc(b), (size_t)b->nrep * 2 * b->q * sizeof(double),
                          (hipStream_t)stream));
    b->nsamples = 0;
    return FLB_OK;
}

flb_status flb_batch_state(const flb_batch* b, void** cur, void** other, uint64_t* step) {
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "batch is NULL");
    if (cur) *cur = b->cur();
    if (other) *other = b->other();
    if (step) *step = b->step;
    return FLB_OK;
}

flb_status flb_batch_graph_capture(flb_batch* b, int64_t nsteps, int32_t stats_stride,
                                   void* stream) {
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "batch is NULL");
    if (nsteps <= 0 || nsteps % 2 != 0 || stats_stride < 0)
        return bfail(FLB_ERR_INVALID_ARG, "graph step count must be positive and even");
    hipStream_t st = (hipStream_t)stream;
    if (!st) return bfail(FLB_ERR_INVALID_ARG, "graph capture needs a non-null stream");
    release_batch_graphs(b);
    // one recording for each buffer the state can be in (see flb_graph_capture)
    const bool cur_a = b->cur_a;
    int64_t ns = 0;
    flb_status r = FLB_OK;
    for (int k = 0; k < 2 && r == FLB_OK; ++k) {
        b->cur_a = k == 1;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            r = bfail(FLB_ERR_HIP, "begin capture: %s", hipGetErrorString(e));
            break;
        }
        r = batch_run(b, nsteps, stats_stride, true, st, &ns);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(st, &g);
        if (r == FLB_OK && e != hipSuccess)
            r = bfail(FLB_ERR_HIP, "capture: %s", hipGetErrorString(e));
        if (r != FLB_OK) {
            if (g) (void)hipGraphDestroy(g);
            break;
        }
        b->graph[k] = g;
        e = hipGraphInstantiate(&b->gexec[k], g, nullptr, nullptr, 0);
        if (e != hipSuccess) r = bfail(FLB_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    b->cur_a = cur_a;   // nothing ran
    if (r != FLB_OK) {
        release_batch_graphs(b);
        return r;
    }
    b->graph_steps = nsteps;
    b->graph_samples = ns;
    return FLB_OK;
}

flb_status flb_batch_graph_launch(flb_batch* b, void* stream) {
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "batch is NULL");
    hipGraphExec_t ex = b->gexec[b->cur_a ? 1 : 0];
    if (!ex) return bfail(FLB_ERR_STATE, "no graph captured");
    BHIP(hipGraphLaunch(ex, (hipStream_t)stream));
    b->step += (uint64_t)b->graph_steps;
    b->nsamples += b->graph_samples;
    return FLB_OK;
}

flb_status flb_batch_autotune(flb_batch* b, int32_t repeats, int32_t* best, double* best_ms,
                              void* stream) {
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "batch is NULL");
    if (repeats < 1) repeats = 1;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    int bi[2] = {b->grid_cfg, b->grid_cfg_stats};
    float bt[2] = {1e30f, 1e30f};
    // statistics trials only add to the per-chunk table, cleared below; the
    // accumulators are not touched
    for (int mode = 0; mode < 2; ++mode) {
        double* part = mode ? b->stats : nullptr;
        for (int c = 0; c < N_GRID_CFG; ++c) {
            BHIP(batch_one(b, c, b->cur(), b->other(), nullptr, b->step, part, st));
            BHIP(hipEventRecord(e0, st));
            for (int r = 0; r < repeats; ++r)
                BHIP(batch_one(b, c, b->cur(), b->other(), nullptr, b->step, part, st));
            BHIP(hipEventRecord(e1, st));
            BHIP(hipEventSynchronize(e1));
            float ms = 0.f;
            BHIP(hipEventElapsedTime(&ms, e0, e1));
            ms /= repeats;
            if (ms < bt[mode]) {
                bt[mode] = ms;
                bi[mode] = c;
            }
        }
    }
    b->grid_cfg = bi[0];
    b->grid_cfg_stats = bi[1];
    // in-place pairs group by group, with statistics: the trials run in place
    // on a copy of the state in the other buffer (the next ordinary step
    // overwrites it), so the state is untouched
    if (b->nrep > 0) {
        BHIP(hipMemcpyAsync(b->other(), b->cur(), b->L.elems * b->rb, hipMemcpyDeviceToDevice,
                            st));
        uint64_t best_bytes = 0;
        int best_cfg = b->pair_cfg;
        float best_pair = bt[1];
        for (uint64_t mib : {64ull, 128ull, 160ull, 192ull, 224ull, 256ull, 320ull}) {
            const std::vector<BatchGroup> groups = batch_groups(b, mib << 20);
            for (int c = 0; c < N_GRID_CFG; ++c) {
                BHIP(hipEventRecord(e0, st));
                for (const BatchGroup& G : groups)
                    for (int j = 0; j < 2 * repeats; ++j)
                        BHIP(batch_ip_one(b, c, j & 1, G, b->other(), nullptr, b->step + j,
                                          b->stats, st));
                BHIP(hipEventRecord(e1, st));
                BHIP(hipEventSynchronize(e1));
                float ms = 0.f;
                BHIP(hipEventElapsedTime(&ms, e0, e1));
                ms /= 2 * repeats;
                if (ms < best_pair) {
                    best_pair = ms;
                    best_bytes = mib << 20;
                    best_cfg = c;
                }
            }
        }
        b->pair_bytes = best_bytes;
        b->pair_cfg = best_cfg;
        // the statistics trials added to the per-chunk slots, which are clear
        // between calls: clear them again
        BHIP(launch_fill_zero(b->stats, (size_t)b->nchunks * 2 * b->q * sizeof(double), st));
        BHIP(hipStreamSynchronize(st));
        b->groups = best_bytes ? batch_groups(b, best_bytes) : std::vector<BatchGroup>();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int m = 0; m < 2; ++m) {
        if (best) best[m] = bi[m];
        if (best_ms) best_ms[m] = bt[m];
    }
    return FLB_OK;
}

flb_status flb_batch_set_pairs(flb_batch* b, uint64_t pair_bytes) {
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "batch is NULL");
    b->pair_bytes = pair_bytes;
    b->groups = pair_bytes ? batch_groups(b, pair_bytes) : std::vector<BatchGroup>();
    return FLB_OK;
}
flb_status flb_batch_pairs(const flb_batch* b, uint64_t* pair_bytes, int32_t* ngroups) {
    if (!b) return bfail(FLB_ERR_INVALID_ARG, "batch is NULL");
    if (pair_bytes) *pair_bytes = b->pair_bytes;
    if (ngroups) *ngroups = (int32_t)b->groups.size();
    return FLB_OK;
}
flb_status flb_batch_destroy(flb_batch* b) {
    if (!b) return FLB_OK;
    release_batch_graphs(b);
    delete b;
    return FLB_OK;
}

}  // extern "C"
