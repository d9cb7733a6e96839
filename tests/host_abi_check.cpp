// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of the library (no GPU needed):
// every call below is answered on the host, from parameter validation, size
// queries and constant tables, before any device work.  Exit status 0 when
// every expectation holds; the sanitizers abort the program on the first
// memory error or undefined behaviour.

#include <cstdio>
#include <cstring>
#include <vector>

#include "../include/flb.h"

static int g_fail = 0;

#define EXPECT(cond)                                                              \
    do {                                                                          \
        if (!(cond)) {                                                            \
            std::fprintf(stderr, "%s:%d: expectation failed: %s (%s)\n", __FILE__, \
                         __LINE__, #cond, flb_last_error());                      \
            ++g_fail;                                                             \
        }                                                                         \
    } while (0)

static flb_params base_params(int lattice) {
    flb_params p;
    std::memset(&p, 0, sizeof p);
    p.lattice = lattice;
    p.precision = FLB_FP32;
    p.nx = 16;
    p.ny = 12;
    p.nz = lattice == FLB_D2Q9 ? 1 : 10;
    p.force_model = FLB_IDEAL;
    p.rho0 = 1.0;
    p.kT = 1e-5;
    p.rate_bulk = 1.2;
    p.rate_shear = 1.6;
    p.rate_ghost = 1.0;
    p.seed = 7;
    return p;
}

static flb_modeq_params modeq_params() {
    flb_modeq_params p;
    std::memset(&p, 0, sizeof p);
    p.nx = 8;
    p.ny = 8;
    p.precision = FLB_FP32;
    p.rho0 = 1.0;
    p.kT = 1e-5;
    p.cs2_0 = 0.07;
    p.kappa = 0.08;
    p.rate_bulk = p.rate_shear = p.rate_ghost = 1.0;
    p.seed = 3;
    return p;
}

int main() {
    // status strings, including an unknown code
    for (int s = 0; s >= -6; --s) EXPECT(flb_strerror((flb_status)s) != nullptr);

    // constant tables of both lattices; an unknown lattice is rejected
    for (int lat = 0; lat < 2; ++lat) {
        int32_t q = 0, c[3 * 19], cls[19];
        double w[19], T[19 * 19], N[19];
        EXPECT(flb_lattice_tables(lat, &q, c, w, T, N, cls) == FLB_OK);
        EXPECT(q == (lat == 0 ? 9 : 19));
        double sw = 0.0;
        for (int i = 0; i < q; ++i) sw += w[i];
        EXPECT(sw > 0.999999 && sw < 1.000001);
    }
    EXPECT(flb_lattice_tables(7, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
           FLB_ERR_INVALID_ARG);

    // sizes: valid parameters of every lattice, precision and force model
    for (int lat = 0; lat < 2; ++lat)
        for (int prec = 0; prec < 2; ++prec)
            for (int force = 0; force < 2; ++force) {
                flb_params p = base_params(lat);
                p.precision = prec;
                p.force_model = force;
                if (force) {
                    p.a = -0.01;
                    p.b = 0.1;
                    p.rho_c = 1.0;
                    p.kappa = 0.05;
                }
                size_t a = 0, b = 0, s = 0;
                EXPECT(flb_query_sizes(&p, &a, &b, &s) == FLB_OK);
                const size_t q = lat == 0 ? 9 : 19, rb = prec ? 8 : 4;
                EXPECT(a >= q * (size_t)p.nx * p.ny * p.nz * rb && a % 256 == 0);
                EXPECT(s > 0);
            }
    // ... and the rejections the header lists
    {
        flb_params bad[10];
        for (auto& p : bad) p = base_params(FLB_D3Q19);
        bad[0].lattice = 5;
        bad[1].precision = 9;
        bad[2].nx = 0;
        bad[3].rate_shear = 2.0;
        bad[4].kT = -1.0;
        bad[5].kT = 1.0;          // above rho0 cs2
        bad[6].rho0 = 0.0;
        bad[7] = base_params(FLB_D2Q9);
        bad[7].nz = 3;            // D2Q9 needs nz = 1
        bad[8].nx = bad[8].ny = bad[8].nz = 1 << 11;   // 2^33 sites
        bad[9].force_model = 4;
        for (auto& p : bad) {
            size_t a, b, s;
            EXPECT(flb_query_sizes(&p, &a, &b, &s) == FLB_ERR_INVALID_ARG);
        }
        EXPECT(flb_query_sizes(nullptr, nullptr, nullptr, nullptr) == FLB_ERR_INVALID_ARG);
    }

    // init: null, misaligned or aliased buffers are rejected before any device call
    {
        flb_params p = base_params(FLB_D3Q19);
        flb_handle* h = nullptr;
        void* A = (void*)(uintptr_t)(1u << 20);
        void* B = (void*)(uintptr_t)(2u << 20);
        void* S = (void*)(uintptr_t)(3u << 20);
        void* odd = (void*)(uintptr_t)((1u << 20) + 8);
        EXPECT(flb_init(&p, nullptr, B, S, S, nullptr, nullptr, &h) == FLB_ERR_INVALID_ARG);
        EXPECT(flb_init(&p, odd, B, S, S, nullptr, nullptr, &h) == FLB_ERR_INVALID_ARG);
        EXPECT(flb_init(&p, A, A, S, S, nullptr, nullptr, &h) == FLB_ERR_INVALID_ARG);
        EXPECT(flb_init(&p, A, B, S, S, nullptr, nullptr, nullptr) == FLB_ERR_INVALID_ARG);
        EXPECT(h == nullptr);
    }

    // calls on a null handle
    EXPECT(flb_step(nullptr, 1, 0, nullptr) == FLB_ERR_INVALID_ARG);
    EXPECT(flb_set_check(nullptr, 1, nullptr) == FLB_ERR_INVALID_ARG);
    EXPECT(flb_reset_stats(nullptr, nullptr) == FLB_ERR_INVALID_ARG);
    EXPECT(flb_graph_launch(nullptr, nullptr) == FLB_ERR_INVALID_ARG);
    EXPECT(flb_set_launch(nullptr, 0) == FLB_ERR_INVALID_ARG);
    EXPECT(flb_autotune(nullptr, 1, nullptr, nullptr, nullptr) == FLB_ERR_INVALID_ARG);

    // batched replicas: sizes for a list of uneven boxes, rejections
    {
        flb_params p = base_params(FLB_D3Q19);
        const int32_t dims[3 * 4] = {16, 16, 16, 9, 7, 5, 1, 1, 1, 40, 20, 10};
        size_t a = 0, b = 0, s = 0;
        EXPECT(flb_batch_query_sizes(&p, 4, dims, &a, &b, &s) == FLB_OK);
        EXPECT(a >= (size_t)19 * (4096 + 315 + 1 + 8000) * 4);
        const int32_t wide[3] = {256, 8, 8};   // batched boxes need nx, ny < 256
        EXPECT(flb_batch_query_sizes(&p, 1, wide, &a, &b, &s) == FLB_ERR_INVALID_ARG);
        EXPECT(flb_batch_query_sizes(&p, 0, dims, &a, &b, &s) == FLB_ERR_INVALID_ARG);
        EXPECT(flb_batch_query_sizes(&p, 4, nullptr, &a, &b, &s) == FLB_ERR_INVALID_ARG);
    }

    // modified-equilibrium model: work sizes in both precisions, rejections
    {
        flb_modeq_params p = modeq_params();
        size_t w = 0;
        EXPECT(flb_modeq_work_bytes(&p, &w) == FLB_OK && w == 24 * 64);
        p.precision = FLB_FP64;
        EXPECT(flb_modeq_work_bytes(&p, &w) == FLB_OK && w == 48 * 64);
        flb_modeq_params bad[5];
        for (auto& q : bad) q = modeq_params();
        bad[0].nx = 2048;
        bad[1].rate_bulk = 2.5;
        bad[2].kappa = 1.0;       // c_s^2(k) above 0.6
        bad[3].kT = -1.0;
        bad[4].precision = 3;
        for (auto& q : bad) EXPECT(flb_modeq_work_bytes(&q, &w) == FLB_ERR_INVALID_ARG);
        size_t fixed = 0;
        EXPECT(flb_modeq_static_work_bytes(&fixed) == FLB_OK && fixed == ((size_t)16 << 20));
        flb_modeq_params big = modeq_params();
        big.nx = 1024;
        big.ny = 1024;            // 24 V bytes above the fixed array
        void* A = (void*)(uintptr_t)(1u << 20);
        void* B = (void*)(uintptr_t)(2u << 20);
        EXPECT(flb_modeq_step_noalloc(&big, A, B, 0, nullptr) == FLB_ERR_INVALID_ARG);
        flb_modeq_params ok = modeq_params();
        EXPECT(flb_modeq_step_noalloc(&ok, A, A, 0, nullptr) == FLB_ERR_INVALID_ARG);
        EXPECT(flb_modeq_step(&ok, A, B, 0, B, 24 * 64 - 1, nullptr) == FLB_ERR_INVALID_ARG);
        EXPECT(flb_modeq_run(&ok, A, B, 0, -1, B, 24 * 64, nullptr) == FLB_ERR_INVALID_ARG);
        EXPECT(flb_modeq_noise(&ok, 0, nullptr, B, 24 * 64, nullptr) == FLB_ERR_INVALID_ARG);
    }

    // field spectra and the roofline probe reject bad shapes on the host
    EXPECT(flb_field_spectrum(nullptr, 1, 8, 8, 1, nullptr, nullptr, nullptr) == FLB_ERR_INVALID_ARG);
    EXPECT(flb_plane_stream_probe(nullptr, nullptr, 19, 1024, 1, nullptr) == FLB_ERR_INVALID_ARG);

    // the last error text is a readable string
    EXPECT(std::strlen(flb_last_error()) > 0);

    std::printf("host ABI checks: %d failed\n", g_fail);
    return g_fail == 0 ? 0 : 1;
}
