// sanitize_host_main.cpp -- drives the host logic of the library (configuration
// checks, the time-step rule, argument checks of every entry point, context
// creation and its clean-up on failure) without a GPU, for a build of the host
// code with AddressSanitizer and UndefinedBehaviorSanitizer.  On a machine
// without a GPU every call that reaches the HIP runtime returns MM_EDEVICE;
// the run checks the status codes and that nothing leaks or trips a sanitizer.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mm.h"

static int fails = 0;
#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                            \
        }                                                                       \
    } while (0)

static mm_config cfg2d()
{
    mm_config c;
    std::memset(&c, 0, sizeof c);
    c.dim = 2;
    c.nx = 16;
    c.ny = 12;
    c.nv1 = 16;
    c.nv2 = 16;
    c.x_hi = c.y_hi = 1.0;
    c.v1_lo = c.v2_lo = -8.0;
    c.v1_hi = c.v2_hi = 8.0;
    c.eps = 1e-2;
    c.cfl = 0.5;
    c.nu = -0.5;
    c.tau_model = MM_TAU_RHO;
    c.tau_coef = 1.0;
    for (int s = 0; s < 4; ++s) {
        c.bc[s].kind = MM_BC_WALL;
        c.bc[s].T_wall = 1.0;
    }
    return c;
}

static mm_config cfg1d()
{
    mm_config c = cfg2d();
    c.dim = 1;
    c.ny = c.nv2 = 1;
    c.bc[0].kind = c.bc[1].kind = MM_BC_PERIODIC;
    return c;
}

// a state at rest: rho = 1, u = 0, T = 1 (2D: Q = (rho, m1, m2, E11, E12, E22))
static std::vector<double> rest_state(const mm_config &c)
{
    const int n = c.nx * (c.dim == 2 ? c.ny : 1), k = c.dim == 2 ? 6 : 3;
    std::vector<double> q((size_t)n * k, 0.0);
    for (int i = 0; i < n; ++i) {
        q[(size_t)i * k] = 1.0;
        if (c.dim == 2) {
            q[(size_t)i * k + 3] = 1.0;
            q[(size_t)i * k + 5] = 1.0;
        } else {
            q[(size_t)i * k + 2] = 0.5;
        }
    }
    return q;
}

int main()
{
    // --- the time-step rule and the configuration checks
    for (const mm_config base : {cfg2d(), cfg1d()}) {
        int n = -1;
        const double dt = mm_dt(&base, 0.0, &n);
        CHECK(dt > 0.0 && n == 0);
        const double dt2 = mm_dt(&base, 0.37, &n);
        CHECK(dt2 > 0.0 && dt2 <= dt && n >= 1 && std::fabs(n * dt2 - 0.37) < 1e-12);
        CHECK(mm_dt(&base, 0.37, nullptr) == dt2);
        CHECK(mm_dt(&base, 1e300, &n) < 0.0);           // more steps than an int holds
        mm_config c = base;
        c.dt = 1e-3;
        CHECK(mm_dt(&c, 0.0, &n) == 1e-3);
        c = base;
        c.cfl_rule = MM_CFL_SUM;
        CHECK(mm_dt(&c, 0.0, &n) > 0.0);
        // every single-field violation is rejected
        const int nmut = 30;
        for (int m = 0; m < nmut; ++m) {
            c = base;
            switch (m) {
            case 0: c.dim = 3; break;
            case 1: c.nx = 1; break;
            case 2: c.nv1 = 0; break;
            case 3: c.x_hi = c.x_lo; break;
            case 4: c.v1_hi = c.v1_lo - 1.0; break;
            case 5: c.eps = 0.0; break;
            case 6: c.eps = INFINITY; break;
            case 7: c.eps = NAN; break;
            case 8: c.cfl = 0.0; break;
            case 9: c.tau_model = 7; break;
            case 10: c.tau_coef = -1.0; break;
            case 11: c.proj_mode = 5; break;
            case 12: c.precision = 9; break;
            case 13: c.bc[0].kind = 17; break;
            case 14: c.bc[0].kind = MM_BC_WALL; c.bc[0].T_wall = 0.0; break;
            case 15: c.bc[0].kind = MM_BC_PERIODIC; c.bc[1].kind = MM_BC_WALL; c.bc[1].T_wall = 1.0; break;
            case 16: c.nx = 2000000000; c.nv1 = 64; break;           // too many points
            case 17: c.dev_buffers[0] = &c; break;                   // partly set
            case 18: c.nv1 = -4; break;
            case 19: c.cfl = NAN; break;
            case 20: c.bc[1].kind = MM_BC_INFLOW; c.bc[1].rho = 0.0; break;
            // 2D only
            case 21: if (c.dim == 2) c.ny = 1; else c.precision = MM_MIXED; break;
            case 22: if (c.dim == 2) c.nu = 1.0; else c.bc[0].kind = c.bc[1].kind = MM_BC_INFLOW; break;
            case 23: if (c.dim == 2) c.nu = -1.5; else c.dev_buffers[0] = c.dev_buffers[1] = c.dev_buffers[2] = &c; break;
            case 24: if (c.dim == 2) { c.nx = 60000; c.ny = 60000; c.nv1 = c.nv2 = 2; } else c.nx = -3; break;
            case 25: if (c.dim == 2) c.dev_buffers[0] = c.dev_buffers[1] = c.dev_buffers[2] = &c; else c.eps = -1.0; break;
            case 26: c.x_hi = INFINITY; break;
            case 27: c.v1_lo = -INFINITY; break;
            case 28: c.cfl = INFINITY; break;
            case 29: c.dt = INFINITY; break;
            }
            if (!(mm_dt(&c, 0.0, &n) < 0.0)) {
                std::fprintf(stderr, "dim %d: mutation %d not rejected\n", base.dim, m);
                ++fails;
                continue;                 // the state below is sized for the base grid
            }
            mm_ctx *ctx = reinterpret_cast<mm_ctx *>(&c);  // a non-NULL stand-in: failure stores NULL
            std::vector<double> q = rest_state(base);
            CHECK(mm_init(&c, q.data(), nullptr, &ctx) == MM_EINVAL);
            CHECK(ctx == nullptr);
        }
    }
    CHECK(mm_dt(nullptr, 0.0, nullptr) < 0.0);

    // --- context creation: without a GPU it fails in the runtime and frees what it made
    for (const mm_config c : {cfg2d(), cfg1d()}) {
        std::vector<double> q = rest_state(c);
        mm_ctx *ctx = nullptr;
        CHECK(mm_init(&c, q.data(), nullptr, nullptr) == MM_EINVAL);
        CHECK(mm_init(&c, nullptr, nullptr, &ctx) == MM_EINVAL && ctx == nullptr);
        const int rc = mm_init(&c, q.data(), nullptr, &ctx);
        CHECK(rc == MM_OK || rc == MM_EDEVICE);
        if (rc == MM_OK) mm_free(ctx);
        else CHECK(ctx == nullptr);
    }

    // --- null handles and bad arguments
    double d[8];
    float f[8];
    int k = 0;
    long long ll = 0;
    void *p = nullptr;
    CHECK(mm_step(nullptr, 1) == MM_EINVAL);
    CHECK(mm_step_async(nullptr, 1) == MM_EINVAL);
    CHECK(mm_sync(nullptr) == MM_EINVAL);
    CHECK(mm_moments(nullptr, d, d, d) == MM_EINVAL);
    CHECK(mm_get_g(nullptr, d) == MM_EINVAL);
    CHECK(mm_get_g_cells(nullptr, &k, 1, d) == MM_EINVAL);
    CHECK(mm_set_state(nullptr, d, d) == MM_EINVAL);
    CHECK(mm_failed_step(nullptr) == -1);
    CHECK(mm_set_source(nullptr, 0, 0.0) == MM_EINVAL);
    CHECK(mm_timing(nullptr, 1) == MM_EINVAL);
    CHECK(mm_timing_get(nullptr, 0, &k, d) == MM_EINVAL);
    CHECK(mm_device_ptrs(nullptr, &p, &p, &p, &k) == MM_EINVAL);
    CHECK(mm_closure_attach(nullptr, nullptr, 0.05, 0) == MM_EINVAL);
    CHECK(mm_closure_cells(nullptr, &ll, nullptr) == MM_EINVAL);
    CHECK(mm_closure_snapshot(nullptr, 0.05, 0, f, f, 1, &k) == MM_EINVAL);
    CHECK(mm_closure_features(nullptr, f, f, nullptr) == MM_EINVAL);
    CHECK(mm_closure_rebuild(nullptr, f, nullptr) == MM_EINVAL);
    mm_free(nullptr);
    for (int s = -3; s <= 8; ++s) CHECK(mm_strerror(s) != nullptr && mm_strerror(s)[0] != 0);

    mm_mlp *net = nullptr;
    CHECK(mm_mlp_create(0, nullptr, 1, nullptr) == MM_EINVAL);
    const int rc = mm_mlp_create(-1, nullptr, 1, &net);
    CHECK(rc == MM_EDEVICE && net == nullptr);
    CHECK(mm_mlp_fit_norm(nullptr, f, f, 1) == MM_EINVAL);
    CHECK(mm_mlp_get(nullptr, f, f) == MM_EINVAL);
    CHECK(mm_mlp_set(nullptr, f, f) == MM_EINVAL);
    CHECK(mm_mlp_forward(nullptr, f, 1, f) == MM_EINVAL);
    CHECK(mm_mlp_grad(nullptr, f, f, 1, f, d) == MM_EINVAL);
    CHECK(mm_mlp_train(nullptr, f, f, 1, 1, 32, 1e-3, 1, d) == MM_EINVAL);
    mm_mlp_free(nullptr);

    // --- the allocation-free step: argument checks before any device work
    {
        mm_config c = cfg2d();
        int failed = 7;
        CHECK(mm_step2d_noalloc(nullptr, d, d, f, nullptr, 1, &failed) == MM_EINVAL && failed == -1);
        CHECK(mm_step2d_noalloc(&c, nullptr, d, f, nullptr, 1, &failed) == MM_EINVAL);
        CHECK(mm_step2d_noalloc(&c, d, d, d, nullptr, 1, &failed) == MM_EINVAL);     // the same G twice
        CHECK(mm_step2d_noalloc(&c, d, d, f, nullptr, -1, &failed) == MM_EINVAL);
        mm_config c1 = cfg1d();
        CHECK(mm_step2d_noalloc(&c1, d, d, f, nullptr, 1, &failed) == MM_EINVAL);
        c.precision = MM_CLOSURE;
        CHECK(mm_step2d_noalloc(&c, d, d, f, nullptr, 1, &failed) == MM_EINVAL);
        c = cfg2d();
        c.nx = c.ny = 4096;                                                       // beyond the static array
        CHECK(mm_step2d_noalloc(&c, d, d, f, nullptr, 1, &failed) == MM_EINVAL);
    }

    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("sanitized host run: all cases completed\n");
    return 0;
}
