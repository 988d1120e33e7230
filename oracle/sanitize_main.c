/*
 * sanitize_main.c -- TEST INFRASTRUCTURE: a driver that runs every entry point of
 * the oracle on small cases, built with -fsanitize=address,undefined (see
 * tests/test_sanitize.py) so that any out-of-bounds access, use after free, leak
 * or undefined operation in the oracle fails the build's run.  It includes
 * mm_oracle.c to use its configuration type; the closure oracle is linked beside.
 */
#include "mm_oracle.c"

#include <stdio.h>

int o_features2d(const void *cfgp, const double *Q, double *feat, double *kn, int *edge);
int o_mlp_nparam(void);
int o_mlp_forward(const double *params, const double *norm, const double *X, int n, int bf16, double *Y);
int o_mlp_grad(const double *params, const double *norm, const double *X, const double *Y, int n, int bf16,
               double *grad, double *loss);
void o_closure_H(const double *q, const double *t, double *H);
int o_closure_grec(const void *cfgp, const double *q, const double *qt, const double *St, const double *tt,
                   double *g);
void o_nsf_closure(const void *cfgp, const double *f, double *qt, double *St, double *tt);

static int fails = 0;
#define CHECK(x) do { if (!(x)) { fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); ++fails; } } while (0)

static o_cfg cfg2d(int nx, int ny, int nv, int kind_x, int kind_y)
{
    o_cfg c;
    memset(&c, 0, sizeof c);
    c.dim = 2; c.nx = nx; c.ny = ny; c.nv1 = nv; c.nv2 = nv;
    c.x_lo = 0.0; c.x_hi = 1.0; c.y_lo = 0.0; c.y_hi = 1.0;
    c.v1_lo = -7.0; c.v1_hi = 7.0; c.v2_lo = -7.0; c.v2_hi = 7.0;
    c.eps = 0.05; c.cfl = 0.5; c.cfl_rule = O_CFL_MIN; c.nu = -0.5;
    c.tau_model = O_TAU_RHO; c.tau_coef = 1.452823;
    for (int s = 0; s < 4; ++s) {
        c.bc[s].kind = s < 2 ? kind_x : kind_y;
        c.bc[s].T_wall = 1.0; c.bc[s].u_wall = s == 3 ? 0.2 : 0.0;
        c.bc[s].rho = 1.0; c.bc[s].u1 = 0.1; c.bc[s].u2 = 0.0; c.bc[s].T = 1.0;
    }
    c.proj_mode = O_PROJ_DISCRETE; c.wall_es_term = 1; c.dt = 0.0;
    return c;
}

static void state2d(const o_cfg *c, double *Q)
{
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
            const double x = (i + 0.5) / c->nx, y = (j + 0.5) / c->ny;
            const double rho = 1.0 + 0.2 * sin(6.0 * x + 1.0) * cos(5.0 * y), u1 = 0.1 * sin(4.0 * y), u2 = 0.1 * cos(3.0 * x);
            const double T = 1.0 + 0.1 * cos(7.0 * x * y);
            double *q = Q + 6 * (size_t)(j * c->nx + i);
            q[0] = rho; q[1] = rho * u1; q[2] = rho * u2;
            q[3] = rho * u1 * u1 + rho * T + 0.01; q[4] = rho * u1 * u2 + 0.005; q[5] = rho * u2 * u2 + rho * T - 0.01;
        }
}

static void run2d_case(int nx, int ny, int nv, int kx, int ky, int proj, int steps)
{
    o_cfg c = cfg2d(nx, ny, nv, kx, ky);
    c.proj_mode = proj;
    const size_t nc = (size_t)nx * ny, nn = nc * nv * nv;
    double *Q = malloc(sizeof(double) * 6 * nc), *G = calloc(nn, sizeof(double)), *H = calloc(4 * nc, sizeof(double));
    double *Gh = malloc(sizeof(double) * nn);
    state2d(&c, Q);
    int fs = 0;
    CHECK(o_run2d(&c, Q, G, steps, H, &fs) == O_OK);
    CHECK(o_micro2d(&c, Q, G, H) == O_OK);
    CHECK(o_macro2d(&c, Q, H) == O_OK);
    CHECK(o_ghat2d(&c, Q, Gh) == O_OK);
    double M[64 * 64], Gs[64 * 64], PF[64 * 64];
    CHECK(o_gaussians2d(&c, Q, M, Gs) == O_OK);
    CHECK(o_project2d(&c, Q, Gs, PF) == O_OK);
    free(Q); free(G); free(H); free(Gh);
}

static void run1d_case(int nx, int nv, int kind, int steps)
{
    o_cfg c;
    memset(&c, 0, sizeof c);
    c.dim = 1; c.nx = nx; c.ny = 1; c.nv1 = nv; c.nv2 = 1;
    c.x_lo = 0.0; c.x_hi = 1.0; c.y_hi = 1.0; c.v1_lo = -6.0; c.v1_hi = 6.0; c.v2_hi = 1.0;
    c.eps = 0.02; c.cfl = 0.9; c.tau_model = O_TAU_P; c.tau_coef = 1.0; c.proj_mode = O_PROJ_DISCRETE;
    c.bc[0].kind = kind; c.bc[1].kind = kind; c.bc[0].T_wall = 1.0; c.bc[1].T_wall = 1.2;
    double *Q = malloc(sizeof(double) * 3 * nx), *G = calloc((size_t)nx * nv, sizeof(double));
    double *H = calloc(nx, sizeof(double));
    for (int i = 0; i < nx; ++i) {
        const double x = (i + 0.5) / nx, rho = 1.0 + 0.3 * x, u = 0.1 * sin(3.0 * x), T = 1.0 + 0.2 * x;
        Q[3 * i] = rho; Q[3 * i + 1] = rho * u; Q[3 * i + 2] = 0.5 * rho * T + 0.5 * rho * u * u;
    }
    int fs = 0;
    CHECK(o_run1d(&c, Q, G, steps, H, &fs) == O_OK);
    free(Q); free(G); free(H);
}

int main(void)
{
    o_set_threads(2);
    /* 2D: walls with a lid, periodic, extrapolation, inflow; both projector modes */
    run2d_case(7, 6, 8, O_BC_WALL, O_BC_WALL, O_PROJ_DISCRETE, 4);
    run2d_case(6, 5, 12, O_BC_PERIODIC, O_BC_PERIODIC, O_PROJ_PAPER, 3);
    run2d_case(5, 7, 10, O_BC_EXTRAP, O_BC_INFLOW, O_PROJ_DISCRETE, 3);
    run2d_case(4, 4, 6, O_BC_INFLOW, O_BC_EXTRAP, O_PROJ_PAPER, 2);
    /* 1D: walls, periodic, extrapolation */
    run1d_case(9, 11, O_BC_WALL, 20);
    run1d_case(8, 12, O_BC_PERIODIC, 10);
    run1d_case(6, 10, O_BC_EXTRAP, 10);
    /* the manufactured-solution runs, stopped early, and their exact data */
    {
        o_cfg c = cfg2d(12, 12, 12, O_BC_PERIODIC, O_BC_PERIODIC);
        c.v1_lo = c.v2_lo = -6.0; c.v1_hi = c.v2_hi = 6.0; c.eps = 0.08; c.nu = -1.0; c.cfl = 0.35;
        double *Q = malloc(sizeof(double) * 6 * 144), *G = malloc(sizeof(double) * 144 * 144), e[2];
        CHECK(o_mms2d_exact(&c, 0.1, Q, G) == O_OK);
        { const int rc = o_mms2d_run(&c, 0.25, 3, Q, G, e); if (rc != O_OK) fprintf(stderr, "mms2d rc %d\n", rc); CHECK(rc == O_OK); }
        free(Q); free(G);
        o_cfg d;
        memset(&d, 0, sizeof d);
        d.dim = 1; d.nx = 8; d.nv1 = 8; d.x_hi = 1.0; d.v1_lo = -6.5; d.v1_hi = 6.5; d.eps = 0.1; d.cfl = 0.95;
        d.tau_model = O_TAU_HS1D; d.tau_coef = 3.2; d.bc[0].kind = d.bc[1].kind = O_BC_PERIODIC;
        double Q1[24], G1[64];
        CHECK(o_mms1d_exact(&d, 0.2, Q1, G1) == O_OK);
        CHECK(o_mms1d_run(&d, 0.9351, 5, Q1, G1, e) == O_OK);
        CHECK(o_mms1d(&d, 0.05, e) == O_OK);
    }
    /* closure pieces */
    {
        o_cfg c = cfg2d(5, 4, 8, O_BC_WALL, O_BC_PERIODIC);
        double Q[6 * 20], F[30 * 20], kn[20];
        int edge[20];
        state2d(&c, Q);
        CHECK(o_features2d(&c, Q, F, kn, edge) == 0);
        const int np = o_mlp_nparam();
        double *par = calloc(np, sizeof(double)), *gr = malloc(sizeof(double) * np), norm[74], Y[7 * 20], loss;
        for (int k = 0; k < np; ++k) par[k] = 0.01 * sin(0.37 * k);
        for (int k = 0; k < 74; ++k) norm[k] = (k >= 30 && k < 60) || k >= 67 ? 1.0 : 0.0;
        CHECK(o_mlp_forward(par, norm, F, 20, 1, Y) == 0);
        CHECK(o_mlp_grad(par, norm, F, Y, 20, 0, gr, &loss) == 0);
        double qt[2] = {0.1, -0.05}, St[3] = {0.02, 0.01, -0.02}, tt[2] = {0.03, -0.01}, Hc[4], g[64];
        o_closure_H(qt, tt, Hc);
        CHECK(o_closure_grec(&c, Q, qt, St, tt, g) == 0);
        o_nsf_closure(&c, F, qt, St, tt);
        free(par); free(gr);
    }
    /* scalar helpers */
    double q6[6] = {1.0, 0.1, -0.2, 1.2, 0.05, 0.9}, out[6], q3[3] = {1.0, 0.2, 0.7};
    o_kfvs_half2d(q6, 0, 1, out);
    o_kfvs_half2d(q6, 1, -1, out);
    o_kfvs_half1d(q3, 1, out);
    CHECK(o_trbdf2_W(0.01, 1.0, -0.5, 1e-3) <= 1.0);
    CHECK(o_wall_R(0.1, 1.0, 1.2, -1) > 0.0);
    if (fails) return 1;
    printf("sanitized oracle run: all cases completed\n");
    return 0;
}
