/*
 * mm_closure_oracle.c -- plain FP64 CPU reference of the learned-closure form
 * of the 2D2V micro-macro step (the closure itself is not in the paper; its
 * ingredients are):
 *   - per-cell features: the primitive state (rho, u1, u2, T, P11, P12, P22)
 *     of the macro vector of Sec. 5.1, its centred x / y differences, the
 *     local mean free path eps sqrt(T) / tau and the second x / y differences
 *     of (rho, u1, u2, T);
 *   - the local Knudsen indicator that decides where the closure may replace
 *     the micro solve;
 *   - a 30 -> 64 -> 64 -> 7 perceptron with exact (erf) GELU, its loss and its
 *     gradient by reverse accumulation;
 *   - the heat-flux tensor H of the closed macro system (eq5-41), four third
 *     moments in 2D, rebuilt from its two contractions (the heat-flux vector q,
 *     h = (H111 + H122, H112 + H222) / 2 of Sec. 6.3) and its two traceless
 *     combinations t = (H111 - 3 H122, 3 H112 - H222), zero in the isotropic
 *     (Grad) form;
 *   - the micro part rebuilt from (q, S, t) with the Hermite form that has
 *     exactly these moments under the Maxwellian, projected with the discrete
 *     projector;
 *   - the Navier-Stokes-Fourier values of (q, S) from the Chapman-Enskog
 *     expansion (eqn:NSF-sigma-q and the ES-BGK transport coefficients of
 *     Sec. 2.2), the closure the network is measured against.
 *
 * TEST INFRASTRUCTURE ONLY (like mm_oracle.c): nothing in the product path
 * links, loads or calls this file.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* these mirror the declarations in mm_oracle.c (same translation unit set, no
 * shared header with the GPU library) */
enum { C_BC_EXTRAP = 0, C_BC_PERIODIC = 1, C_BC_WALL = 2, C_BC_INFLOW = 3 };
enum { C_TAU_RHO = 0, C_TAU_P = 1, C_TAU_HS1D = 2, C_TAU_CONST = 3 };

typedef struct {
    int kind;
    double T_wall, u_wall, rho, u1, u2, T;
} c_bc;

typedef struct {
    int dim, nx, ny, nv1, nv2;
    double x_lo, x_hi, y_lo, y_hi, v1_lo, v1_hi, v2_lo, v2_hi;
    double eps, cfl;
    int cfl_rule;
    double nu;
    int tau_model;
    double tau_coef;
    c_bc bc[4];
    int proj_mode, wall_es_term;
    double dt;
} c_cfg;

/* from mm_oracle.c */
int o_project2d(const void *cfg, const double *q, const double *F, double *PF);

#define NF 30
#define NH 64
#define NO 7   /* (q1, q2, S11, S12, S22, t1, t2) / eps */
#define NPARAM (NH * NF + NH + NH * NH + NH + NO * NH + NO)

int o_mlp_nparam(void) { return NPARAM; }

static double tau_of(const c_cfg *c, double rho, double T)
{
    switch (c->tau_model) {
    case C_TAU_RHO: return c->tau_coef * rho;
    case C_TAU_P: return c->tau_coef * rho * T;
    case C_TAU_HS1D: return c->tau_coef * sqrt(T / (2.0 * 3.14159265358979323846));
    default: return c->tau_coef;
    }
}

/* primitive state of one cell: rho, u1, u2, T, P11, P12, P22 (Sec. 5.1:
 * E = rho u u^T + P, T = tr P / (2 rho)) */
static void prim_of(const double *q, double *w)
{
    const double rho = q[0], u1 = q[1] / rho, u2 = q[2] / rho;
    const double P11 = q[3] - rho * u1 * u1, P12 = q[4] - rho * u1 * u2, P22 = q[5] - rho * u2 * u2;
    w[0] = rho; w[1] = u1; w[2] = u2; w[3] = 0.5 * (P11 + P22) / rho;
    w[4] = P11; w[5] = P12; w[6] = P22;
}

/* centred difference along one axis; one-sided next to a side that is not
 * periodic; n == 1 gives zero */
static double diff1(const double *wm, const double *w0, const double *wp, int has_m, int has_p, double h, int a)
{
    if (has_m && has_p) return (wp[a] - wm[a]) / (2.0 * h);
    if (has_p) return (wp[a] - w0[a]) / h;
    if (has_m) return (w0[a] - wm[a]) / h;
    return 0.0;
}

/*
 * Features, indicator and the "always micro" mask of every cell.
 *   feat[c][0..6]   = (rho, u1, u2, T, P11, P12, P22)
 *   feat[c][7..13]  = d/dx of the same, feat[c][14..20] = d/dy
 *   feat[c][21]     = eps sqrt(T) / tau (the local mean free path)
 *   feat[c][22..25] = d2/dx2 of (rho, u1, u2, T), feat[c][26..29] = d2/dy2: the
 *                     central second difference, zero where a neighbour is
 *                     missing (next to a side that is not periodic)
 *   kn[c]  = (eps sqrt(T) / tau) max(|grad rho| / rho, |grad T| / T, |grad u|_F / sqrt(T))
 *   edge[c] = 1 for cells next to a side that is not periodic (their micro part
 *             is always solved), else 0.
 */
int o_features2d(const void *cfgp, const double *Q, double *feat, double *kn, int *edge)
{
    const c_cfg *c = (const c_cfg *)cfgp;
    const int nx = c->nx, ny = c->ny;
    const double dx = (c->x_hi - c->x_lo) / nx, dy = (c->y_hi - c->y_lo) / ny;
    const int px = c->bc[0].kind == C_BC_PERIODIC, py = c->bc[2].kind == C_BC_PERIODIC;
    double *W = malloc(sizeof(double) * 7 * (size_t)nx * ny);
    if (!W) return 2;
    for (int t = 0; t < nx * ny; ++t) prim_of(Q + 6 * (size_t)t, W + 7 * (size_t)t);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int cidx = j * nx + i;
            int im = i - 1, ip = i + 1, jm = j - 1, jp = j + 1;
            int hm = 1, hp = 1, vm = 1, vp = 1;
            if (im < 0) { if (px) im = nx - 1; else { hm = 0; im = i; } }
            if (ip >= nx) { if (px) ip = 0; else { hp = 0; ip = i; } }
            if (jm < 0) { if (py) jm = ny - 1; else { vm = 0; jm = j; } }
            if (jp >= ny) { if (py) jp = 0; else { vp = 0; jp = j; } }
            const double *w0 = W + 7 * (size_t)cidx;
            const double *wxm = W + 7 * (size_t)(j * nx + im), *wxp = W + 7 * (size_t)(j * nx + ip);
            const double *wym = W + 7 * (size_t)(jm * nx + i), *wyp = W + 7 * (size_t)(jp * nx + i);
            double *f = feat + NF * (size_t)cidx;
            for (int a = 0; a < 7; ++a) {
                f[a] = w0[a];
                f[7 + a] = diff1(wxm, w0, wxp, hm, hp, dx, a);
                f[14 + a] = diff1(wym, w0, wyp, vm, vp, dy, a);
            }
            const double rho = w0[0], T = w0[3];
            f[21] = c->eps * sqrt(T) / tau_of(c, rho, T);
            for (int a = 0; a < 4; ++a) {
                f[22 + a] = hm && hp ? (wxp[a] - 2.0 * w0[a] + wxm[a]) / (dx * dx) : 0.0;
                f[26 + a] = vm && vp ? (wyp[a] - 2.0 * w0[a] + wym[a]) / (dy * dy) : 0.0;
            }
            const double gr = sqrt(f[7] * f[7] + f[14] * f[14]) / rho;
            const double gT = sqrt(f[10] * f[10] + f[17] * f[17]) / T;
            const double gu = sqrt(f[8] * f[8] + f[15] * f[15] + f[9] * f[9] + f[16] * f[16]) / sqrt(T);
            double m = gr;
            if (gT > m) m = gT;
            if (gu > m) m = gu;
            kn[cidx] = f[21] * m;
            edge[cidx] = (!px && (i == 0 || i == nx - 1)) || (!py && (j == 0 || j == ny - 1));
        }
    free(W);
    return 0;
}

/* ---------------------------------------------------------------- the MLP */

/* GELU with the exact normal CDF, and its derivative */
double o_gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }
double o_gelu_d(double x)
{
    return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * exp(-0.5 * x * x) / sqrt(2.0 * 3.14159265358979323846);
}

/* nearest-even rounding of a double to bfloat16 (8 significand bits), kept as a
 * double: used to evaluate the network at the precision of its weights */
double o_bf16(double x)
{
    if (!isfinite(x) || x == 0.0) return x;
    int e;
    const double m = frexp(x, &e);               /* x = m 2^e, 0.5 <= |m| < 1 */
    const double s = ldexp(m, 8);                /* 8 significand bits */
    double r = nearbyint(s);                     /* default rounding: to nearest, ties to even */
    return ldexp(r, e - 8);
}

/* parameter block: W1[64][30], b1[64], W2[64][64], b2[64], W3[7][64], b3[7] */
typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3;
} mlp_view;

static mlp_view view(const double *p)
{
    mlp_view v;
    v.W1 = p; v.b1 = v.W1 + NH * NF; v.W2 = v.b1 + NH; v.b2 = v.W2 + NH * NH; v.W3 = v.b2 + NH; v.b3 = v.W3 + NO * NH;
    return v;
}

/* one sample: normalised input xh[30] -> pre-activations z1, z2, activations a1,
 * a2 and the normalised output yh[7].  With bf16 != 0 every matrix-product input
 * (xh, a1, a2) is rounded to bfloat16 first, as the GPU kernels feed them to the
 * matrix cores; sums and everything else stay FP64. */
static void forward1(const mlp_view *v, const double *xh_in, int bf16, double *z1, double *a1, double *z2, double *a2,
                     double *yh)
{
    double xh[NF], a1r[NH], a2r[NH];
    for (int k = 0; k < NF; ++k) xh[k] = bf16 ? o_bf16(xh_in[k]) : xh_in[k];
    for (int h = 0; h < NH; ++h) {
        double s = v->b1[h];
        for (int k = 0; k < NF; ++k) s += v->W1[h * NF + k] * xh[k];
        z1[h] = s;
        a1[h] = o_gelu(s);
        a1r[h] = bf16 ? o_bf16(a1[h]) : a1[h];
    }
    for (int h = 0; h < NH; ++h) {
        double s = v->b2[h];
        for (int k = 0; k < NH; ++k) s += v->W2[h * NH + k] * a1r[k];
        z2[h] = s;
        a2[h] = o_gelu(s);
        a2r[h] = bf16 ? o_bf16(a2[h]) : a2[h];
    }
    for (int o = 0; o < NO; ++o) {
        double s = v->b3[o];
        for (int k = 0; k < NH; ++k) s += v->W3[o * NH + k] * a2r[k];
        yh[o] = s;
    }
}

/*
 * Network outputs for n samples of raw features X[n][30]:
 *   xh = (x - in_mean) / in_std, yh = MLP(xh), y = yh * out_std + out_mean.
 * norm = [in_mean(30), in_std(30), out_mean(7), out_std(7)].
 */
int o_mlp_forward(const double *params, const double *norm, const double *X, int n, int bf16, double *Y)
{
    const mlp_view v = view(params);
    for (int s = 0; s < n; ++s) {
        double xh[NF], z1[NH], a1[NH], z2[NH], a2[NH], yh[NO];
        for (int k = 0; k < NF; ++k) xh[k] = (X[(size_t)s * NF + k] - norm[k]) / norm[NF + k];
        forward1(&v, xh, bf16, z1, a1, z2, a2, yh);
        for (int o = 0; o < NO; ++o) Y[(size_t)s * NO + o] = yh[o] * norm[2 * NF + NO + o] + norm[2 * NF + o];
    }
    return 0;
}

/*
 * Loss L = (1 / (5 n)) sum_s sum_o (yh_o - (y_o - out_mean_o) / out_std_o)^2 of
 * n samples and its gradient with respect to every parameter (same layout as
 * params), by reverse accumulation through the three layers.  With bf16 != 0
 * the forward rounds as o_mlp_forward does, and every matrix-product input of
 * the backward pass (the output error, the back-propagated errors, the weights
 * already are) is rounded to bfloat16 as well.
 */
int o_mlp_grad(const double *params, const double *norm, const double *X, const double *Y, int n, int bf16,
               double *grad, double *loss)
{
    const mlp_view v = view(params);
    memset(grad, 0, sizeof(double) * NPARAM);
    double *gW1 = grad, *gb1 = gW1 + NH * NF, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH, *gW3 = gb2 + NH,
           *gb3 = gW3 + NO * NH;
    double L = 0.0;
    const double scale = 1.0 / (double)(NO * n);
    for (int s = 0; s < n; ++s) {
        double xh[NF], z1[NH], a1[NH], z2[NH], a2[NH], yh[NO];
        for (int k = 0; k < NF; ++k) xh[k] = (X[(size_t)s * NF + k] - norm[k]) / norm[NF + k];
        forward1(&v, xh, bf16, z1, a1, z2, a2, yh);
        double dy[NO];
        for (int o = 0; o < NO; ++o) {
            const double t = (Y[(size_t)s * NO + o] - norm[2 * NF + o]) / norm[2 * NF + NO + o];
            const double r = yh[o] - t;
            L += r * r;
            dy[o] = 2.0 * r * scale;
            if (bf16) dy[o] = o_bf16(dy[o]);
        }
        /* layer 3 */
        double da2[NH], dz2[NH], da1[NH], dz1[NH];
        for (int o = 0; o < NO; ++o) {
            gb3[o] += dy[o];
            for (int k = 0; k < NH; ++k) gW3[o * NH + k] += dy[o] * (bf16 ? o_bf16(a2[k]) : a2[k]);
        }
        for (int k = 0; k < NH; ++k) {
            double sacc = 0.0;
            for (int o = 0; o < NO; ++o) sacc += v.W3[o * NH + k] * dy[o];
            da2[k] = sacc;
            dz2[k] = sacc * o_gelu_d(z2[k]);
            if (bf16) dz2[k] = o_bf16(dz2[k]);
        }
        /* layer 2 */
        for (int h = 0; h < NH; ++h) {
            gb2[h] += dz2[h];
            for (int k = 0; k < NH; ++k) gW2[h * NH + k] += dz2[h] * (bf16 ? o_bf16(a1[k]) : a1[k]);
        }
        for (int k = 0; k < NH; ++k) {
            double sacc = 0.0;
            for (int h = 0; h < NH; ++h) sacc += v.W2[h * NH + k] * dz2[h];
            da1[k] = sacc;
            dz1[k] = sacc * o_gelu_d(z1[k]);
            if (bf16) dz1[k] = o_bf16(dz1[k]);
        }
        /* layer 1 */
        for (int h = 0; h < NH; ++h) {
            gb1[h] += dz1[h];
            for (int k = 0; k < NF; ++k) gW1[h * NF + k] += dz1[h] * (bf16 ? o_bf16(xh[k]) : xh[k]);
        }
    }
    *loss = L * scale;
    return 0;
}

/* ---------------------------------------------- closure moments and g */

/* H (H111, H112, H122, H222) from its contractions q (the heat-flux vector,
 * q_a = (H_a11 + H_a22) / 2) and its traceless part t = (H111 - 3 H122,
 * 3 H112 - H222): the isotropic form H_abc = (q_a d_bc + q_b d_ac + q_c d_ab) / 2
 * (2D: the contraction over b = c gives (d_v + 2) / 2 q_a = 2 q_a, i.e. h = q)
 * has t = 0, and t adds (t1 / 4)(1, 0, -1, 0) + (t2 / 4)(0, 1, 0, -1), which has
 * zero contractions.  t may be NULL (t = 0). */
void o_closure_H(const double *q, const double *t, double *H)
{
    const double t1 = t ? t[0] : 0.0, t2 = t ? t[1] : 0.0;
    H[0] = 1.5 * q[0] + 0.25 * t1;
    H[1] = 0.5 * q[1] + 0.25 * t2;
    H[2] = 0.5 * q[0] - 0.25 * t1;
    H[3] = 1.5 * q[1] - 0.25 * t2;
}

/*
 * Micro part of one cell rebuilt from the closure moments: qt = q / eps (2) and
 * St = (S11, S12, S22) / eps with S the stress deviation eps dv sum (w w^T) g.
 * With p = rho T and the traceless part S' of St,
 *   g = M / (2 p T) [ S' : (w w^T) + (qt . w) (|w|^2 / (2T) - 2) ]
 *       + M / (24 p T^2) [ tt1 (w1^3 - 3 w1 w2^2) + tt2 (3 w1^2 w2 - w2^3) ]
 * has, under the Maxwellian M of the cell, zero (1, v, |v|^2) moments, stress
 * deviation eps S', heat flux eps qt and traceless third moments eps tt (the
 * cubic harmonics have zero moments of order below three and zero contractions;
 * under M, int (w1^3 - 3 w1 w2^2) w1^3 M = 6 rho T^3 and
 * int (w1^3 - 3 w1 w2^2) w1 w2^2 M = -6 rho T^3, so tt1 = 24 rho T^3 / (24 p T^2) tt1);
 * on the velocity grid it is then projected with the discrete projector, so its
 * discrete conserved moments vanish to round-off.  q is the cell's conserved
 * state (6); tt may be NULL (tt = 0).
 */
int o_closure_grec(const void *cfgp, const double *q, const double *qt, const double *St, const double *tt,
                   double *g)
{
    const c_cfg *c = (const c_cfg *)cfgp;
    const int nv1 = c->nv1, nv2 = c->nv2;
    const double dv1 = (c->v1_hi - c->v1_lo) / nv1, dv2 = (c->v2_hi - c->v2_lo) / nv2;
    double w[7];
    prim_of(q, w);
    const double rho = w[0], u1 = w[1], u2 = w[2], T = w[3], p = rho * T;
    const double tr = 0.5 * (St[0] + St[2]);
    const double a11 = St[0] - tr, a12 = St[1], a22 = St[2] - tr;
    double *raw = malloc(sizeof(double) * (size_t)nv1 * nv2);
    if (!raw) return 2;
    for (int l = 0; l < nv2; ++l)
        for (int k = 0; k < nv1; ++k) {
            const double w1 = c->v1_lo + (k + 0.5) * dv1 - u1, w2 = c->v2_lo + (l + 0.5) * dv2 - u2;
            const double ww = w1 * w1 + w2 * w2;
            const double M = rho / (2.0 * 3.14159265358979323846 * T) * exp(-ww / (2.0 * T));
            const double herm = a11 * w1 * w1 + 2.0 * a12 * w1 * w2 + a22 * w2 * w2 +
                                (qt[0] * w1 + qt[1] * w2) * (ww / (2.0 * T) - 2.0);
            const double cub = tt ? tt[0] * (w1 * w1 * w1 - 3.0 * w1 * w2 * w2) +
                                        tt[1] * (3.0 * w1 * w1 * w2 - w2 * w2 * w2)
                                  : 0.0;
            raw[l * nv1 + k] = M / (2.0 * p * T) * herm + M / (24.0 * p * T * T) * cub;
        }
    /* g = (I - Pi) raw with the projector of the configured mode */
    double *pr = malloc(sizeof(double) * (size_t)nv1 * nv2);
    if (!pr) { free(raw); return 2; }
    const int rc = o_project2d(cfgp, q, raw, pr);
    for (int t = 0; t < nv1 * nv2; ++t) g[t] = raw[t] - pr[t];
    free(raw);
    free(pr);
    return rc;
}

/*
 * Navier-Stokes-Fourier closure values of one cell from its features (the
 * layout of o_features2d), divided by eps:
 *   qt = -(2 p / tau) grad T                    (kappa = (d_v + 2) p / (2 tau))
 *   St = -(p / tau) sigma + nu (P - p I) / eps   (the stress of the first-order
 * micro part G-hat: its B : sigma term, plus the ES term (G - M) / eps)
 * with sigma = grad u + grad u^T - (div u) I.  Returns qt[2], St[3] and the
 * traceless third moments tt[2], which are zero to first order (the cubic
 * harmonics are orthogonal to the first-order micro part), if tt is not NULL.
 */
void o_nsf_closure(const void *cfgp, const double *f, double *qt, double *St, double *tt)
{
    const c_cfg *c = (const c_cfg *)cfgp;
    const double rho = f[0], T = f[3], p = rho * T, tau = tau_of(c, rho, T);
    qt[0] = -2.0 * p / tau * f[10];
    qt[1] = -2.0 * p / tau * f[17];
    const double u1x = f[8], u1y = f[15], u2x = f[9], u2y = f[16];
    const double s11 = u1x - u2y, s12 = u1y + u2x;
    St[0] = -(p / tau) * s11 + c->nu * (f[4] - p) / c->eps;
    St[1] = -(p / tau) * s12 + c->nu * f[5] / c->eps;
    St[2] = (p / tau) * s11 + c->nu * (f[6] - p) / c->eps;
    if (tt) tt[0] = tt[1] = 0.0;
}
